/*
 * gsdp.h -- C ABI of the Gaussian-parameter hot path of GS-Scale-style 3D
 * Gaussian Splatting training (arXiv 2509.15645), for AMD MI355X (gfx950).
 *
 * One training step t (1-based Adam step) is:
 *   gs_cull               frustum/screen cull of every Gaussian's current geometry
 *                         + ordered compaction into valid_ids            (Sec. 4.1, 4.2.1)
 *   gs_gather             current (restored) parameters of valid_ids, read-only
 *                         on the stored state                            (Sec. 4.3.3)
 *   [caller's renderer forward/backward -> compact gradients]
 *   gs_scatter_grad       compact -> dense gradient rows (optional)      (Sec. 4.1 step 4)
 *   gs_adam_step_deferred deferred Adam on update_ids = valid_ids U saturated rows
 *                                                           (Sec. 4.3, Eq. 2-3)
 *   gs_adam_flush         catch up every skipped step (checkpoint, eval, densify)
 *
 * Conventions shared by every entry point
 *   - Pointers inside gs_model and all array arguments are DEVICE pointers owned
 *     by the caller; the library never allocates memory the caller can see.
 *     `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous on `stream`, perform no host synchronisation and read
 *     counts from device memory, so a step can be captured in a hipGraph.
 *   - Return value: GS_OK (0) or a negative gs_status; nothing is launched
 *     when an argument check fails.
 *   - Row-major layouts.  Geometric group G: 10 FP32 columns per Gaussian
 *     (mean xyz, log-scale xyz, quaternion wxyz).  Appearance group A: `dim`
 *     columns (49 = opacity + 48 SH coefficients in 3DGS).  Each of w, m, v
 *     has its own row stride (in elements) so interleaved or padded layouts
 *     are allowed; G.w must be dense (stride 10) and 16-byte aligned.
 *   - Step semantics: gs_cull(t) and gs_gather(t) see the parameters before
 *     update t; gs_adam_step_deferred(t) applies update t; gs_adam_flush(t)
 *     makes every row current as of after update t.  Successive updates of
 *     one model use t = 1, 2, 3, ...
 *   - last_step[i] is the last update step applied to Gaussian i (0 = never);
 *     its defer count at step t is d = t - 1 - last_step[i] (the paper's
 *     per-Gaussian counter).  Initialise it to 0 with m = v = 0.
 */
#ifndef GSDP_H
#define GSDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
    GS_OK = 0,
    GS_EINVAL = -1,        /* bad argument: null pointer, size, stride, alignment, step */
    GS_EHIP = -2,          /* a HIP runtime call or launch failed (text: gs_last_hip_error) */
    GS_EUNSUPPORTED = -3,  /* a mode/dtype combination that is not implemented */
    GS_ESPACE = -4         /* workspace or LUT buffer too small for this call */
} gs_status;

typedef enum gs_dtype { GS_F32 = 0, GS_BF16 = 1, GS_FP8E4M3 = 2 } gs_dtype;

/* Pinhole training camera.  p_cam = R p_world + t; OpenCV axes (x right,
 * y down, z forward); pixel u = fx x/z + cx, v = fy y/z + cy. */
typedef struct gs_camera {
    float R[9];            /* world -> camera rotation, row-major */
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float near_plane, far_plane;
} gs_camera;

/* One parameter group (G or A) with its Adam moments. */
typedef struct gs_group {
    float *w;              /* [n][w_ld] parameters (FP32) */
    void *m;               /* [n][m_ld] first moment, element type `state` */
    void *v;               /* [n][v_ld] second moment */
    int32_t dim;           /* columns: 10 for G, 1..54 for A */
    int32_t w_ld, m_ld, v_ld;
    int32_t state;         /* gs_dtype of m and v: GS_F32, GS_BF16 (stochastic rounding) or
                              GS_FP8E4M3 (E4M3 codes, sqrt(v) stored, one FP32 power-of-two
                              scale per 128 rows, stochastic rounding) */
    int32_t pad_;
    float *m_scale;        /* FP8 only: [ceil(n/128)] block scales of m, zero-initialised */
    float *v_scale;        /* FP8 only: [ceil(n/128)] block scales of sqrt(v), zero-initialised */
    float lr[64];          /* learning rate of each column (dim entries used) */
} gs_group;

/* The optimisation problem: n Gaussians, both groups, the per-row step
 * counter and the Adam constants. */
typedef struct gs_model {
    int64_t n;
    gs_group geo;
    gs_group app;
    int32_t *last_step;    /* [n] */
    void *lut;             /* device tables from gs_lut_build (or its variants); every
                              gs_adam_step_deferred moves their restore rows to the next
                              step, and calls record step mismatches in their header */
    int32_t lut_max_steps; /* largest update step the tables cover */
    int32_t max_defer;     /* 0 = unbounded; K > 0: a row deferred K steps is force-updated
                              (the paper's saturating counter, MAX = 15) */
    double beta1, beta2, eps;
    int32_t cull_mode;     /* 0 = exact restoring cull, 1 = band cull (exact result,
                              restores only rows near a decision boundary) */
    int32_t geo_mode;      /* 0 = geometry deferred like the rest (default); 1 = geometric
                              columns updated by dense Adam on every row every step, the
                              split of Sec. 4.2.2 step 4 (appearance stays deferred) */
    uint64_t sr_seed;      /* seed of the stochastic-rounding stream of quantised moments */
    const int32_t *step_dev; /* device step counter used by calls with step == 0 */
    int32_t optimizer;     /* GS_OPT_ADAM (default), GS_OPT_ADAMW or GS_OPT_SGD_MOMENTUM */
    int32_t reserved_;
    float *cull_sum;       /* optional device [n][4], 16-byte aligned: the cull summary of each
                              row (see gs_cull_summary_build), or NULL */
    float *cull_chunk;     /* optional device [ceil(n / GS_CHUNK_ROWS)][8], 32-byte aligned:
                              bounds of the summaries of each chunk of rows (see
                              gs_cull_summary_build), or NULL; needs cull_sum */
} gs_model;

/* Optimizers.  GS_OPT_SGD_MOMENTUM is the momentum-optimizer extension the
 * paper names in Sec. 4.3: buf = beta1 buf + g, w -= lr buf (no dampening, no
 * Nesterov; beta1 is the momentum, beta2/eps and the v buffers are unused).
 * With zero gradients the buffer decays geometrically, so the deferred
 * catch-up is exact.  It needs tables from gs_lut_build_sgd_momentum, FP32 or
 * BF16 state, cull_mode 0 and geo_mode 0, and is not available in the batched
 * form. */
enum { GS_OPT_ADAM = 0, GS_OPT_ADAMW = 1, GS_OPT_SGD_MOMENTUM = 2 };

/* GS_OPT_ADAMW is Adam with decoupled weight decay (the other optimizer of
 * Sec. 4.3): each update first scales w by 1 - lr lambda (lr the column's
 * rate times the step's multiplier), then applies the Adam update.  Skipped
 * updates are caught up exactly like Eq. 3 with every deferred term also
 * shrunk by the later decays; the tables (gs_lut_build_adamw) hold one set
 * per distinct column rate, at most 8 distinct rates.  FP32 or BF16 state,
 * cull_mode 0, geo_mode 0; not available in the batched form. */

/* ---------------------------------------------------------------- tables */

/* Tables of the deferred update (Sec. 4.3.2 and its pseudocode, Eq. 2-3).
 * The paper precomputes, for the current step, the restore coefficient w_scale
 * of Eq. 3 for every defer count, and m_scale = b1^(d+1), v_scale = b2^(d+1) of
 * Eq. 2.  Here the tables hold the restore coefficients of two steps only (two
 * row slots, slot = step & 1) and each gs_adam_step_deferred(t) ends by
 * computing the rows of step t + 1 from those of t on the device: a row
 * deferred d steps at t is deferred d + 1 at t + 1 and has also skipped step
 * t, so W_{t+1}[d+1] = W_t[d] + (b1/sqrt(b2))^d c(t), with c(k) the unit-rate
 * bias-corrected step of Eq. 3, in FP64 (each entry rounded once to FP32).
 * Memory is O(max_steps + max_defer): with D = max_defer, or max_steps when
 * max_defer = 0, about 40 D + 16 max_steps bytes (a 30000-step run with
 * unbounded deferral needs 1.7 MB).  Byte layout (8-byte aligned):
 *   header (64 B: int32 t_row[2] = step held by each slot, T, K, nclass,
 *           error, kind, reserved)
 *   Wf [2][D+1] f32 | Mf [D+1] f32 | Vf [D+1] f32 | SS [T+2] f32 | BC [T+2] f32
 *   | pad to 8 | Wd [2][D+1] f64 | R [D+1] f64 | Cn [T+2] f64
 *   | per AdamW decay class: Wlf [2][D+1] f32, Pf [2][D+1] f32, qf [T+2] f32,
 *     pad to 8, Wld [2][D+1] f64, Pd [2][D+1] f64, qd [T+2] f64
 * A call of step t (cull, gather, update; the flush of t reads the rows of
 * t + 1) whose row slot does not hold that step -- steps must run 1, 2, 3 ...
 * -- or whose step lies outside [1, T] sets the header's error word (bit 0:
 * wrong step, bit 1: out of range); the update and the flush then store
 * nothing.  One table buffer serves one model. */
int gs_lut_bytes(int32_t max_steps, int32_t max_defer, size_t *bytes);

/* Compute the tables of step 1 on the host in FP64 (powers by repeated
 * multiplication, unit learning rate), round them once to FP32 and copy them
 * to `lut_dev` (a device buffer of at least gs_lut_bytes bytes, 8-byte
 * aligned).  Synchronous: returns after the copy completed. */
int gs_lut_build(double beta1, double beta2, int32_t max_steps, int32_t max_defer,
                 void *lut_dev, size_t bytes);

/* Move the tables of `model` forward to `step` (>= the step they hold, <=
 * lut_max_steps + 1), doing each step's advance in turn on `stream`, so that
 * a model can start (or resume) at any step.  Synchronises `stream` before
 * and after (setup only). */
int gs_lut_seek(const gs_model *model, int64_t step, void *stream);

/* The same on a host image of the tables (from the *_host builders): the
 * same FP64 operations as the device advance, so the rows agree bit for bit. */
int gs_lut_seek_host(void *lut_host, size_t bytes, int64_t step);

/* Tables of deferred SGD with momentum (same layout and size as the Adam
 * tables): W_t[d] = sum_{i=1..d} s[t-i] mu^(d+1-i), advanced as
 * W_{t+1}[d+1] = W_t[d] + mu^(d+1) s[t]; the first-moment table holds
 * mu^(d+1), the step table s[t] (lr_scale may be NULL: s = 1), the others 1.
 * FP64, rounded once. */
int gs_lut_build_sgd_momentum(double momentum, int32_t max_steps, int32_t max_defer, const double *lr_scale,
                              void *lut_dev, size_t bytes);
int gs_lut_build_sgd_momentum_host(double momentum, int32_t max_steps, int32_t max_defer, const double *lr_scale,
                                   void *lut_host, size_t bytes);

/* AdamW tables for `model` (its betas, column rates, lut_max_steps and
 * max_defer) with weight decay lambda >= 0 and an optional rate schedule
 * (as gs_lut_build_schedule).  The Adam tables come first, then per decay
 * class c -- the distinct column rates in order of first appearance, G columns
 * before A columns -- the decayed restore rows Wl, the decay products P (both
 * two slots like W) and the step decays q[t] = 1 - lr s[t] lambda; advanced as
 * Wl_{t+1}[d+1] = q[t] Wl_t[d] + r^d c(t), P_{t+1}[d+1] = q[t] P_t[d].
 * gs_lut_bytes_adamw gives the size; model->lut is not read. */
int gs_lut_bytes_adamw(const gs_model *model, size_t *bytes);
int gs_lut_build_adamw(const gs_model *model, double weight_decay, const double *lr_scale, void *lut_dev,
                       size_t bytes);
int gs_lut_build_adamw_host(const gs_model *model, double weight_decay, const double *lr_scale, void *lut_host,
                            size_t bytes);

/* Same tables written to host memory (for inspection and tests). */
int gs_lut_build_host(double beta1, double beta2, int32_t max_steps, int32_t max_defer,
                      void *lut_host, size_t bytes);

/* Tables for a learning-rate schedule: at update t every column's rate is
 * lr * lr_scale[t] (lr_scale: host array of max_steps + 2 finite values >= 0,
 * index t).  The pseudocode's LUT term (lr b1)/(...) of the skipped step k
 * then carries that step's rate, lr_scale[k] c(k), and the step size is
 * lr_scale[t] / (1 - b1^t).  A constant 1 gives gs_lut_build's tables. */
int gs_lut_build_schedule(double beta1, double beta2, int32_t max_steps, int32_t max_defer,
                          const double *lr_scale, void *lut_dev, size_t bytes);
int gs_lut_build_schedule_host(double beta1, double beta2, int32_t max_steps, int32_t max_defer,
                               const double *lr_scale, void *lut_host, size_t bytes);

/* ------------------------------------------------------------- workspace */

/* Bytes of the scratch workspace that gs_cull and gs_adam_step_deferred
 * share for one model: per-tile keep ballots, counts and prefixes of the
 * compaction, the list of saturated rows and diagnostic counters (about 0.2
 * bytes per Gaussian, plus 4.1 with max_defer > 0).  Zero-fill it once so the
 * diagnostic counters start at zero; the caller must not write it afterwards.
 * One workspace serves one model and one stream at a time. */
int gs_workspace_bytes(const gs_model *model, size_t *bytes);

/* ------------------------------------------------------------------ path */

/* Cull (Sec. 2.4 step 1 and Sec. 3.4: drop Gaussians outside the near/far
 * planes and those whose projected 3-sigma footprint misses the image, from
 * mean, scale and quaternion only) of every Gaussian's CURRENT geometry before
 * update `step` -- stored G restored with Eq. 3 for deferred rows -- against
 * `cam`, then ordered compaction: ids[0..M) = visible Gaussian ids ascending
 * (valid_ids, Sec. 4.1).  *count_dev = M (device).  If M > capacity only the
 * first `capacity` ids are written and *count_dev still holds M.  With
 * max_defer > 0 the saturated invisible rows are listed in the workspace for
 * gs_adam_step_deferred.  Deterministic: same inputs, same bits. */
int gs_cull(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids,
            uint32_t *count_dev, uint32_t capacity, void *ws, size_t ws_bytes, void *stream);

/* gs_cull for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * cull and ordered compaction, same ids and count, with the workspace taken
 * from an array of GS_CULL_NOALLOC_MAX_WS bytes that the library keeps in the
 * memory of each GPU it runs on until the process ends, instead of `ws`.
 * Calls no allocating routine.
 *   - Limit: the model's workspace (gs_workspace_bytes with max_defer = 0)
 *     must fit the array, about 95M Gaussians; larger models get GS_ESPACE
 *     (text in gs_last_hip_error).
 *   - max_defer > 0 and geo_mode = 1 return GS_EUNSUPPORTED: the update that
 *     follows those culls reads the cull's workspace, which the caller cannot
 *     reach here.
 *   - Every call on one GPU uses that GPU's one array: calls that overlap in
 *     time on one GPU (two streams, two host threads) race and give wrong
 *     ids.  Serialise them.  The workspace header's diagnostic counters are
 *     shared by all models culled this way. */
#define GS_CULL_NOALLOC_MAX_WS ((size_t)16 << 20)
int gs_cull_noalloc(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids,
                    uint32_t *count_dev, uint32_t capacity, void *stream);

/* Cull summaries (a data layout of this library, not of the paper).  When
 * model->cull_sum is set, the band cull (cull_mode 1, Adam) reads per row a
 * 16-byte summary instead of the 40-byte geometry row and the 4-byte last
 * step (with lut_max_steps > 65536 it also reads the last step), and loads
 * the row only where its conservative classification cannot decide; the
 * visible list is the same as without summaries.  cull_sum[i] = (x, y, z, w):
 * the centre of row i, and w: bits 31..17 are those of the FP32 value s =
 * (largest of the three log-scales) + 1e-6 (largest of their magnitudes)
 * rounded toward +infinity to 7 significand bits, bit 16 is set when the
 * quaternion's squared norm (evaluated in FP32) is at least 0.64, and the
 * high 16 bits are 0x7fc0 (a NaN) instead when a geometric value is not
 * finite or s >= 80; the low 16 bits of w are last_step[i] modulo 2^16.
 * Every call of this library that stores geometry or last steps
 * (gs_adam_step_deferred, gs_adam_flush, gs_densify_apply into dst) also
 * stores the summaries of the rows it writes; after geometry or last steps
 * are written any other way (initialisation, loading, a caller's own
 * kernels), call this to recompute all n summaries from model->geo.w and
 * model->last_step.  Not available with geo_mode 1 (GS_EUNSUPPORTED from
 * every call).  GS_EINVAL when cull_sum is NULL. */
int gs_cull_summary_build(const gs_model *model, void *stream);

/* Chunk bounds of the summaries (a data layout of this library, not of the
 * paper).  Rows i with i / GS_CHUNK_ROWS = c form chunk c.  When
 * model->cull_chunk is also set, record c = cull_chunk[8c .. 8c+8) holds
 * (lo_x, lo_y, lo_z, s_c, hi_x, hi_y, hi_z, 0): every summary centre of the
 * chunk lies in the box [lo, hi], and every summary s of the chunk (w &
 * 0xfffe0000 as an FP32 value) is at most s_c; s_c is a NaN when some row's
 * summary is.  With max_defer = 0 the summary cull first tests a chunk's box,
 * widened by the largest drift and footprint any of its rows can have at
 * this step, against the camera, and skips the chunk's rows when the test
 * shows that every one of them is culled (same visible list).  With rows in
 * a spatial order (for instance sorted by the Morton code of their centre)
 * most chunks of a camera that sees a small part of the scene are skipped.
 * The calls that store summaries widen the records of the rows they write
 * (records only grow); gs_cull_summary_build also recomputes every record
 * tightly from the summaries. */
#define GS_CHUNK_ROWS 1024

/* The summary cull's chunk decisions for a camera (a diagnostic): flags[c] =
 * 1 when gs_cull(model, cam, step, ...) skips chunk c (its record shows
 * every row culled), else 0, for c < ceil(n / GS_CHUNK_ROWS); flags is
 * device memory.  GS_EUNSUPPORTED unless the summary cull runs with chunk
 * records: cull_mode = 1, eps > 0, Adam, geo_mode = 0, max_defer = 0,
 * cull_sum and cull_chunk set. */
int gs_cull_chunk_flags(const gs_model *model, const gs_camera *cam, int64_t step, uint8_t *flags, void *stream);

/* gs_cull with the camera taken from device memory: record (t - 1) % n_cams
 * of `cams` (n_cams records from gs_camera_pack, uploaded by the caller,
 * 16-byte aligned), t the update step (step, or with step == 0 the model's
 * device step counter).  So a whole training step, its camera included, can
 * be captured once in a hipGraph and replayed.  Same outputs as gs_cull with
 * that camera.  Only the band cull from cull summaries reads its camera this
 * way: GS_EUNSUPPORTED unless cull_mode = 1, eps > 0, Adam, geo_mode = 0 and
 * cull_sum is set. */
int gs_cull_table(const gs_model *model, const void *cams, int32_t n_cams, int64_t step, uint32_t *ids,
                  uint32_t *count_dev, uint32_t capacity, void *ws, size_t ws_bytes, void *stream);

/* Gather: out_geo[i][0..10) and out_app[i][0..dim) = current values of row
 * ids[i] before update `step`, for i < min(*count_dev, capacity).  Deferred
 * rows are restored with the w_scale LUT and their stored moments (Eq. 3);
 * nothing in the model is written (read-only forwarding, Sec. 4.3.3).
 * out_geo / out_app are dense [capacity][10] / [capacity][dim]; either may
 * be NULL to skip that group.  Ids >= model->n are skipped. */
int gs_gather(const gs_model *model, int64_t step, const uint32_t *ids, const uint32_t *count_dev,
              uint32_t capacity, float *out_geo, float *out_app, void *stream);

/* Scatter compact gradient rows into dense rows: g_dense[ids[i]][:] =
 * g_compact[i][:] (accumulate != 0: +=) for i < min(*count_dev, capacity).
 * ids must be unique (they are, from gs_cull), so no atomics are used.  Used
 * to sum the gradients of split images before one update (Sec. 4.4). */
int gs_scatter_grad(const uint32_t *ids, const uint32_t *count_dev, uint32_t capacity, int32_t dim,
                    const float *g_compact, float *g_dense, int32_t accumulate, void *stream);

/* Deferred Adam update `step` (Sec. 4.3.2 and its pseudocode) on update_ids = the
 * visible rows ids[0..min(M,capacity)) plus, when max_defer > 0, the
 * saturated rows the preceding gs_cull listed in `ws`.  Per row with defer
 * count d and per column: restore w with the stored (old) moments (Eq. 3),
 * m = b1^(d+1) m + (1-b1) g, v = b2^(d+1) v + (1-b2) g^2 (Eq. 2), then the
 * standard Adam step with the new moments; last_step = step.
 * Gradients: compact g_geo [capacity][10] / g_app [capacity][dim] aligned
 * with ids (the scatter is fused), or, when g_geo/g_app are NULL, dense rows
 * g_geo_dense[id] / g_app_dense[id] that are read and then cleared to zero.
 * Saturated rows use g = 0.  The ids must be distinct (gs_cull's are); ids
 * >= model->n are skipped. */
/* (With geo_mode = 1 and compact gradients, the call must follow the gs_cull
 * of the same step on the same workspace: the dense geometric update finds
 * each visible row's compact gradient from the cull's keep ballots.) */
int gs_adam_step_deferred(const gs_model *model, int64_t step, const uint32_t *ids,
                          const uint32_t *count_dev, uint32_t capacity, const float *g_geo,
                          const float *g_app, float *g_geo_dense, float *g_app_dense, void *ws,
                          size_t ws_bytes, void *stream);

/* Graph replay: every entry point that takes `step` also accepts step == 0,
 * meaning "read the step from *model->step_dev when the kernels run" (clamped
 * to [1, lut_max_steps]), so a captured step can be replayed.  This call adds
 * one to *step_dev on `stream`. */
int gs_step_advance(int32_t *step_dev, void *stream);

/* Flush after update `step`: every row with last_step < step skipped
 * delta = step - last_step zero-gradient steps; bring it current (w restored
 * with the LUT of step+1 at delta, m *= b1^delta, v *= b2^delta, Eq. 2-3) and
 * set last_step = step.  Required before saving, evaluating or densifying. */
int gs_adam_flush(const gs_model *model, int64_t step, void *stream);

/* ------------------------------------------------------------ batched form */

/* Many scenes, many cameras per step, in one launch: the scenes are row
 * ranges of one model [scene_row0[s], scene_row0[s+1]), each starting at a
 * multiple of 1024 rows (pad with rows of NaN geometry, which never become
 * visible).  Camera slot c of scene s at update t is record
 * cams[((t-1) % n_sets) * n_scenes * C + s * C + c] (records from
 * gs_camera_pack, uploaded by the caller).  Outputs of gs_cull_multi:
 *   union_ids[0..U)  rows visible to at least one camera of their scene,
 *                    ascending (U = *union_count; gather and update these);
 *   cam_pos[c*cap_cam + i]  union positions of the rows camera slot c sees,
 *                    ascending over all scenes (cam_count[c] entries);
 *   scene_start[s*(1+C) + j]  first entry of scene s in the union list (j = 0)
 *                    and in each camera list (j = 1 + c).
 * Deterministic; counts beyond a capacity are reported, not written.  Only
 * max_defer = 0 and geo_mode = 0 models are supported. */
typedef struct gs_multi {
    int32_t n_scenes, cams_per_scene, n_sets, variant;   /* variant: see gs_cull_multi_autotune */
    const int64_t *scene_row0;   /* device [n_scenes + 1] */
    const void *cams;            /* device camera records */
    uint32_t *union_ids, *union_count;
    uint32_t *cam_pos, *cam_count;
    uint32_t cap_union, cap_cam;
    uint32_t *scene_start;       /* device [n_scenes][1 + cams_per_scene] */
    uint32_t *chunk_start;       /* optional device [ceil(cap_union / 128) + 1][cams_per_scene]:
                                    for union position 128 k and camera slot c, the index in list c
                                    of its first entry at a position >= 128 k (written by
                                    gs_cull_multi, read by gs_grad_sum_multi instead of binary
                                    searches); NULL: gs_grad_sum_multi searches */
} gs_multi;

/* Size of one camera record (256 bytes), and packing of `count` cameras for
 * `model` (camera matrices plus the rounded-up constants of the band
 * classifier and of the summary cull's side test).  Records feed
 * gs_cull_multi and gs_cull_table. */
int gs_camera_pack_bytes(size_t *bytes);
int gs_camera_pack(const gs_model *model, const gs_camera *cams, int32_t count, void *out_host);

/* Workspace of gs_cull_multi: per-row camera bits and per-tile counts and
 * prefixes (about 6.1 bytes per Gaussian; needs no initialisation). */
int gs_multi_workspace_bytes(const gs_model *model, size_t *bytes);

/* Batched cull + ordered compaction of every (scene, camera) pair (Sec. 2.4
 * step 1 per camera; the union is the paper's valid_ids of a multi-image
 * batch).  Each tile of geometry is read once and tested against all cameras
 * of its scene. */
int gs_cull_multi(const gs_model *model, const gs_multi *desc, int64_t step, void *ws, size_t ws_bytes,
                  void *stream);

/* Times every variant of gs_cull_multi on the given inputs (synchronising
 * `stream`), stores the fastest in desc->variant and, when times_ms is not
 * NULL, each variant's mean time (times_ms holds GS_MULTI_VARIANTS floats).
 * Variant v = (block size, rows per thread): 0..4 = (64; 1, 2, 4, 8, 16),
 * 5..8 = (128; 1, 2, 4, 8), 9..11 = (256; 1, 2, 4), 12..13 = (512; 1, 2),
 * 14 = (1024, 1).  A tile of block x rows is at most 1024 rows because a tile
 * must lie inside one scene. */
#define GS_MULTI_VARIANTS 15
int gs_cull_multi_autotune(const gs_model *model, gs_multi *desc, int64_t step, void *ws, size_t ws_bytes,
                           void *stream, float *times_ms, int32_t *n_variants);

/* Deterministic gradient sum of a batch: out[p] = sum over camera slots c, in
 * slot order, of g_cam[c*cap_cam + i] for the entry i of list c with
 * cam_pos = p.  g_cam rows are [10 + adim] floats (G columns then A); the
 * result is split into out_geo [cap_union][10] and out_app [cap_union][adim],
 * ready for gs_adam_step_deferred with ids = union_ids. */
int gs_grad_sum_multi(const gs_multi *desc, int32_t adim, const float *g_cam, float *out_geo, float *out_app,
                      void *stream);

/* Balance-aware image split (Sec. 4.4), a planning call (synchronises
 * `stream`): if more than mem_limit * n Gaussians are visible in `cam`, find
 * a split column x so that the crops [0, x) and [x, W) (same intrinsics, the
 * right crop's principal point shifted by -x) see similar counts: start at
 * the midpoint and move x toward the less populated side with a 5-step
 * binary search, culling both sides each time.  *split_x = 0 means no split.
 * counts (optional, 3 entries): visible in the whole image, in the left and
 * in the right crop at the chosen x.  desc must describe one scene, two
 * cameras and one set; its camera records are overwritten and its capacities
 * are ignored (only counts are produced).  Train a split image as a batch of
 * the two crops: gs_cull_multi gives the union and the per-crop lists,
 * gs_grad_sum_multi sums the crops' gradients, one gs_adam_step_deferred. */
int gs_plan_image_split(const gs_model *model, const gs_camera *cam, int64_t step, double mem_limit, gs_multi *desc,
                        void *ws, size_t ws_bytes, void *stream, int32_t *split_x, uint32_t *counts);

/* ----------------------------------------------------------- densification */

/* Densification (Sec. 2.4 step 7: rows with large accumulated gradients are
 * cloned or split, insignificant low-opacity rows pruned), with the criteria
 * of 3D Gaussian Splatting on current FP32 values (flush the model at `step`
 * first).  Per row: g = accum/denom (0 when denom = 0); grad = g >= threshold;
 * smax = largest log-scale; clone if grad and smax <= log(percent_dense *
 * extent), split if grad and above; prune if the opacity logit (appearance
 * column 0) < logit(min_opacity), if prune_big and smax > log(0.1 extent), or
 * (originals only) if max_screen_size > 0 and radii > max_screen_size.  A clone
 * copies its row; a split row is replaced by two children with log-scales
 * s - log 1.6 and positions mu + R(q) (exp(s) * z), z a normal-approximation
 * draw (sum of the four 16-bit fields of SplitMix64(seed, row, child, axis),
 * centred and scaled to unit variance in FP64); children are pruned on their
 * own scales.  Output rows: kept originals in order, then kept clones, then
 * kept children (parent order, child 0 first).  New rows start with zero
 * moments; every output row has last_step = step.  Thresholds are FP64 logs
 * rounded once to FP32.  FP32 or BF16 state (FP8 block scales do not move
 * with rows). */
typedef struct gs_densify_params {
    float grad_threshold;  /* 3DGS: 0.0002 */
    float percent_dense;   /* 3DGS: 0.01 */
    float scene_extent;    /* > 0 */
    float min_opacity;     /* 3DGS: 0.005, in (0, 1) */
    float max_screen_size; /* pixels; 0 = off */
    int32_t prune_big;     /* 1: prune rows larger than 0.1 extent in world space */
    uint64_t seed;         /* split draws */
} gs_densify_params;

/* Workspace of the two calls below (per-row codes and per-tile counts). */
int gs_densify_workspace_bytes(const gs_model *model, size_t *bytes);

/* Classify every row of `model` and count the output rows (originals, clones,
 * children; counts optional, 3 entries).  grad_accum, grad_denom: device [n];
 * max_radii2d: device [n] or NULL.  Synchronises `stream` to return *n_out. */
int gs_densify_plan(const gs_model *model, const float *grad_accum, const float *grad_denom,
                    const float *max_radii2d, const gs_densify_params *params, void *ws, size_t ws_bytes,
                    void *stream, int64_t *n_out, int64_t *counts);

/* Write the planned rows into `dst` (dst->n == *n_out of the plan, same
 * column rates, appearance dim and moment storage as src; any layout).  Reads
 * the codes the plan left in `ws`; asynchronous. */
int gs_densify_apply(const gs_model *src, const gs_densify_params *params, const gs_model *dst, int64_t step,
                     void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------------------------------- harness */

/* Synthetic gradients for benchmarks and tests (not part of the method):
 * out[i][c] for i < min(*count_dev, capacity), c < dim, is the SplitMix64
 * (Steele, Lea & Flood 2014) derived value for key = ids[i] (or i when ids is
 * NULL) and global column col0 + c: s1 = at(seed, step), s2 = at(s1, key),
 * h = at(s2, col) with at(s, k) = mix64(s + (k+1)*0x9E3779B97F4A7C15); the
 * four 16-bit fields of h are summed, centred and scaled to std `sigma`. */
int gs_synth_grad(uint64_t seed, int64_t step, const uint32_t *ids, const uint32_t *count_dev,
                  uint32_t capacity, int32_t dim, int32_t col0, double sigma, float *out,
                  void *stream);

/* Measurement helper (not part of the method): one streaming read of `bytes`
 * bytes at device address `buf` (16-byte aligned, bytes a multiple of 16) in
 * the cull's access pattern: one block per 20 KB tile, non-temporal 16-byte
 * loads all in flight before the first is used.  Timing it on the [n][10]
 * geometry array gives the read bandwidth the cull's main stream can reach on
 * this part.  *sink (device float) is written only when the data sum to a
 * value finite data never sum to, so nothing is stored in practice.  Returns
 * GS_EINVAL on a null or misaligned argument or more than 2^31 - 1 tiles. */
int gs_stream_read_probe(const void *buf, size_t bytes, float *sink, void *stream);

/* Measurement only: the row kernels' access pattern without their
 * arithmetic.  For i < count, one wavefront loads row ids[i] (row_bytes, a
 * multiple of 16 up to 1024, rows contiguous from `base`, 16-byte aligned)
 * with 16-byte loads, four rows in flight; with write != 0 it stores every
 * loaded 16 bytes back unchanged (the same bits: the traffic of a
 * read-modify-write that changes nothing).  Ids >= n_rows are skipped.
 * Timing it on a model's fused rows and an update's visible ids gives the
 * bandwidth the hardware reaches for that row set.  GS_EINVAL on a null or
 * misaligned argument or a row size out of range. */
int gs_row_probe(const uint32_t *ids, uint32_t count, void *base, uint64_t n_rows, uint32_t row_bytes, int32_t write,
                 float *sink, void *stream);

/* Number of compute units of the current device (0 when none). */
int gs_device_cu_count(void);

/* Human-readable name of a status code. */
const char *gs_status_string(int status);

/* Text of the last HIP error seen by this thread ("" if none). */
const char *gs_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GSDP_H */
