/*
 * gs_oracle.c -- CPU oracle for the per-iteration Gaussian-parameter path of
 * GS-Scale (arXiv 2509.15645).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header
 * or table with the HIP library; the two meet only through seeded inputs.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * Every float expression below is evaluated one IEEE binary32 (or binary64)
 * operation at a time, left to right as parenthesised, with no contraction.
 *
 * Contents
 *   orc_exp_gs          exp for the cull (Cody & Waite 1980 reduction + Taylor)
 *   orc_cull_v1         FP32 frustum/screen cull of one camera (Sec. 2.4 step 1,
 *                       Sec. 3.4 challenge 1; formula fixed as the 3-sigma EWA box)
 *   orc_compact         ascending ids of the kept rows (valid_ids, Sec. 4.1)
 *   orc_adam_dense_f64  dense Adam, Eq. 1 -- the definition the method reaches
 *   orc_restore_coeff_f64  restore coefficients of Eq. 3 as the sum over the
 *                       skipped steps, FP64 (the paper's lookup tables)
 *   orc_deferred_rows_f64  restore + decayed moments + Adam step, FP64 (model O2)
 *   orc_lut_spec        FP32 tables of the implementation spec (model O3)
 *   orc_restore_bound   clamp of the restore factor (above the Adam ratio bound)
 *   orc_deferred_rows_f32  the same update with FP32 math and FP32 (O3) or
 *                       BF16 stochastically rounded (O4) moments, fixed op order
 *   orc_restore_rows_f32   restore-only (read-only forwarding, Sec. 4.3.3)
 *   orc_flush_rows_*    catch-up of skipped zero-gradient steps (Eq. 2-3)
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* exp for the cull: Cody-Waite argument reduction with ln2 split into a
 * 9-bit head (355/512, so k*LN2_HI is exact for |k| <= 128) and an FP32 tail,
 * then the degree-7 Taylor polynomial of e^r on |r| <= ln2/2 in Horner form,
 * then scaling by 2^k.  Only +,-,*, rint and ldexp are used, each exactly
 * rounded, so any IEEE machine gets the same bits.  NaN propagates (the
 * clamp uses ordered comparisons). */
float orc_exp_gs(float x)
{
    const float LOG2E = 1.44269504088896341f;
    const float LN2_HI = 0.693359375f;          /* 355/512 */
    const float LN2_LO = -2.12194440e-4f;       /* ln2 - 355/512 */
    if (x < -87.0f) x = -87.0f;
    if (x > 88.0f) x = 88.0f;
    float k = rintf(x * LOG2E);
    float r = (x - k * LN2_HI) - k * LN2_LO;
    float p = 1.98412698e-4f;                   /* 1/7! */
    p = p * r + 1.38888889e-3f;                 /* 1/6! */
    p = p * r + 8.33333333e-3f;                 /* 1/5! */
    p = p * r + 4.16666667e-2f;                 /* 1/4! */
    p = p * r + 1.66666667e-1f;                 /* 1/3! */
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return ldexpf(p, (int)k);
}

/* ------------------------------------------------------------------------ */
/* Cull of one Gaussian.  The paper states what culling does -- drop Gaussians
 * outside the near/far planes, project mean and covariance to the image, drop
 * 2D Gaussians outside the image -- using only mean, scale and quaternion
 * (Sec. 2.4 step 1; Sec. 4.1 step 1; Sec. 4.2.1).  It does not print a formula;
 * this is the EWA screen-space test of 3D Gaussian Splatting: 3-sigma radius of
 * the projected covariance (with the 0.3 px low-pass dilation) around the
 * projected centre, tested against the image rectangle.
 *
 * cam[20] = R(9, row-major world->camera), t(3), fx, fy, cx, cy, W, H, near, far.
 * detail (optional, 11 floats): x y z u v a b c det lambda r. */
static int cull_one(const float *g, const float *cam, float *detail)
{
    const float *R = cam, *T = cam + 9;
    const float fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const float W = cam[16], H = cam[17], zn = cam[18], zf = cam[19];

    /* 1. centre in camera space */
    float x = ((R[0] * g[0] + R[1] * g[1]) + R[2] * g[2]) + T[0];
    float y = ((R[3] * g[0] + R[4] * g[1]) + R[5] * g[2]) + T[1];
    float z = ((R[6] * g[0] + R[7] * g[1]) + R[8] * g[2]) + T[2];

    /* 2. unit quaternion (w,x,y,z) -> rotation */
    float qw = g[6], qx = g[7], qy = g[8], qz = g[9];
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    float inv = 1.0f / sqrtf(n2);
    qw = qw * inv; qx = qx * inv; qy = qy * inv; qz = qz * inv;
    float Q[9];
    Q[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
    Q[1] = 2.0f * (qx * qy - qw * qz);
    Q[2] = 2.0f * (qx * qz + qw * qy);
    Q[3] = 2.0f * (qx * qy + qw * qz);
    Q[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
    Q[5] = 2.0f * (qy * qz - qw * qx);
    Q[6] = 2.0f * (qx * qz - qw * qy);
    Q[7] = 2.0f * (qy * qz + qw * qx);
    Q[8] = 1.0f - 2.0f * (qx * qx + qy * qy);

    /* 3. scales from log-scales */
    float s0 = orc_exp_gs(g[3]), s1 = orc_exp_gs(g[4]), s2 = orc_exp_gs(g[5]);

    /* 4. world covariance  Sigma = (Q S)(Q S)^T */
    float M[9];
    for (int a = 0; a < 3; ++a) {
        M[3 * a + 0] = Q[3 * a + 0] * s0;
        M[3 * a + 1] = Q[3 * a + 1] * s1;
        M[3 * a + 2] = Q[3 * a + 2] * s2;
    }
    float S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            S[3 * a + b] = (M[3 * a + 0] * M[3 * b + 0] + M[3 * a + 1] * M[3 * b + 1])
                           + M[3 * a + 2] * M[3 * b + 2];

    /* 5. Jacobian of the pinhole projection at the centre, with the
     *    tangent clamped to 1.3x the half field of view */
    float rz = 1.0f / z;
    float limx = 1.3f * ((0.5f * W) / fx);
    float limy = 1.3f * ((0.5f * H) / fy);
    float tx = x * rz, ty = y * rz;
    if (tx < -limx) tx = -limx;
    if (tx > limx) tx = limx;
    if (ty < -limy) ty = -limy;
    if (ty > limy) ty = limy;
    float J00 = fx * rz, J02 = -(fx * tx) * rz;
    float J11 = fy * rz, J12 = -(fy * ty) * rz;

    /* 6. 2D covariance  T Sigma T^T  with T = J R */
    float T0[3], T1[3];
    for (int j = 0; j < 3; ++j) {
        T0[j] = J00 * R[j] + J02 * R[6 + j];
        T1[j] = J11 * R[3 + j] + J12 * R[6 + j];
    }
    float U0[3], U1[3];
    for (int j = 0; j < 3; ++j) {
        U0[j] = (T0[0] * S[j] + T0[1] * S[3 + j]) + T0[2] * S[6 + j];
        U1[j] = (T1[0] * S[j] + T1[1] * S[3 + j]) + T1[2] * S[6 + j];
    }
    float a = ((U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2]) + 0.3f;
    float b = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
    float c = ((U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2]) + 0.3f;

    /* 7. largest eigenvalue and 3-sigma pixel radius */
    float det = a * c - b * b;
    float mid = 0.5f * (a + c);
    float disc = mid * mid - det;
    if (!(disc > 0.1f)) disc = 0.1f;
    float lam = mid + sqrtf(disc);
    float r = ceilf(3.0f * sqrtf(lam));

    /* 8. projected centre in pixels */
    float u = (fx * x) * rz + cx;
    float v = (fy * y) * rz + cy;

    if (detail) {
        detail[0] = x; detail[1] = y; detail[2] = z; detail[3] = u; detail[4] = v;
        detail[5] = a; detail[6] = b; detail[7] = c; detail[8] = det; detail[9] = lam;
        detail[10] = r;
    }
    /* 9. conjunction of positive comparisons: any NaN culls */
    return (z > zn) && (z < zf) && (det > 0.0f) && (u + r > 0.0f) && (u - r < W)
           && (v + r > 0.0f) && (v - r < H);
}

void orc_cull_v1(int64_t n, const float *geo, const float *cam, uint8_t *keep, float *detail)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        keep[i] = (uint8_t)cull_one(geo + 10 * i, cam, detail ? detail + 11 * i : NULL);
}

/* Thread count of the OpenMP loops (the CPU baseline times one thread and
 * all cores); returns the previous maximum. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
#else
    (void)n;
    return 1;
#endif
}

/* valid_ids: ids of kept rows in ascending order.  Returns the count. */
int64_t orc_compact(int64_t n, const uint8_t *keep, uint32_t *ids)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (keep[i]) ids[m++] = (uint32_t)i;
    return m;
}

/* ------------------------------------------------------------------------ */
/* Dense Adam, Eq. 1, stepped on every row (g = NULL means all-zero grads):
 *   m = b1 m + (1-b1) g ;  v = b2 v + (1-b2) g^2
 *   w = w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)                */
void orc_adam_dense_f64(int64_t n, int dim, double *w, double *m, double *v, const double *g,
                        const double *lr, double b1, double b2, double eps, int64_t t)
{
    const double bc1 = 1.0 - pow(b1, (double)t);
    const double bc2 = 1.0 - pow(b2, (double)t);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < dim; ++k) {
            int64_t e = i * dim + k;
            double gi = g ? g[e] : 0.0;
            m[e] = b1 * m[e] + (1.0 - b1) * gi;
            v[e] = b2 * v[e] + (1.0 - b2) * gi * gi;
            double mhat = m[e] / bc1;
            double vhat = v[e] / bc2;
            w[e] = w[e] - lr[k] * mhat / (sqrt(vhat) + eps);
        }
    }
}

/* Dense Adam where only the listed rows carry a gradient (compact rows
 * g_rows[j] belong to row ids[j]); every other row steps with g = 0. */
void orc_adam_dense_sparse_grad_f64(int64_t n, int dim, double *w, double *m, double *v,
                                    int64_t n_ids, const uint32_t *ids, const float *g_rows,
                                    const double *lr, double b1, double b2, double eps, int64_t t)
{
    double *g = (double *)calloc((size_t)n * dim, sizeof(double));
    for (int64_t j = 0; j < n_ids; ++j)
        for (int k = 0; k < dim; ++k)
            g[(int64_t)ids[j] * dim + k] = (double)g_rows[j * dim + k];
    orc_adam_dense_f64(n, dim, w, m, v, g, lr, b1, b2, eps, t);
    free(g);
}

/* ------------------------------------------------------------------------ */
/* Restore coefficients of Eq. 3, FP64, for update t with a unit learning rate
 * (the restore is linear in lr; callers multiply by the column's rate).  A row
 * deferred d steps last took update s0 = t-1-d and skipped k = s0+1 .. t-1.
 * With g = 0 its moments at step k are b1^(k-s0) m and b2^(k-s0) v, so step k
 * moves w by lr (b1^(k-s0) m/(1-b1^k)) / (sqrt(b2^(k-s0) v/(1-b2^k)) + eps);
 * with eps moved out of the sum (the paper's approximation, Sec. 4.3.1) the d
 * steps move w by lr coef[d] m/(sqrt(v)+eps), where
 *   coef[d] = sum_{k=s0+1}^{t-1} s_k (b1/sqrt(b2))^(k-s0) sqrt(1-b2^k)/(1-b1^k)
 * (s_k: the rate multiplier of step k under a schedule, else 1).  The moments
 * reach m_dec[d] m, v_dec[d] v at step t before its own gradient is added:
 *   m_dec[d] = b1^(d+1),  v_dec[d] = b2^(d+1).
 * Entries exist for d = 0..dmax, dmax <= t-1 (a row cannot have skipped more). */
void orc_restore_coeff_f64(double b1, double b2, int64_t t, int dmax, const double *sched,
                           double *coef, double *m_dec, double *v_dec)
{
    for (int d = 0; d <= dmax; ++d) {
        const int64_t s0 = t - 1 - d;
        double sum = 0.0;
        for (int64_t k = s0 + 1; k <= t - 1; ++k) {
            const double decay = pow(b1 / sqrt(b2), (double)(k - s0));
            const double corr = sqrt(1.0 - pow(b2, (double)k)) / (1.0 - pow(b1, (double)k));
            sum += (sched ? sched[k] : 1.0) * decay * corr;
        }
        coef[d] = sum;
        m_dec[d] = pow(b1, (double)(d + 1));
        v_dec[d] = pow(b2, (double)(d + 1));
    }
}

/* Model O2: the deferred update in FP64 for the update rows rows[j] with
 * defer counts d[j] and compact gradients g[j][:] (zero rows for saturated
 * Gaussians).  Per column k with rate lr[k] (Eq. 2-3):
 *   restore the skipped steps with the stored moments:
 *       w -= lr coef[d] m / (sqrt(v) + eps)                     (d > 0)
 *   decay the moments over them and add this step's gradient (Eq. 2):
 *       m <- b1^(d+1) m + (1-b1) g,   v <- b2^(d+1) v + (1-b2) g^2
 *   take the ordinary Adam step of update t with the new moments (Eq. 1):
 *       w -= (lr s_t / (1-b1^t)) m / (sqrt(v) / sqrt(1-b2^t) + eps)
 * (The new v belongs in the last line: the text applies the standard Adam
 * update there; the old v would make the step diverge.) */
void orc_deferred_rows_f64(int dim, double *w, double *m, double *v, int64_t n_rows,
                           const uint32_t *rows, const int64_t *d, const double *g,
                           const double *lr, double b1, double b2, double eps, int64_t t, double lr_scale_t,
                           const double *coef, const double *m_dec, const double *v_dec)
{
    const double corr2 = sqrt(1.0 - pow(b2, (double)t));
    const double corr1 = 1.0 - pow(b1, (double)t);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        const int64_t id = rows[j];
        const int64_t dj = d[j];
        for (int k = 0; k < dim; ++k) {
            const int64_t e = id * dim + k;
            const double gk = g ? g[j * dim + k] : 0.0;
            double wk = w[e];
            if (dj > 0) wk -= (coef[dj] * lr[k] * m[e]) / (sqrt(v[e]) + eps);
            const double m1 = m_dec[dj] * m[e] + (1.0 - b1) * gk;
            const double v1 = v_dec[dj] * v[e] + (1.0 - b2) * gk * gk;
            m[e] = m1;
            v[e] = v1;
            w[e] = wk - ((lr[k] * lr_scale_t) / corr1) * m1 / (sqrt(v1) / corr2 + eps);
        }
    }
}

/* Restore-only in FP64: current value of rows with defer count d (read-only). */
void orc_restore_rows_f64(int dim, const double *w, const double *m, const double *v,
                          int64_t n_rows, const uint32_t *rows, const int64_t *d,
                          const double *lr, double eps, const double *coef, double *out)
{
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * dim + k;
            double wk = w[e];
            if (d[j] > 0) wk -= (coef[d[j]] * lr[k] * m[e]) / (sqrt(v[e]) + eps);
            out[j * dim + k] = wk;
        }
    }
}

/* Flush in FP64 after update `t`: rows rows[j] skipped delta[j] >= 1 steps.
 * Their value after update t is the restore of update t+1 with d = delta
 * (coef_next: the coefficients of step t+1), and the moments decay by b^delta. */
void orc_flush_rows_f64(int dim, double *w, double *m, double *v, int64_t n_rows,
                        const uint32_t *rows, const int64_t *delta, const double *lr,
                        double b1, double b2, double eps, const double *coef_next)
{
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dl = delta[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * dim + k;
            w[e] -= (coef_next[dl] * lr[k] * m[e]) / (sqrt(v[e]) + eps);
            m[e] *= pow(b1, (double)dl);
            v[e] *= pow(b2, (double)dl);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Model O3: the implementation's FP32 arithmetic, written out independently.
 *
 * FP32 tables for update step t (computed in FP64, rounded once):
 *   P1[k] = b1^k, P2[k] = b2^k by repeated multiplication from P[0] = 1
 *   C[k]  = s_k b1 / ( sqrt(b2 / (1 - P2[k])) * (1 - P1[k]) )       k >= 1
 *   R[j]  = (b1/sqrt(b2))^j by repeated multiplication from R[0] = 1
 *   W[d]  = the restore coefficient of Eq. 3 summed over the skipped steps in
 *           time order, k = t-d .. t-1, from 0:
 *           (((0 + R[0] C[t-d]) + R[1] C[t-d+1]) + ...) + R[d-1] C[t-1]
 *           (the implementation keeps these sums for the current step and
 *           extends them by one skipped step per update)
 *   Wf[d] = W[d], Mf[d] = P1[d+1], Vf[d] = P2[d+1],
 *   ss = s_t/(1 - P1[t]),  bc = sqrt(1 - P2[t])              (all as FP32)     */
void orc_lut_spec(double b1, double b2, int64_t t, int dmax, const double *sched, float *Wf, float *Mf,
                  float *Vf, float *ss, float *bc)
{
    int64_t kmax = t > dmax + 1 ? t : dmax + 1;
    double *P1 = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *P2 = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *C = (double *)calloc((size_t)(kmax + 1), sizeof(double));
    double *R = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    P1[0] = 1.0; P2[0] = 1.0;
    for (int64_t k = 1; k <= kmax; ++k) { P1[k] = P1[k - 1] * b1; P2[k] = P2[k - 1] * b2; }
    for (int64_t k = 1; k < t; ++k) {
        C[k] = b1 / (sqrt(b2 / (1.0 - P2[k])) * (1.0 - P1[k]));
        if (sched) C[k] = sched[k] * C[k];
    }
    double r = b1 / sqrt(b2);
    R[0] = 1.0;
    for (int j = 1; j <= dmax; ++j) R[j] = R[j - 1] * r;
    for (int d = 0; d <= dmax; ++d) {
        double W = 0.0;
        for (int j = 0; j < d; ++j) W = W + R[j] * C[t - d + j];
        Wf[d] = (float)W;
    }
    for (int d = 0; d <= dmax; ++d) { Mf[d] = (float)P1[d + 1]; Vf[d] = (float)P2[d + 1]; }
    *ss = sched ? (float)(sched[t] / (1.0 - P1[t])) : (float)(1.0 / (1.0 - P1[t]));
    *bc = (float)sqrt(1.0 - P2[t]);
    free(P1); free(P2); free(C); free(R);
}

/* Bound on the restore factor m/(sqrt(v)+eps).  For Adam moments grown from
 * zero, Cauchy-Schwarz gives |m|/sqrt(v) <= (1-b1)/sqrt((1-b2)(1-b1^2/b2))
 * (7.27 for b = 0.9, 0.999); the restore clamps the factor at 1.03 times
 * that, which leaves every reachable FP32 state untouched and bounds how far
 * a restore can move a parameter whatever the stored moments are.
 * +inf (no clamp) when b1^2 >= b2. */
float orc_restore_bound(double b1, double b2)
{
    if (!(b1 * b1 < b2)) return INFINITY;
    return (float)((1.0 - b1) / sqrt((1.0 - b2) * (1.0 - b1 * b1 / b2)) * 1.03);
}

/* Moment storage: state 0 = FP32, state 1 = BF16 (upper 16 bits of the FP32
 * pattern).  Stores round stochastically: the 16 random bits are added to the
 * FP32 pattern before truncation, so x rounds up with probability equal to
 * the dropped fraction.  Inf stays Inf, NaN stays a quiet NaN. */
static float mom_load(const void *p, int state, int64_t e)
{
    if (state == 0) return ((const float *)p)[e];
    uint32_t u = (uint32_t)((const uint16_t *)p)[e] << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

static void mom_store(void *p, int state, int64_t e, float x, uint32_t r16)
{
    if (state == 0) {
        ((float *)p)[e] = x;
        return;
    }
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        uint16_t h = (uint16_t)(u >> 16);
        if (u & 0x007fffffu) h |= 0x0040u;
        ((uint16_t *)p)[e] = h;
        return;
    }
    u += r16;
    ((uint16_t *)p)[e] = (uint16_t)(u >> 16);
}

/* One BF16 stochastic rounding (exposed for tests). */
uint16_t orc_bf16_sr(float x, uint32_t r16)
{
    uint16_t h;
    mom_store(&h, 1, 0, x, r16);
    return h;
}

/* SplitMix64 (Steele, Lea & Flood 2014): output k of the stream seeded s. */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t sm_at(uint64_t s, uint64_t k) { return mix64(s + (k + 1) * 0x9E3779B97F4A7C15ull); }

/* Random bits of element (step t, row id, global column col): bits 0..15 round m,
 * bits 16..31 round v. */
static uint64_t sr_bits(uint64_t seed, int64_t t, int64_t id, int64_t col)
{
    return sm_at(sm_at(sm_at(seed, (uint64_t)t), (uint64_t)id), (uint64_t)col);
}

/* O3 restore of one element (d > 0 only): q = m / (sqrt(v)+eps) clamped to
 * [-rb, rb], then w - (Wf[d]*lr) * q. */
static float restore32(float w, float m, float v, float wd, float lr, float eps, float rb)
{
    float den = sqrtf(v) + eps;
    float q = m / den;
    if (q > rb) q = rb;
    else if (q < -rb) q = -rb;
    float wsc = wd * lr;
    return w - wsc * q;
}

/* Adam step of one element: (st*m1) / (sqrt(v1)/bc + eps), with the step
 * clamped to st*bc*rb.  For moments grown from zero |m1|/sqrt(v1) <= 7.27 < rb,
 * so the clamp never acts on an FP32 state; it bounds the step when quantised
 * moments lose the second moment to underflow. */
static float adam_step32(float m1, float v1, float st, float bc, float eps, float rb)
{
    float den = sqrtf(v1) / bc + eps;
    float upd = (st * m1) / den;
    float lim = (st * bc) * rb;
    if (upd > lim) upd = lim;
    else if (upd < -lim) upd = -lim;
    return upd;
}

/* ------------------------------------------------------------------------ */
/* A-posteriori error bound of the quantised-moment models (O4) against dense
 * FP64 Adam (Eq. 1), carried along the model's own trajectory.
 *
 * Given the visible sets and the gradients, the moments of an element evolve
 * independently of w, and every move of w is a sum of per-step terms:
 *   exact (dense FP64):  lr c_k m_k / (sqrt(v_k) + eps_k)      c_k = s_k bc_k / (1 - b1^k)
 *   model:               lr c_k clamp(m~ / (sqrt(v~) + eps), +-rb)
 * (a deferred row's catch-up is the sum over its skipped steps k of
 * lr c_k r^j with r = b1/sqrt(b2), i.e. lr W[d] times one ratio).  Per
 * element we keep
 *   em >= |m~ - m|, ev >= |v~ - v|   the stored (decoded) moments against the
 *                                    exact ones: each update multiplies the
 *                                    old bound by b^(d+1) and adds the actual
 *                                    rounding of the store (|stored - value|,
 *                                    an FP8 re-encode adds its own) plus an
 *                                    FP32 arithmetic slack;
 *   bw >= |w~ - w|                   the sum over steps of lr c_k times the
 *                                    largest ratio difference over every
 *                                    exact (m, v) inside the moment bounds,
 *                                    plus the FP32 rounding of w.
 * Exact moments grown from zero obey |m| / sqrt(v) <= cs = (1-b1) /
 * sqrt((1-b2)(1 - b1^2/b2)) (Cauchy-Schwarz), so the exact ratio is clipped
 * to [-cs, cs]; the model's ratio is clamped to [-rb, rb].  Nothing else is
 * assumed: a code far below its block scale (E4M3 subnormals, a lost second
 * moment) widens the interval and the bound falls back towards lr c_k (rb + cs)
 * per step. */
typedef struct orc_track {
    const uint32_t *keys;   /* stochastic-rounding key of each local row (NULL: the row index) */
    double *em, *ev, *bw;   /* [n][ld] bounds, or NULL (no tracking) */
    double cs;              /* Cauchy-Schwarz bound of |m| / sqrt(v) */
} orc_track;

#define ORC_U32 5.9604644775390625e-08      /* 2^-24: unit roundoff of binary32 */

static int64_t sr_key(const orc_track *trk, int64_t id)
{
    return (trk && trk->keys) ? (int64_t)trk->keys[id] : id;
}

/* Largest |clamp(mt / (sqrt(vt) + eps), +-rb) - m / (sqrt(v) + eps)| over
 * m in [mt - em, mt + em], v in [max(vt - ev, 0), vt + ev], with the exact
 * ratio clipped to [-cs, cs].  The model evaluates its ratio in FP32: three
 * roundings of at most 2^-24 relative are added. */
static double ratio_dev(double mt, double vt, double em, double ev, double eps, double rb, double cs)
{
    double a = mt / (sqrt(vt) + eps);
    if (!(a == a)) return rb + cs;
    if (a > rb) a = rb;
    else if (a < -rb) a = -rb;
    double mlo = mt - em, mhi = mt + em;
    double vlo = vt - ev;
    if (vlo < 0.0) vlo = 0.0;
    double dlo = sqrt(vlo) + eps, dhi = sqrt(vt + ev) + eps;
    if (dlo < 1e-300) dlo = 1e-300;
    double ulo, uhi;
    if (mlo >= 0.0) {
        ulo = mlo / dhi;
        uhi = mhi / dlo;
    } else if (mhi <= 0.0) {
        ulo = mlo / dlo;
        uhi = mhi / dhi;
    } else {
        ulo = mlo / dlo;
        uhi = mhi / dlo;
    }
    if (ulo < -cs) ulo = -cs;
    if (ulo > cs) ulo = cs;
    if (uhi < -cs) uhi = -cs;
    if (uhi > cs) uhi = cs;
    double d = fabs(a - ulo);
    if (fabs(a - uhi) > d) d = fabs(a - uhi);
    return d * (1.0 + 1e-12) + 4.0 * ORC_U32 * fabs(a);
}

/* Bound of the catch-up of one element deferred d > 0 steps (restore of
 * Eq. 3 with the stored moments mt, vt): lr W (ratio difference + the eps
 * factor-out), plus FP32 slack.  The exact skipped step j after the last
 * update divides m by sqrt(v) + e' with e' = eps bc_k b2^(-j/2) in
 * [eps sqrt(1-b2), eps b2^(-d/2)] instead of sqrt(v) + eps, which changes the
 * ratio by at most |m| e_max / ((sqrt(v) + eps)(sqrt(v) + e_min)) (and by at
 * most cs, both ratios lying in [-cs, cs]). */
static double restore_dev(double mt, double vt, double em, double ev, double eps, double rb, double cs,
                          double wd, double lr, int64_t d, double b2)
{
    double dev = ratio_dev(mt, vt, em, ev, eps, rb, cs);
    double vlo = vt - ev;
    double sv = vlo > 0.0 ? sqrt(vlo) : 0.0;
    double emax = eps * pow(b2, -0.5 * (double)d), emin = eps * sqrt(1.0 - b2);
    double mabs = fabs(mt) + em;
    double et = 0.0;
    if (mabs > 0.0) {
        double den = (sv + eps) * (sv + emin);
        et = den > 0.0 ? mabs * emax / den : cs;
        if (!(et <= cs)) et = cs;
    }
    return fabs(lr) * wd * (1.0 + 4.0 * ORC_U32) * (dev + et);
}

/* O3/O4 update of the rows rows[j] (defer count d[j], FP32 compact gradient
 * g[j][:] or zero when g == NULL).  w is [n][ld] FP32; m, v are [n][ld] in the
 * given storage.  Global column of k is col0 + k (SR random stream). */
/* Bound bookkeeping of one update of a tracked element (see orc_track):
 * stored moments (mk, vk) with gap d, restore w0 -> wr (d > 0), new FP32
 * moments (m1, v1) from gradient gk, Adam step upd (wr -> w1), stored
 * results decoded as (ms, vs). */
static void track_update(const orc_track *trk, int64_t e, int64_t d, double Wd, double Mfd, double Vfd,
                         double omb1, double omb2, double gk, double lr, double ss, double bc, double eps,
                         double rb, double b2, double w0, double wr, double w1, double upd, double mk,
                         double vk, double m1, double v1, double ms, double vs)
{
    const double u = ORC_U32, cs = trk->cs;
    double em0 = trk->em[e], ev0 = trk->ev[e], b = trk->bw[e];
    if (d > 0) b += restore_dev(mk, vk, em0, ev0, eps, rb, cs, Wd, lr, d, b2) + 4.0 * u * fabs(w0 - wr);
    /* the FP32 moment update against the exact one: decayed old bound plus
     * the roundings of the tables (1 - b1 and b^(d+1) rounded once) and of the
     * three operations */
    double em1 = Mfd * em0 * (1.0 + 2.0 * u) + 4.0 * u * (fabs(Mfd * mk) + fabs(omb1 * gk)) + 1e-14 * fabs(m1);
    double ev1 = Vfd * ev0 * (1.0 + 2.0 * u) + 5.0 * u * (fabs(Vfd * vk) + fabs(omb2 * gk * gk)) + 1e-14 * fabs(v1);
    /* the Adam step lr ss bc clamp(m1 / (sqrt(v1) + bc eps)), evaluated in FP32
     * with tables rounded once: about nine roundings of the step */
    b += fabs(lr) * ss * bc * ratio_dev(m1, v1, em1, ev1, bc * eps, rb, cs) + 12.0 * u * fabs(upd);
    /* FP32 rounding of the two subtractions from w */
    b += 2.0 * u * (fabs(w0) + fabs(wr) + fabs(w1));
    trk->em[e] = em1 + fabs(ms - m1);
    trk->ev[e] = ev1 + fabs(vs - v1);
    trk->bw[e] = b;
}

/* Bound bookkeeping of one flushed element (delta skipped steps, moments
 * decayed by Mfd = b1^delta, Vfd = b2^delta, then stored as ms, vs). */
static void track_flush(const orc_track *trk, int64_t e, int64_t dl, double Wn, double Mfd, double Vfd,
                        double lr, double eps, double rb, double b2, double w0, double w1, double mk, double vk,
                        double ms, double vs)
{
    const double u = ORC_U32, cs = trk->cs;
    double em0 = trk->em[e], ev0 = trk->ev[e];
    trk->bw[e] += restore_dev(mk, vk, em0, ev0, eps, rb, cs, Wn, lr, dl, b2) + 4.0 * u * fabs(w0 - w1) +
                  2.0 * u * (fabs(w0) + fabs(w1));
    double m1 = Mfd * mk, v1 = Vfd * vk;
    trk->em[e] = Mfd * em0 * (1.0 + 2.0 * u) + 2.0 * u * fabs(m1) + fabs(ms - (double)(float)m1);
    trk->ev[e] = Vfd * ev0 * (1.0 + 2.0 * u) + 2.0 * u * fabs(v1) + fabs(vs - (double)(float)v1);
}

/* trk (optional): stochastic-rounding keys and the error-bound bookkeeping. */
void orc_deferred_rows_f32(int dim, float *w, void *m, void *v, int state, int64_t ld, int64_t n_rows,
                           const uint32_t *rows, const int64_t *d, const float *g, int64_t g_ld,
                           const float *lr, double b1, double b2, double eps,
                           const float *Wf, const float *Mf, const float *Vf, float ss, float bc, float rb,
                           uint64_t seed, int64_t t, int col0, const orc_track *trk)
{
    const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2), eps32 = (float)eps;
    const int track = trk && trk->bw;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dj = d[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float w0 = w[e], wk = w0, mk = mom_load(m, state, e), vk = mom_load(v, state, e);
            float gk = g ? g[j * g_ld + k] : 0.0f;
            if (dj > 0) wk = restore32(wk, mk, vk, Wf[dj], lr[k], eps32, rb);
            float m1 = Mf[dj] * mk + omb1 * gk;
            float v1 = Vf[dj] * vk + (omb2 * gk) * gk;
            float st = lr[k] * ss;
            float upd = adam_step32(m1, v1, st, bc, eps32, rb);
            w[e] = wk - upd;
            uint64_t r = state ? sr_bits(seed, t, sr_key(trk, id), col0 + k) : 0;
            mom_store(m, state, e, m1, (uint32_t)(r & 0xffffu));
            mom_store(v, state, e, v1, (uint32_t)((r >> 16) & 0xffffu));
            if (track)
                track_update(trk, e, dj, Wf[dj], Mf[dj], Vf[dj], omb1, omb2, gk, lr[k], ss, bc, eps, rb, b2, w0,
                             wk, w[e], upd, mk, vk, m1, v1, mom_load(m, state, e), mom_load(v, state, e));
        }
    }
}

/* O3/O4 restore-only: out[j][:] = current FP32 value of row rows[j]. */
void orc_restore_rows_f32(int dim, const float *w, const void *m, const void *v, int state, int64_t ld,
                          int64_t n_rows, const uint32_t *rows, const int64_t *d,
                          const float *lr, double eps, const float *Wf, float rb, float *out)
{
    const float eps32 = (float)eps;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float wk = w[e];
            if (d[j] > 0)
                wk = restore32(wk, mom_load(m, state, e), mom_load(v, state, e), Wf[d[j]], lr[k], eps32, rb);
            out[j * dim + k] = wk;
        }
    }
}

/* O3/O4 flush after update t: rows skipped delta[j] >= 1 steps; Wf_next is the
 * table of step t+1.  Quantised moments round with the stream of step t. */
void orc_flush_rows_f32(int dim, float *w, void *m, void *v, int state, int64_t ld, int64_t n_rows,
                        const uint32_t *rows, const int64_t *delta, const float *lr, double eps,
                        const float *Wf_next, const float *Mf, const float *Vf, float rb,
                        uint64_t seed, int64_t t, int col0, double b2, const orc_track *trk)
{
    const float eps32 = (float)eps;
    const int track = trk && trk->bw;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dl = delta[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float w0 = w[e], mk = mom_load(m, state, e), vk = mom_load(v, state, e);
            w[e] = restore32(w0, mk, vk, Wf_next[dl], lr[k], eps32, rb);
            uint64_t r = state ? sr_bits(seed, t, sr_key(trk, id), col0 + k) : 0;
            mom_store(m, state, e, Mf[dl - 1] * mk, (uint32_t)(r & 0xffffu));
            mom_store(v, state, e, Vf[dl - 1] * vk, (uint32_t)((r >> 16) & 0xffffu));
            if (track)
                track_flush(trk, e, dl, Wf_next[dl], Mf[dl - 1], Vf[dl - 1], lr[k], eps, rb, b2, w0, w[e], mk, vk,
                            mom_load(m, state, e), mom_load(v, state, e));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Model O4 with FP8 moments: OCP E4M3FN codes (bias 7, largest finite 448, no
 * Inf, NaN = S.1111.111) times one FP32 power-of-two scale per block of 128
 * rows, per group and per moment.  A scale of 0 marks a block that has never
 * held a nonzero moment. */
#define FP8_BLOCK 128

static float e4m3_decode(uint8_t b)
{
    int e = (b >> 3) & 0xf, m = b & 7;
    if (e == 15 && m == 7) return NAN;
    float a = e == 0 ? ldexpf((float)m, -9) : ldexpf((float)(8 + m), e - 10);
    return (b & 0x80) ? -a : a;
}

/* Stochastic rounding of y to E4M3 with 16 random bits: magnitudes above 448
 * saturate; within a binade of quantum q the value k*q + f*q rounds up with
 * probability f (f*65536 > r16). */
uint8_t orc_e4m3_sr(float y, uint32_t r16)
{
    if (isnan(y)) return 0x7f;
    uint8_t sign = signbit(y) ? 0x80 : 0;
    float a = fabsf(y);
    if (a > 448.0f) a = 448.0f;
    int e;
    if (a < 0.015625f) {
        e = -6;                          /* subnormal range: quantum 2^-9 */
    } else {
        uint32_t u;
        memcpy(&u, &a, 4);
        e = (int)((u >> 23) & 0xff) - 127;
    }
    float quantum = ldexpf(1.0f, e - 3);
    float yq = a / quantum;
    float k = floorf(yq);
    float f = yq - k;
    if (f * 65536.0f > (float)r16) k = k + 1.0f;
    float val = k * quantum;
    if (val == 0.0f) return sign;
    if (val < 0.015625f) return (uint8_t)(sign | (uint8_t)(val / ldexpf(1.0f, -9)));
    uint32_t u;
    memcpy(&u, &val, 4);
    int ev = (int)((u >> 23) & 0xff) - 127;
    int mant = (int)(val / ldexpf(1.0f, ev) * 8.0f) - 8;
    return (uint8_t)(sign | (uint8_t)((ev + 7) << 3) | (uint8_t)mant);
}

/* Smallest power of two p with amax / p <= 448 (amax / 448 rounded once). */
float orc_fp8_scale_for(float amax)
{
    if (!(amax > 0.0f) || !(amax < INFINITY)) return 0.0f;
    float r = amax / 448.0f;
    int e;
    float fr = frexpf(r, &e);            /* r = fr * 2^e, fr in [0.5, 1) */
    return fr == 0.5f ? ldexpf(1.0f, e - 1) : ldexpf(1.0f, e);
}

static float fp8_load(const uint8_t *q, const float *s, int64_t row, int64_t e)
{
    return e4m3_decode(q[e]) * s[row / FP8_BLOCK];
}

/* The second moment is stored as its square root (halving its dynamic range
 * in the 4-bit exponent); v = (code * scale)^2. */
static float fp8_load_v(const uint8_t *q, const float *s, int64_t row, int64_t e)
{
    float r = e4m3_decode(q[e]) * s[row / FP8_BLOCK];
    return r * r;
}

/* One update step of the rows rows[j] of a group with FP8 moments:
 *  1. new moments of every update row in FP32, per-block max |m'|, |v'|;
 *  2. every block whose max no longer fits (|x| > 448 s) gets the new scale
 *     and all its rows are re-encoded (random column col0+k+64);
 *  3. the update proper from the re-encoded moments: restore, Adam step,
 *     moments encoded with the final scales (random column col0+k). */
void orc_deferred_rows_fp8(int dim, float *w, uint8_t *mq, uint8_t *vq, float *ms, float *vs, int64_t ld,
                           int64_t n, int64_t n_rows, const uint32_t *rows, const int64_t *d, const float *g,
                           int64_t g_ld, const float *lr, double b1, double b2, double eps, const float *Wf,
                           const float *Mf, const float *Vf, float ss, float bc, float rb, uint64_t seed,
                           int64_t t, int col0, const orc_track *trk)
{
    const int track = trk && trk->bw;
    const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2), eps32 = (float)eps;
    const int64_t nb = (n + FP8_BLOCK - 1) / FP8_BLOCK;
    float *amax_m = (float *)calloc((size_t)nb, sizeof(float));
    float *amax_v = (float *)calloc((size_t)nb, sizeof(float));
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j], dj = d[j], b = id / FP8_BLOCK;
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float gk = g ? g[j * g_ld + k] : 0.0f;
            float m1 = Mf[dj] * fp8_load(mq, ms, id, e) + omb1 * gk;
            float v1 = Vf[dj] * fp8_load_v(vq, vs, id, e) + (omb2 * gk) * gk;
            float r1 = sqrtf(v1);
            if (fabsf(m1) > 448.0f * ms[b] && fabsf(m1) > amax_m[b]) amax_m[b] = fabsf(m1);
            if (r1 > 448.0f * vs[b] && r1 > amax_v[b]) amax_v[b] = r1;
        }
    }
    for (int64_t b = 0; b < nb; ++b) {
        for (int mv = 0; mv < 2; ++mv) {
            float amax = mv ? amax_v[b] : amax_m[b];
            float *sc = mv ? vs : ms;
            uint8_t *q = mv ? vq : mq;
            if (!(amax > 0.0f)) continue;
            float snew = orc_fp8_scale_for(amax);
            if (!(snew > sc[b])) continue;
            for (int64_t id = b * FP8_BLOCK; id < (b + 1) * FP8_BLOCK && id < n; ++id)
                for (int k = 0; k < dim; ++k) {
                    int64_t e = id * ld + k;
                    float x = e4m3_decode(q[e]) * sc[b];
                    uint64_t r = sr_bits(seed, t, sr_key(trk, id), col0 + k + 64);
                    q[e] = orc_e4m3_sr(x / snew, (uint32_t)((mv ? r >> 16 : r) & 0xffffu));
                    if (track) {
                        /* the re-encode moves the decoded moment (v = code^2 scale^2) */
                        double xo = x, xn = (double)e4m3_decode(q[e]) * snew;
                        if (mv) trk->ev[e] += fabs(xn * xn - xo * xo);
                        else trk->em[e] += fabs(xn - xo);
                    }
                }
            sc[b] = snew;
        }
    }
    free(amax_m);
    free(amax_v);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j], dj = d[j], b = id / FP8_BLOCK;
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float w0 = w[e], wk = w0, mk = fp8_load(mq, ms, id, e), vk = fp8_load_v(vq, vs, id, e);
            float gk = g ? g[j * g_ld + k] : 0.0f;
            if (dj > 0) wk = restore32(wk, mk, vk, Wf[dj], lr[k], eps32, rb);
            float m1 = Mf[dj] * mk + omb1 * gk;
            float v1 = Vf[dj] * vk + (omb2 * gk) * gk;
            float st = lr[k] * ss;
            float upd = adam_step32(m1, v1, st, bc, eps32, rb);
            w[e] = wk - upd;
            uint64_t r = sr_bits(seed, t, sr_key(trk, id), col0 + k);
            mq[e] = ms[b] > 0.0f ? orc_e4m3_sr(m1 / ms[b], (uint32_t)(r & 0xffffu)) : 0;
            vq[e] = vs[b] > 0.0f ? orc_e4m3_sr(sqrtf(v1) / vs[b], (uint32_t)((r >> 16) & 0xffffu)) : 0;
            if (track) {
                double rs = (double)e4m3_decode(vq[e]) * vs[b];
                track_update(trk, e, dj, Wf[dj], Mf[dj], Vf[dj], omb1, omb2, gk, lr[k], ss, bc, eps, rb, b2, w0,
                             wk, w[e], upd, mk, vk, m1, v1, (double)e4m3_decode(mq[e]) * ms[b], rs * rs);
            }
        }
    }
}

void orc_restore_rows_fp8(int dim, const float *w, const uint8_t *mq, const uint8_t *vq, const float *ms,
                          const float *vs, int64_t ld, int64_t n_rows, const uint32_t *rows, const int64_t *d,
                          const float *lr, double eps, const float *Wf, float rb, float *out)
{
    const float eps32 = (float)eps;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float wk = w[e];
            if (d[j] > 0)
                wk = restore32(wk, fp8_load(mq, ms, id, e), fp8_load_v(vq, vs, id, e), Wf[d[j]], lr[k], eps32, rb);
            out[j * dim + k] = wk;
        }
    }
}

void orc_flush_rows_fp8(int dim, float *w, uint8_t *mq, uint8_t *vq, const float *ms, const float *vs,
                        int64_t ld, int64_t n_rows, const uint32_t *rows, const int64_t *delta, const float *lr,
                        double eps, const float *Wf_next, const float *Mf, const float *Vf, float rb, uint64_t seed,
                        int64_t t, int col0, double b2, const orc_track *trk)
{
    const float eps32 = (float)eps;
    const int track = trk && trk->bw;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j], dl = delta[j], b = id / FP8_BLOCK;
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float w0 = w[e], mk = fp8_load(mq, ms, id, e), vk = fp8_load_v(vq, vs, id, e);
            w[e] = restore32(w0, mk, vk, Wf_next[dl], lr[k], eps32, rb);
            uint64_t r = sr_bits(seed, t, sr_key(trk, id), col0 + k);
            mq[e] = ms[b] > 0.0f ? orc_e4m3_sr(Mf[dl - 1] * mk / ms[b], (uint32_t)(r & 0xffffu)) : 0;
            vq[e] = vs[b] > 0.0f ? orc_e4m3_sr(sqrtf(Vf[dl - 1] * vk) / vs[b], (uint32_t)((r >> 16) & 0xffffu)) : 0;
            if (track) {
                double rs = (double)e4m3_decode(vq[e]) * vs[b];
                track_flush(trk, e, dl, Wf_next[dl], Mf[dl - 1], Vf[dl - 1], lr[k], eps, rb, b2, w0, w[e], mk, vk,
                            (double)e4m3_decode(mq[e]) * ms[b], rs * rs);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* SGD with momentum, the momentum-optimizer extension named in Sec. 4.3
 * (heavy ball, no dampening, no Nesterov: buf = mu buf + g; w -= lr s_t buf,
 * with s_t an optional per-step rate multiplier).  With g = 0 for d skipped
 * steps the buffer decays as mu^j, so the skipped steps move w by
 * lr buf Ws[d], Ws[d] = sum_{i=1..d} s_{t-i} mu^(d+1-i); this is exact (no eps
 * term to factor out, unlike Adam's Eq. 3). */

/* Dense definition: every row steps every update, g = 0 unless listed. */
void orc_sgdm_dense_sparse_grad_f64(int64_t n, int dim, double *w, double *m, int64_t n_ids,
                                    const uint32_t *ids, const float *g, const double *lr, double mu,
                                    double s_t)
{
    double *gd = (double *)calloc((size_t)n * dim, sizeof(double));
    for (int64_t j = 0; j < n_ids; ++j)
        for (int k = 0; k < dim; ++k) gd[(int64_t)ids[j] * dim + k] = (double)g[j * dim + k];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            int64_t e = i * dim + k;
            m[e] = mu * m[e] + gd[e];
            w[e] = w[e] - (lr[k] * s_t) * m[e];
        }
    free(gd);
}

/* Tables of update t in FP64.  With g = 0 the momentum buffer decays as mu^j,
 * so the skipped steps k = t-d .. t-1 of a row last updated at s0 = t-1-d
 * move w by lr buf Ws[d] with Ws[d] = sum_{k=s0+1}^{t-1} s_k mu^(k-s0)
 * (pow for the powers); Mf[d] = mu^(d+1) is the buffer's decay to step t. */
void orc_lut_sgdm_f64(double mu, int64_t t, int dmax, const double *sched, double *Ws, double *Mf)
{
    for (int d = 0; d <= dmax; ++d) {
        const int64_t s0 = t - 1 - d;
        double sum = 0.0;
        for (int64_t k = s0 + 1; k <= t - 1; ++k) sum += (sched ? sched[k] : 1.0) * pow(mu, (double)(k - s0));
        Ws[d] = sum;
        Mf[d] = pow(mu, (double)(d + 1));
    }
}

/* FP32 tables of the implementation spec: R[j] = mu^(j+1) by repeated
 * multiplication, Ws[d] summed over the skipped steps in time order from 0,
 * (((0 + R[0] s_{t-d}) + R[1] s_{t-d+1}) + ...) + R[d-1] s_{t-1}, Mf[d] =
 * R[d], each rounded once; and the step multiplier s_t. */
void orc_lut_sgdm_spec(double mu, int64_t t, int dmax, const double *sched, float *Wf, float *Mf, float *ss)
{
    double *R = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double p = 1.0;
    for (int d = 0; d <= dmax; ++d) {
        p = p * mu;
        R[d] = p;
        Mf[d] = (float)p;
    }
    for (int d = 0; d <= dmax; ++d) {
        double W = 0.0;
        for (int j = 0; j < d; ++j) W = W + R[j] * (sched ? sched[t - d + j] : 1.0);
        Wf[d] = (float)W;
    }
    *ss = sched ? (float)sched[t] : 1.0f;
    free(R);
}

/* Deferred update in FP64, the paper's order: catch up the d skipped steps,
 * then take step t with the row's gradient. */
void orc_sgdm_deferred_rows_f64(int dim, double *w, double *m, int64_t n_rows, const uint32_t *rows,
                                const int64_t *d, const double *g, const double *lr, double s_t,
                                const double *Ws, const double *Mf)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * dim + k;
            double wk = w[e] - (lr[k] * Ws[d[j]]) * m[e];
            double m1 = Mf[d[j]] * m[e] + g[j * dim + k];
            w[e] = wk - (lr[k] * s_t) * m1;
            m[e] = m1;
        }
    }
}

/* FP64 flush: delta skipped steps with the tables of update t+1. */
void orc_sgdm_flush_rows_f64(int dim, double *w, double *m, int64_t n_rows, const uint32_t *rows,
                             const int64_t *delta, const double *lr, const double *Ws_next, double mu)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * dim + k;
            w[e] = w[e] - (lr[k] * Ws_next[delta[j]]) * m[e];
            m[e] = m[e] * pow(mu, (double)delta[j]);
        }
    }
}

/* FP32 model with the spec's operation order: restore w - (Wf[d] lr) buf;
 * buf1 = Mf[d] buf + g; w - (lr ss) buf1.  buf is stored FP32 or BF16 (stochastic
 * rounding with bits 0..15 of the element's random word). */
void orc_sgdm_rows_f32(int dim, float *w, void *m, int state, int64_t ld, int64_t n_rows, const uint32_t *rows,
                       const int64_t *d, const float *g, int64_t g_ld, const float *lr, const float *Wf,
                       const float *Mf, float ss, uint64_t seed, int64_t t, int col0)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dj = d[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float wk = w[e], mk = mom_load(m, state, e);
            float gk = g ? g[j * g_ld + k] : 0.0f;
            if (dj > 0) wk = wk - (Wf[dj] * lr[k]) * mk;
            float m1 = Mf[dj] * mk + gk;
            w[e] = wk - (lr[k] * ss) * m1;
            uint64_t r = state ? sr_bits(seed, t, id, col0 + k) : 0;
            mom_store(m, state, e, m1, (uint32_t)(r & 0xffffu));
        }
    }
}

/* FP32 restore-only (gather and the cull's current geometry). */
void orc_sgdm_restore_rows_f32(int dim, const float *w, const void *m, int state, int64_t ld, int64_t n_rows,
                               const uint32_t *rows, const int64_t *d, const float *lr, const float *Wf, float *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float wk = w[e];
            if (d[j] > 0) wk = wk - (Wf[d[j]] * lr[k]) * mom_load(m, state, e);
            out[j * dim + k] = wk;
        }
    }
}

/* FP32 flush after update t (tables of t+1). */
void orc_sgdm_flush_rows_f32(int dim, float *w, void *m, int state, int64_t ld, int64_t n_rows,
                             const uint32_t *rows, const int64_t *delta, const float *lr, const float *Wf_next,
                             const float *Mf, uint64_t seed, int64_t t, int col0)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dl = delta[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float mk = mom_load(m, state, e);
            w[e] = w[e] - (Wf_next[dl] * lr[k]) * mk;
            uint64_t r = state ? sr_bits(seed, t, id, col0 + k) : 0;
            mom_store(m, state, e, Mf[dl - 1] * mk, (uint32_t)(r & 0xffffu));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* AdamW (decoupled weight decay; the other optimizer Sec. 4.3 names), in the
 * common form where step k first scales w by q_k = 1 - lr s_k lambda and then
 * applies the Adam update.  With g = 0 for d skipped steps the catch-up is
 *   w_cur = P_d w - lr (m / (sqrt(v) + eps)) Wl[d]
 *   P_d   = prod_{i=1..d} q_{t-i}
 *   Wl[d] = sum_{i=1..d} (prod_{j=1..i-1} q_{t-j}) r^(d-i) s_{t-i} c(t-i)
 * (r = b1/sqrt(b2), c(k) the unit-rate coefficient of Eq. 3), i.e. Eq. 3 with
 * every skipped update also shrunk by the decays that follow it.  Built by
 *   Wl[d] = r Wl[d-1] + P_{d-1} s_{t-d} c(t-d),   P_d = P_{d-1} q_{t-d}.
 * The tables depend on the column's rate through q. */

/* Dense definition (rates lr[] already include the step's multiplier). */
void orc_adamw_dense_sparse_grad_f64(int64_t n, int dim, double *w, double *m, double *v, int64_t n_ids,
                                     const uint32_t *ids, const float *g_rows, const double *lr, double b1,
                                     double b2, double eps, double lam, int64_t t)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) w[i * dim + k] = w[i * dim + k] * (1.0 - lr[k] * lam);
    orc_adam_dense_sparse_grad_f64(n, dim, w, m, v, n_ids, ids, g_rows, lr, b1, b2, eps, t);
}

/* FP64 tables of update t for one column rate lr.  Step k first scales w by
 * q_k = 1 - lr s_k lambda, then takes its Adam step; with g = 0 the skipped
 * steps k = t-d .. t-1 of a row last updated at s0 = t-1-d move it to
 * P[d] w - lr Wl[d] m/(sqrt(v)+eps) (eps moved out as in Eq. 3), where every
 * skipped step's Adam term is shrunk by the decays of the later skipped steps:
 *   Wl[d] = sum_{k=s0+1}^{t-1} (prod_{j=k+1}^{t-1} q_j) s_k (b1/sqrt(b2))^(k-s0)
 *                               sqrt(1-b2^k)/(1-b1^k),
 *   P[d]  = prod_{k=s0+1}^{t-1} q_k                      (pow for the powers) */
void orc_lut_adamw_f64(double b1, double b2, double lam, double lr, int64_t t, int dmax, const double *sched,
                       double *Wl, double *P)
{
    for (int d = 0; d <= dmax; ++d) {
        const int64_t s0 = t - 1 - d;
        double sum = 0.0, prod = 1.0;
        for (int64_t k = s0 + 1; k <= t - 1; ++k) {
            double later = 1.0;
            for (int64_t j = k + 1; j <= t - 1; ++j) later *= 1.0 - lr * (sched ? sched[j] : 1.0) * lam;
            const double s = sched ? sched[k] : 1.0;
            sum += later * s * pow(b1 / sqrt(b2), (double)(k - s0)) * sqrt(1.0 - pow(b2, (double)k)) /
                   (1.0 - pow(b1, (double)k));
            prod *= 1.0 - lr * s * lam;
        }
        Wl[d] = sum;
        P[d] = prod;
    }
}

/* FP32 tables of the implementation spec: C[k] = s_k b1/(sqrt(b2/(1-P2[k]))
 * (1-P1[k])) with repeated-multiplication powers, R[j] = (b1/sqrt(b2))^j,
 * q_k = 1 - lr s_k lambda; over the skipped steps k = t-d+j in time order,
 * from Wl = 0, P = 1:  Wl = q_k Wl + R[j] C[k],  P = q_k P  (each product and
 * sum one binary64 operation, rounded once to FP32); and q_t. */
void orc_lut_adamw_spec(double b1, double b2, double lam, double lr, int64_t t, int dmax, const double *sched,
                        float *Wf, float *Pf, float *qt)
{
    double P1 = 1.0, P2 = 1.0;
    double *C = (double *)calloc((size_t)t + 1, sizeof(double));
    double *R = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    for (int64_t k = 1; k <= t; ++k) {
        P1 = P1 * b1;
        P2 = P2 * b2;
        C[k] = b1 / (sqrt(b2 / (1.0 - P2)) * (1.0 - P1));
        if (sched) C[k] = sched[k] * C[k];
    }
    const double r = b1 / sqrt(b2);
    R[0] = 1.0;
    for (int j = 1; j <= dmax; ++j) R[j] = R[j - 1] * r;
    for (int d = 0; d <= dmax; ++d) {
        double W = 0.0, P = 1.0;
        for (int j = 0; j < d; ++j) {
            const int64_t k = t - d + j;
            const double q = 1.0 - lr * (sched ? sched[k] : 1.0) * lam;
            W = q * W + R[j] * C[k];
            P = q * P;
        }
        Wf[d] = (float)W;
        Pf[d] = (float)P;
    }
    *qt = (float)(1.0 - lr * (sched ? sched[t] : 1.0) * lam);
    free(C);
    free(R);
}

/* Model O2 with decoupled weight decay (AdamW): as orc_deferred_rows_f64,
 * with the restore of d skipped steps w <- P[d] w - lr Wl[d] m / (sqrt(v) +
 * eps) (per column tables [dim][ldt]) and the step of update t taken on the
 * decayed value: w <- (1 - lr s_t lam) w - (lr s_t / (1-b1^t)) m / (sqrt(v) /
 * sqrt(1-b2^t) + eps), m and v the new moments. */
void orc_adamw_deferred_rows_f64(int dim, double *w, double *m, double *v, int64_t n_rows, const uint32_t *rows,
                                 const int64_t *d, const double *g, const double *lr, double b1, double b2,
                                 double eps, int64_t t, double s_t, double lam, const double *Wl, const double *P,
                                 int64_t ldt, const double *m_dec, const double *v_dec)
{
    const double corr2 = sqrt(1.0 - pow(b2, (double)t));
    const double corr1 = 1.0 - pow(b1, (double)t);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        const int64_t id = rows[j];
        const int64_t dj = d[j];
        for (int k = 0; k < dim; ++k) {
            const int64_t e = id * dim + k;
            const double gk = g ? g[j * dim + k] : 0.0;
            double wk = w[e];
            if (dj > 0) wk = P[k * ldt + dj] * wk - (Wl[k * ldt + dj] * lr[k] * m[e]) / (sqrt(v[e]) + eps);
            const double m1 = m_dec[dj] * m[e] + (1.0 - b1) * gk;
            const double v1 = v_dec[dj] * v[e] + (1.0 - b2) * gk * gk;
            const double rate = lr[k] * s_t;
            wk = wk * (1.0 - rate * lam);
            m[e] = m1;
            v[e] = v1;
            w[e] = wk - (rate / corr1) * m1 / (sqrt(v1) / corr2 + eps);
        }
    }
}

/* FP64 restore (read-only) and flush (tables of t+1, moments decay by b^delta). */
void orc_adamw_restore_rows_f64(int dim, const double *w, const double *m, const double *v, int64_t n_rows,
                                const uint32_t *rows, const int64_t *d, const double *lr, double eps,
                                const double *Wl, const double *P, int64_t ldt, double *out)
{
    for (int64_t j = 0; j < n_rows; ++j)
        for (int k = 0; k < dim; ++k) {
            int64_t e = (int64_t)rows[j] * dim + k;
            double wk = w[e];
            if (d[j] > 0) wk = P[k * ldt + d[j]] * wk - (Wl[k * ldt + d[j]] * lr[k] * m[e]) / (sqrt(v[e]) + eps);
            out[j * dim + k] = wk;
        }
}

void orc_adamw_flush_rows_f64(int dim, double *w, double *m, double *v, int64_t n_rows, const uint32_t *rows,
                              const int64_t *delta, const double *lr, double b1, double b2, double eps,
                              const double *Wl_next, const double *P_next, int64_t ldt)
{
    for (int64_t j = 0; j < n_rows; ++j)
        for (int k = 0; k < dim; ++k) {
            int64_t e = (int64_t)rows[j] * dim + k, dl = delta[j];
            w[e] = P_next[k * ldt + dl] * w[e] - (Wl_next[k * ldt + dl] * lr[k] * m[e]) / (sqrt(v[e]) + eps);
            m[e] *= pow(b1, (double)dl);
            v[e] *= pow(b2, (double)dl);
        }
}

/* FP32 model, the spec's order: restore (Pf w) - (Wf lr) q with q the clamped
 * m/(sqrt(v)+eps); step qf w - adam_step.  Tables per column [dim][ldt]. */
static float restore32_w(float w, float m, float v, float wd, float pd, float lr, float eps, float rb)
{
    float den = sqrtf(v) + eps;
    float q = m / den;
    if (q > rb) q = rb;
    else if (q < -rb) q = -rb;
    float a = pd * w;
    float b = (wd * lr) * q;
    return a - b;
}

void orc_adamw_rows_f32(int dim, float *w, void *m, void *v, int state, int64_t ld, int64_t n_rows,
                        const uint32_t *rows, const int64_t *d, const float *g, int64_t g_ld, const float *lr,
                        double b1, double b2, double eps, const float *Wf, const float *Pf, int64_t ldt,
                        const float *qf, const float *Mf, const float *Vf, float ss, float bc, float rb,
                        uint64_t seed, int64_t t, int col0)
{
    const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2), eps32 = (float)eps;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dj = d[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float wk = w[e], mk = mom_load(m, state, e), vk = mom_load(v, state, e);
            float gk = g ? g[j * g_ld + k] : 0.0f;
            if (dj > 0) wk = restore32_w(wk, mk, vk, Wf[k * ldt + dj], Pf[k * ldt + dj], lr[k], eps32, rb);
            float m1 = Mf[dj] * mk + omb1 * gk;
            float v1 = Vf[dj] * vk + (omb2 * gk) * gk;
            float st = lr[k] * ss;
            float wq = qf[k] * wk;
            w[e] = wq - adam_step32(m1, v1, st, bc, eps32, rb);
            uint64_t r = state ? sr_bits(seed, t, id, col0 + k) : 0;
            mom_store(m, state, e, m1, (uint32_t)(r & 0xffffu));
            mom_store(v, state, e, v1, (uint32_t)((r >> 16) & 0xffffu));
        }
    }
}

void orc_adamw_restore_rows_f32(int dim, const float *w, const void *m, const void *v, int state, int64_t ld,
                                int64_t n_rows, const uint32_t *rows, const int64_t *d, const float *lr, double eps,
                                const float *Wf, const float *Pf, int64_t ldt, float rb, float *out)
{
    const float eps32 = (float)eps;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float wk = w[e];
            if (d[j] > 0)
                wk = restore32_w(wk, mom_load(m, state, e), mom_load(v, state, e), Wf[k * ldt + d[j]],
                                 Pf[k * ldt + d[j]], lr[k], eps32, rb);
            out[j * dim + k] = wk;
        }
    }
}

void orc_adamw_flush_rows_f32(int dim, float *w, void *m, void *v, int state, int64_t ld, int64_t n_rows,
                              const uint32_t *rows, const int64_t *delta, const float *lr, double eps,
                              const float *Wf_next, const float *Pf_next, int64_t ldt, const float *Mf,
                              const float *Vf, float rb, uint64_t seed, int64_t t, int col0)
{
    const float eps32 = (float)eps;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_rows; ++j) {
        int64_t id = rows[j];
        int64_t dl = delta[j];
        for (int k = 0; k < dim; ++k) {
            int64_t e = id * ld + k;
            float mk = mom_load(m, state, e), vk = mom_load(v, state, e);
            w[e] = restore32_w(w[e], mk, vk, Wf_next[k * ldt + dl], Pf_next[k * ldt + dl], lr[k], eps32, rb);
            uint64_t r = state ? sr_bits(seed, t, id, col0 + k) : 0;
            mom_store(m, state, e, Mf[dl - 1] * mk, (uint32_t)(r & 0xffffu));
            mom_store(v, state, e, Vf[dl - 1] * vk, (uint32_t)((r >> 16) & 0xffffu));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Densification (Sec. 2.4 step 7: Gaussians with large accumulated gradients
 * are cloned or split, low-opacity ones pruned), with the procedure of 3D
 * Gaussian Splatting the paper builds on.  Per row i on current FP32 values:
 *   g      = accum/denom (0 when denom = 0);  grad = g >= grad_thr
 *   smax   = largest of the three log-scales
 *   clone  = grad and smax <= log_dense;   split = grad and smax > log_dense
 *   low    = opacity logit < logit_min;    big = big_on and smax > log_big
 *   screen = radii given, max_screen > 0 and radii > max_screen (originals only)
 *   kept original: not split, not low, not big, not screen
 *   kept clone (a copy):   clone, not low, not big
 *   kept children (two):   split, not low, not big on the child's scales
 * A child j of row i has scales s - log_split and position
 *   mu + Q (exp(s) * z),  z_a = normal-approximation draw of (seed, i, j, a),
 * Q the rotation of the normalised quaternion (same expressions as the cull).
 * Output order: kept originals, kept clones, kept children (parent order,
 * child 0 before child 1), as 3DGS's append-then-prune leaves them.
 * Returns the number of output rows (capacity permitting, rows past cap are
 * only counted); counts[3] = originals, clones, children. */
static float split_normal(uint64_t seed, int64_t row, int child, int axis)
{
    uint64_t h = sm_at(sm_at(sm_at(seed, (uint64_t)row), (uint64_t)child), (uint64_t)axis);
    uint64_t u = (h & 0xffffull) + ((h >> 16) & 0xffffull) + ((h >> 32) & 0xffffull) + ((h >> 48) & 0xffffull);
    const double inv_sd = 1.0 / sqrt(4.0 * (65536.0 * 65536.0 - 1.0) / 12.0);
    return (float)(((double)u - 131070.0) * inv_sd);
}

int64_t orc_densify(int64_t n, int adim, const float *geo, const float *app, const float *accum,
                    const float *denom, const float *radii, float grad_thr, float log_dense, int big_on,
                    float log_big, float logit_min, float max_screen, float log_split, uint64_t seed,
                    int64_t cap, float *out_geo, float *out_app, int64_t *src, uint8_t *kind, int64_t *counts)
{
    uint8_t *code = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t nk = 0, nc = 0, ns = 0;
    for (int64_t i = 0; i < n; ++i) {
        const float *g = geo + i * 10;
        float gr = denom[i] > 0.0f ? accum[i] / denom[i] : 0.0f;
        int grad = gr >= grad_thr;
        float smax = g[3];
        if (g[4] > smax) smax = g[4];
        if (g[5] > smax) smax = g[5];
        int clone = grad && (smax <= log_dense);
        int split = grad && (smax > log_dense);
        int low = app[i * adim] < logit_min;  /* opacity logit: appearance column 0 */
        int big = big_on && (smax > log_big);
        int screen = radii && max_screen > 0.0f && radii[i] > max_screen;
        float cmax = smax - log_split;
        int cbig = big_on && (cmax > log_big);
        uint8_t c = 0;
        if (!split && !low && !big && !screen) { c |= 1; ++nk; }
        if (clone && !low && !big) { c |= 2; ++nc; }
        if (split && !low && !cbig) { c |= 4; ns += 2; }
        code[i] = c;
    }
    counts[0] = nk; counts[1] = nc; counts[2] = ns;
    int64_t pos[3] = {0, nk, nk + nc};
    for (int pass = 0; pass < 3; ++pass) {
        for (int64_t i = 0; i < n; ++i) {
            if (!(code[i] & (1 << pass))) continue;
            const float *g = geo + i * 10;
            int nchild = pass == 2 ? 2 : 1;
            for (int j = 0; j < nchild; ++j) {
                int64_t o = pos[pass]++;
                if (o >= cap) continue;
                float *og = out_geo + o * 10;
                for (int k = 0; k < 10; ++k) og[k] = g[k];
                for (int k = 0; k < adim; ++k) out_app[o * adim + k] = app[i * adim + k];
                src[o] = i;
                kind[o] = (uint8_t)(pass == 2 ? 2 + j : pass);
                if (pass != 2) continue;
                float qw = g[6], qx = g[7], qy = g[8], qz = g[9];
                float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
                float inv = 1.0f / sqrtf(n2);
                qw = qw * inv; qx = qx * inv; qy = qy * inv; qz = qz * inv;
                float Q[9];
                Q[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
                Q[1] = 2.0f * (qx * qy - qw * qz);
                Q[2] = 2.0f * (qx * qz + qw * qy);
                Q[3] = 2.0f * (qx * qy + qw * qz);
                Q[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
                Q[5] = 2.0f * (qy * qz - qw * qx);
                Q[6] = 2.0f * (qx * qz - qw * qy);
                Q[7] = 2.0f * (qy * qz + qw * qx);
                Q[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
                float v[3];
                for (int a = 0; a < 3; ++a) v[a] = orc_exp_gs(g[3 + a]) * split_normal(seed, i, j, a);
                for (int a = 0; a < 3; ++a)
                    og[a] = g[a] + ((Q[3 * a] * v[0] + Q[3 * a + 1] * v[1]) + Q[3 * a + 2] * v[2]);
                for (int a = 0; a < 3; ++a) og[3 + a] = g[3 + a] - log_split;
            }
        }
    }
    free(code);
    return nk + nc + ns;
}

/* Thresholds of the densification criteria, computed in FP64 and rounded
 * once: log(percent_dense extent), log(0.1 extent), logit(min_opacity), log(1.6). */
void orc_densify_thresholds(double percent_dense, double extent, double min_opacity, float *out4)
{
    out4[0] = (float)log(percent_dense * extent);
    out4[1] = (float)log(0.1 * extent);
    out4[2] = (float)log(min_opacity / (1.0 - min_opacity));
    out4[3] = (float)log(1.6);
}
