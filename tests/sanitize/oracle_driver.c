/* Host-sanitizer driver of the oracle (test infrastructure): runs its main
 * routines on small inputs with NaN, infinite and degenerate rows, every
 * moment storage and deferral pattern, under -fsanitize=address,undefined.
 * Exit status 0 = no finding (the sanitizers abort on the first one). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_track {
    const uint32_t *keys;
    double *em, *ev, *bw;
    double cs;
} orc_track;

void orc_cull_v1(int64_t n, const float *geo, const float *cam, uint8_t *keep, float *detail);
int64_t orc_compact(int64_t n, const uint8_t *keep, uint32_t *ids);
void orc_restore_coeff_f64(double b1, double b2, int64_t t, int dmax, const double *sched, double *coef,
                           double *m_dec, double *v_dec);
void orc_deferred_rows_f64(int dim, double *w, double *m, double *v, int64_t n_rows, const uint32_t *rows,
                           const int64_t *d, const double *g, const double *lr, double b1, double b2, double eps,
                           int64_t t, double lr_scale_t, const double *coef, const double *m_dec,
                           const double *v_dec);
void orc_lut_spec(double b1, double b2, int64_t t, int dmax, const double *sched, float *Wf, float *Mf, float *Vf,
                  float *ss, float *bc);
float orc_restore_bound(double b1, double b2);
void orc_deferred_rows_f32(int dim, float *w, void *m, void *v, int state, int64_t ld, int64_t n_rows,
                           const uint32_t *rows, const int64_t *d, const float *g, int64_t g_ld, const float *lr,
                           double b1, double b2, double eps, const float *Wf, const float *Mf, const float *Vf,
                           float ss, float bc, float rb, uint64_t seed, int64_t t, int col0, const orc_track *trk);
void orc_flush_rows_f32(int dim, float *w, void *m, void *v, int state, int64_t ld, int64_t n_rows,
                        const uint32_t *rows, const int64_t *delta, const float *lr, double eps, const float *Wf_next,
                        const float *Mf, const float *Vf, float rb, uint64_t seed, int64_t t, int col0, double b2,
                        const orc_track *trk);
void orc_deferred_rows_fp8(int dim, float *w, uint8_t *mq, uint8_t *vq, float *ms, float *vs, int64_t ld, int64_t n,
                           int64_t n_rows, const uint32_t *rows, const int64_t *d, const float *g, int64_t g_ld,
                           const float *lr, double b1, double b2, double eps, const float *Wf, const float *Mf,
                           const float *Vf, float ss, float bc, float rb, uint64_t seed, int64_t t, int col0,
                           const orc_track *trk);

static uint64_t st = 88172645463325252ull;
static double urand(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) / 9007199254740992.0;
}

int main(void)
{
    const int64_t n = 3000;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-15;
    float *geo = malloc(sizeof(float) * 10 * n);
    for (int64_t i = 0; i < n * 10; ++i) geo[i] = (float)(urand() * 20.0 - 10.0);
    geo[10 * 5 + 2] = NAN;
    geo[10 * 7 + 0] = INFINITY;
    for (int k = 0; k < 10; ++k) geo[10 * 9 + k] = 0.0f;   /* zero quaternion and scale */
    float cam[20] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 30, 1000, 1000, 640, 360, 1280, 720, 0.01f, 1000};
    uint8_t *keep = malloc((size_t)n);
    float *detail = malloc(sizeof(float) * 11 * n);
    uint32_t *ids = malloc(sizeof(uint32_t) * n);
    orc_cull_v1(n, geo, cam, keep, detail);
    int64_t m = orc_compact(n, keep, ids);
    orc_cull_v1(0, geo, cam, keep, NULL);

    /* tables and the FP64 deferred model over 40 steps with random visibility */
    const int T = 40, dim = 59;
    double coef[64], mdec[64], vdec[64], sched[64];
    for (int t = 0; t < 64; ++t) sched[t] = 0.5 + urand();
    float Wf[64], Mf[64], Vf[64], ss, bc;
    const float rb = orc_restore_bound(b1, b2);
    double *w = calloc((size_t)n * dim, sizeof(double)), *mm = calloc((size_t)n * dim, sizeof(double)),
           *vv = calloc((size_t)n * dim, sizeof(double)), *g = malloc(sizeof(double) * n * dim);
    float *w32 = calloc((size_t)n * dim, sizeof(float)), *m32 = calloc((size_t)n * dim, sizeof(float)),
          *v32 = calloc((size_t)n * dim, sizeof(float)), *g32 = malloc(sizeof(float) * n * dim);
    uint16_t *mb = calloc((size_t)n * dim, 2), *vb = calloc((size_t)n * dim, 2);
    uint8_t *mq = calloc((size_t)n * dim, 1), *vq = calloc((size_t)n * dim, 1);
    float *ms = calloc((size_t)(n + 127) / 128, sizeof(float)), *vs = calloc((size_t)(n + 127) / 128, sizeof(float));
    double *em = calloc((size_t)n * dim, sizeof(double)), *ev = calloc((size_t)n * dim, sizeof(double)),
           *bw = calloc((size_t)n * dim, sizeof(double));
    orc_track trk = {NULL, em, ev, bw, 7.27};
    float lr[64];
    double lr64[64];
    for (int k = 0; k < dim; ++k) lr[k] = (float)(lr64[k] = k < 3 ? 1.6e-4 : 5e-3);
    int64_t *last = calloc((size_t)n, sizeof(int64_t)), *d = malloc(sizeof(int64_t) * n);
    uint32_t *rows = malloc(sizeof(uint32_t) * n);
    for (int t = 1; t <= T; ++t) {
        int64_t nr = 0;
        for (int64_t i = 0; i < n; ++i)
            if (urand() < 0.3) {
                rows[nr] = (uint32_t)i;
                d[nr] = t - 1 - last[i];
                ++nr;
            }
        for (int64_t j = 0; j < nr * dim; ++j) g32[j] = (float)(g[j] = (urand() - 0.5) * 2e-3);
        orc_restore_coeff_f64(b1, b2, t, t - 1, sched, coef, mdec, vdec);
        orc_deferred_rows_f64(dim, w, mm, vv, nr, rows, d, g, lr64, b1, b2, eps, t, sched[t], coef, mdec, vdec);
        orc_lut_spec(b1, b2, t, t - 1, sched, Wf, Mf, Vf, &ss, &bc);
        orc_deferred_rows_f32(dim, w32, m32, v32, 0, dim, nr, rows, d, g32, dim, lr, b1, b2, eps, Wf, Mf, Vf, ss, bc,
                              rb, 5, t, 0, &trk);
        orc_deferred_rows_f32(dim, w32, mb, vb, 1, dim, nr, rows, d, g32, dim, lr, b1, b2, eps, Wf, Mf, Vf, ss, bc,
                              rb, 5, t, 0, NULL);
        orc_deferred_rows_fp8(dim, w32, mq, vq, ms, vs, dim, n, nr, rows, d, g32, dim, lr, b1, b2, eps, Wf, Mf, Vf,
                              ss, bc, rb, 5, t, 0, &trk);
        for (int64_t j = 0; j < nr; ++j) last[rows[j]] = t;
    }
    /* flush every row behind */
    int64_t nr = 0;
    for (int64_t i = 0; i < n; ++i)
        if (last[i] < T) {
            rows[nr] = (uint32_t)i;
            d[nr] = T - last[i];
            ++nr;
        }
    orc_lut_spec(b1, b2, T + 1, T, sched, Wf, Mf, Vf, &ss, &bc);
    orc_flush_rows_f32(dim, w32, m32, v32, 0, dim, nr, rows, d, lr, eps, Wf, Mf, Vf, rb, 5, T, 0, b2, &trk);
    printf("oracle driver: %lld visible of %lld, %lld rows flushed\n", (long long)m, (long long)n, (long long)nr);
    free(geo); free(keep); free(detail); free(ids); free(w); free(mm); free(vv); free(g); free(w32); free(m32);
    free(v32); free(g32); free(mb); free(vb); free(mq); free(vq); free(ms); free(vs); free(em); free(ev); free(bw);
    free(last); free(d); free(rows);
    return 0;
}
