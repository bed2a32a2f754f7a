// Host construction of the deferred-update tables (FP64 math, one FP32 rounding).
//
// The paper precomputes three lookup tables per update step (Sec. 4.3.2 and
// its pseudocode): w_scale of Eq. 3 by the recurrence
//     W[0] = 0,   W[d] = (b1/sqrt(b2)) W[d-1] + c(t-d),
//     c(k) = b1 / ( sqrt(b2 / (1 - b2^k)) * (1 - b1^k) )      (unit learning rate)
// and m_scale = b1^(d+1), v_scale = b2^(d+1) of Eq. 2.  Here the tables for
// every step of a run are built once: powers come from repeated
// multiplication (no pow), every operation is one IEEE binary64 operation, and
// each entry is rounded once to FP32, so the values are fully determined by
// (b1, b2, t, d).  An optional learning-rate schedule s[t] (a multiplier of
// every column's rate at update t) enters as s[k] c(k) for the skipped step k
// and as s[t] / (1 - b1^t) in the step size.
#include <cmath>
#include <vector>

#include "gsdp_internal.h"

namespace gsdp {

int build_lut_host(double b1, double b2, int32_t T, int32_t K, const double *sched, float *out, int64_t nfloats)
{
    const LutLayout L = lut_layout(T, K);
    if (nfloats < L.total) return -1;
    const int64_t kmax = T + 2 > L.nMV + 1 ? T + 2 : L.nMV + 1;
    std::vector<double> P1(kmax + 1), P2(kmax + 1), Ck(T + 2, 0.0);
    P1[0] = 1.0;
    P2[0] = 1.0;
    for (int64_t k = 1; k <= kmax; ++k) {
        P1[k] = P1[k - 1] * b1;
        P2[k] = P2[k - 1] * b2;
    }
    const double r = b1 / std::sqrt(b2);
    for (int64_t k = 1; k <= T; ++k) {
        Ck[k] = b1 / (std::sqrt(b2 / (1.0 - P2[k])) * (1.0 - P1[k]));
        // a learning-rate schedule scales the skipped step k by its own rate
        if (sched) Ck[k] = sched[k] * Ck[k];
    }

    for (int64_t i = 0; i < L.total; ++i) out[i] = 0.0f;
    for (int64_t t = 1; t <= T + 1; ++t) {
        float *row = out + lut_w_row(t, K);
        int64_t dm = t - 1;
        if (K > 0 && dm > K) dm = K;
        double W = 0.0;
        row[0] = 0.0f;
        for (int64_t d = 1; d <= dm; ++d) {
            W = r * W + Ck[t - d];
            row[d] = (float)W;
        }
    }
    for (int64_t d = 0; d < L.nMV; ++d) {
        out[L.offM + d] = (float)P1[d + 1];
        out[L.offV + d] = (float)P2[d + 1];
    }
    for (int64_t t = 1; t <= T + 1; ++t) {
        out[L.offSS + t] = sched ? (float)(sched[t] / (1.0 - P1[t])) : (float)(1.0 / (1.0 - P1[t]));
        out[L.offBC + t] = (float)std::sqrt(1.0 - P2[t]);
    }
    return 0;
}

// SGD with momentum mu: with zero gradients the buffer decays as mu^j, so the
// skipped steps move w by lr buf W[d], W[d] = sum_{i=1..d} s[t-i] mu^(d+1-i),
// built as W[d] = mu (W[d-1] + s[t-d]); the first-moment table holds
// mu^(d+1), the step table s[t]; the second-moment and bias tables are 1.
int build_lut_sgdm_host(double mu, int32_t T, int32_t K, const double *sched, float *out, int64_t nfloats)
{
    const LutLayout L = lut_layout(T, K);
    if (nfloats < L.total) return -1;
    for (int64_t i = 0; i < L.total; ++i) out[i] = 0.0f;
    for (int64_t t = 1; t <= T + 1; ++t) {
        float *row = out + lut_w_row(t, K);
        int64_t dm = t - 1;
        if (K > 0 && dm > K) dm = K;
        double W = 0.0;
        row[0] = 0.0f;
        for (int64_t d = 1; d <= dm; ++d) {
            W = mu * (W + (sched ? sched[t - d] : 1.0));
            row[d] = (float)W;
        }
    }
    double p = 1.0;
    for (int64_t d = 0; d < L.nMV; ++d) {
        p = p * mu;
        out[L.offM + d] = (float)p;
        out[L.offV + d] = 1.0f;
    }
    for (int64_t t = 1; t <= T + 1; ++t) {
        out[L.offSS + t] = sched ? (float)sched[t] : 1.0f;
        out[L.offBC + t] = 1.0f;
    }
    return 0;
}

// AdamW: every step k first scales w by q_k = 1 - lr s[k] lambda, so the
// catch-up of d skipped steps is w P[d] - lr (m/(sqrt(v)+eps)) Wl[d] with
//   Wl[d] = r Wl[d-1] + P[d-1] s[t-d] c(t-d),   P[d] = P[d-1] q_{t-d},
// and step t scales by q_t before its Adam update.  The tables depend on the
// column rate through q: one set per decay class (distinct rate).
int build_lut_adamw_host(double b1, double b2, double lam, const float *rates, int nclass, int32_t T, int32_t K,
                         const double *sched, float *out, int64_t nfloats)
{
    const LutLayout L = lut_layout(T, K);
    if (nfloats < adamw_total_floats(T, K, nclass)) return -1;
    if (build_lut_host(b1, b2, T, K, sched, out, L.total) != 0) return -1;
    std::vector<double> P1(T + 2), P2(T + 2), Ck(T + 2, 0.0);
    P1[0] = 1.0;
    P2[0] = 1.0;
    for (int64_t k = 1; k <= T + 1; ++k) {
        P1[k] = P1[k - 1] * b1;
        P2[k] = P2[k - 1] * b2;
    }
    for (int64_t k = 1; k <= T; ++k) {
        Ck[k] = b1 / (std::sqrt(b2 / (1.0 - P2[k])) * (1.0 - P1[k]));
        if (sched) Ck[k] = sched[k] * Ck[k];
    }
    const double r = b1 / std::sqrt(b2);
    for (int c = 0; c < nclass; ++c) {
        const double lr = (double)rates[c];
        float *base = out + L.total + c * adamw_class_floats(T, K);
        float *Wl = base, *P = base + L.nW, *q = base + 2 * L.nW;
        for (int64_t i = 0; i < 2 * L.nW + T + 2; ++i) base[i] = 0.0f;
        for (int64_t t = 1; t <= T + 1; ++t) {
            float *wrow = Wl + lut_w_row(t, K), *prow = P + lut_w_row(t, K);
            int64_t dm = t - 1;
            if (K > 0 && dm > K) dm = K;
            double W = 0.0, Pd = 1.0;
            wrow[0] = 0.0f;
            prow[0] = 1.0f;
            for (int64_t d = 1; d <= dm; ++d) {
                const int64_t k = t - d;
                W = r * W + Pd * Ck[k];
                Pd = Pd * (1.0 - lr * (sched ? sched[k] : 1.0) * lam);
                wrow[d] = (float)W;
                prow[d] = (float)Pd;
            }
        }
        for (int64_t t = 0; t <= T + 1; ++t) q[t] = (float)(1.0 - lr * (sched ? sched[t] : 1.0) * lam);
    }
    return 0;
}

}  // namespace gsdp
