// Host construction of the deferred-update tables (FP64 math, one FP32 rounding).
//
// A row deferred d steps at update t skipped the steps k = t-d .. t-1.  Eq. 3
// restores it with w -= lr W_t[d] m/(sqrt(v)+eps), where each skipped step k
// contributes its bias-corrected Adam step, decayed by the moments' decay
// since the row's last update (Sec. 4.3.1-4.3.2):
//     W_t[d] = sum_{k=t-d}^{t-1} r^(k-(t-d)) Cn[k],   r = b1/sqrt(b2),
//     Cn[k]  = b1 / ( sqrt(b2 / (1 - b2^k)) * (1 - b1^k) )     (unit rate)
// The paper precomputes these coefficients per step in a lookup table.  Here
// only the rows of the current and the next step are kept: going from step t
// to t+1, every row gains the newly skipped step t, W_{t+1}[d+1] = W_t[d] +
// r^d Cn[t], so the tables need O(T + max_defer) memory and each step costs
// O(min(t, max_defer)) work (done on the device by the update call).  Powers
// come from repeated multiplication (no pow), every operation is one IEEE
// binary64 operation, and each entry is rounded once to FP32, so the values
// are fully determined by (b1, b2, t, d) and the schedule.  A learning-rate
// schedule s[t] (a multiplier of every column's rate at update t) enters as
// s[k] Cn[k] for the skipped step k and as s[t] / (1 - b1^t) in the step size.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gsdp_internal.h"

namespace gsdp {

namespace {

// typed views of a host image
struct Img {
    char *b;
    LutLayout L;
    LutHeader *h() const { return reinterpret_cast<LutHeader *>(b); }
    float *Wf(int s) const { return reinterpret_cast<float *>(b + L.oWf) + s * L.nrow; }
    float *Mf() const { return reinterpret_cast<float *>(b + L.oMf); }
    float *Vf() const { return reinterpret_cast<float *>(b + L.oVf); }
    float *SS() const { return reinterpret_cast<float *>(b + L.oSS); }
    float *BC() const { return reinterpret_cast<float *>(b + L.oBC); }
    double *Wd(int s) const { return reinterpret_cast<double *>(b + L.oWd) + s * L.nrow; }
    double *R() const { return reinterpret_cast<double *>(b + L.oR); }
    double *Cn() const { return reinterpret_cast<double *>(b + L.oC); }
    char *cls(int c) const { return b + L.oCls + c * L.cls_bytes; }
    float *Wlf(int c, int s) const { return reinterpret_cast<float *>(cls(c) + L.cWlf) + s * L.nrow; }
    float *Pf(int c, int s) const { return reinterpret_cast<float *>(cls(c) + L.cPf) + s * L.nrow; }
    float *qf(int c) const { return reinterpret_cast<float *>(cls(c) + L.cqf); }
    double *Wld(int c, int s) const { return reinterpret_cast<double *>(cls(c) + L.cWld) + s * L.nrow; }
    double *Pd(int c, int s) const { return reinterpret_cast<double *>(cls(c) + L.cPd) + s * L.nrow; }
    double *qd(int c) const { return reinterpret_cast<double *>(cls(c) + L.cqd); }
};

void set_wbound(const Img &im);

// Adam tables of a zeroed image: powers, Cn, R, Mf, Vf, SS, BC and the header
// (row slot 1 holds step 1: W_1 = [0]).
void fill_adam(const Img &im, double b1, double b2, const double *sched, int kind, int nclass)
{
    const LutLayout &L = im.L;
    const int64_t T = L.T;
    const int64_t kmax = (T + 2 > L.nrow + 1 ? T + 2 : L.nrow + 1);
    std::vector<double> P1(kmax + 1), P2(kmax + 1);
    P1[0] = 1.0;
    P2[0] = 1.0;
    for (int64_t k = 1; k <= kmax; ++k) {
        P1[k] = P1[k - 1] * b1;
        P2[k] = P2[k - 1] * b2;
    }
    const double r = b1 / std::sqrt(b2);
    double *Cn = im.Cn(), *R = im.R();
    for (int64_t k = 1; k <= T + 1; ++k) {
        Cn[k] = b1 / (std::sqrt(b2 / (1.0 - P2[k])) * (1.0 - P1[k]));
        // a learning-rate schedule scales the skipped step k by its own rate
        if (sched) Cn[k] = sched[k] * Cn[k];
    }
    R[0] = 1.0;
    for (int64_t d = 1; d < L.nrow; ++d) R[d] = R[d - 1] * r;
    for (int64_t d = 0; d < L.nrow; ++d) {
        im.Mf()[d] = (float)P1[d + 1];
        im.Vf()[d] = (float)P2[d + 1];
    }
    for (int64_t t = 1; t <= T + 1; ++t) {
        im.SS()[t] = sched ? (float)(sched[t] / (1.0 - P1[t])) : (float)(1.0 / (1.0 - P1[t]));
        im.BC()[t] = (float)std::sqrt(1.0 - P2[t]);
    }
    LutHeader *h = im.h();
    h->t_row[0] = 0;
    h->t_row[1] = 1;
    h->T = (int32_t)T;
    h->K = (int32_t)L.K;
    h->nclass = nclass;
    h->kind = kind;
    h->error = 0;
    set_wbound(im);
}

// A bound of every restore coefficient the tables will hold: W_t[d] is a sum
// of d per-step contributions Cn[k] weighted by R[0..d-1], all positive, so
// W_t[d] <= max_k Cn[k] * sum_{j < D} R[j] for the largest defer count D.
// Raised by 1e-6 relative (the FP64 sums' and the FP32 rounding's error)
// and rounded up to FP32.
void set_wbound(const Img &im)
{
    const LutLayout &L = im.L;
    double cmax = 0.0, rsum = 0.0;
    for (int64_t k = 1; k <= L.T + 1; ++k) cmax = std::max(cmax, im.Cn()[k]);
    for (int64_t d = 0; d + 1 < L.nrow; ++d) rsum += im.R()[d];
    const double wb = cmax * rsum * (1.0 + 1e-6);
    float f = (float)wb;
    if ((double)f < wb) f = std::nextafter(f, HUGE_VALF);
    im.h()->wbound = f;
}

bool open_image(void *out, int64_t nbytes, int32_t T, int32_t K, int nclass, Img *im)
{
    if (!out || T < 1 || K < 0 || nclass < 0) return false;
    if (nbytes < lut_total_bytes(T, K, nclass)) return false;
    std::memset(out, 0, (size_t)lut_total_bytes(T, K, nclass));
    im->b = static_cast<char *>(out);
    im->L = lut_layout(T, K);
    return true;
}

// Rows of step t -> rows of step t + 1 (the device advance does the same
// operations in the same order).
void advance_host(const Img &im, int64_t t)
{
    const LutLayout &L = im.L;
    const int so = (int)(t & 1), sn = (int)((t + 1) & 1);
    const int64_t dn = t < L.nrow - 1 ? t : L.nrow - 1;
    const double *R = im.R();
    const double c = im.Cn()[t];
    double *wo = im.Wd(so), *wn = im.Wd(sn);
    float *fn = im.Wf(sn);
    wn[0] = 0.0;
    fn[0] = 0.0f;
    for (int64_t d = 0; d < dn; ++d) {
        wn[d + 1] = wo[d] + R[d] * c;
        fn[d + 1] = (float)wn[d + 1];
    }
    for (int cl = 0; cl < im.h()->nclass; ++cl) {
        const double q = im.qd(cl)[t];
        double *lo = im.Wld(cl, so), *ln = im.Wld(cl, sn), *po = im.Pd(cl, so), *pn = im.Pd(cl, sn);
        float *lf = im.Wlf(cl, sn), *pf = im.Pf(cl, sn);
        ln[0] = 0.0;
        pn[0] = 1.0;
        lf[0] = 0.0f;
        pf[0] = 1.0f;
        for (int64_t d = 0; d < dn; ++d) {
            ln[d + 1] = q * lo[d] + R[d] * c;
            pn[d + 1] = q * po[d];
            lf[d + 1] = (float)ln[d + 1];
            pf[d + 1] = (float)pn[d + 1];
        }
    }
    im.h()->t_row[sn] = (int32_t)(t + 1);
}

}  // namespace

int build_lut_host(double b1, double b2, int32_t T, int32_t K, const double *sched, void *out, int64_t nbytes)
{
    Img im;
    if (!open_image(out, nbytes, T, K, 0, &im)) return -1;
    fill_adam(im, b1, b2, sched, kLutAdam, 0);
    return 0;
}

// SGD with momentum mu: with zero gradients the buffer decays as mu^j, so the
// skipped steps move w by lr buf W[d], W_t[d] = sum_{k=t-d}^{t-1} mu^(k-(t-d)+1) s[k]
// (R[d] = mu^(d+1), Cn[k] = s[k]); the first-moment table holds mu^(d+1), the
// step table s[t]; the second-moment and bias tables are 1.
int build_lut_sgdm_host(double mu, int32_t T, int32_t K, const double *sched, void *out, int64_t nbytes)
{
    Img im;
    if (!open_image(out, nbytes, T, K, 0, &im)) return -1;
    const LutLayout &L = im.L;
    double *Cn = im.Cn(), *R = im.R();
    for (int64_t k = 1; k <= T + 1; ++k) Cn[k] = sched ? sched[k] : 1.0;
    double p = 1.0;
    for (int64_t d = 0; d < L.nrow; ++d) {
        p = p * mu;
        R[d] = p;
        im.Mf()[d] = (float)p;
        im.Vf()[d] = 1.0f;
    }
    for (int64_t t = 1; t <= T + 1; ++t) {
        im.SS()[t] = sched ? (float)sched[t] : 1.0f;
        im.BC()[t] = 1.0f;
    }
    LutHeader *h = im.h();
    h->t_row[0] = 0;
    h->t_row[1] = 1;
    h->T = T;
    h->K = K;
    h->nclass = 0;
    h->kind = kLutSgdm;
    set_wbound(im);
    return 0;
}

// AdamW: every step k first scales w by q_k = 1 - lr s[k] lambda, so the
// catch-up of d skipped steps is w P[d] - lr (m/(sqrt(v)+eps)) Wl[d], every
// skipped step's term also shrunk by the decays after it:
//   Wl_t[d] = sum_{k=t-d}^{t-1} r^(k-(t-d)) (prod_{j=k+1}^{t-1} q_j) Cn[k],
//   P_t[d]  = prod_{k=t-d}^{t-1} q_k,
// advanced as Wl'[d+1] = q_t Wl[d] + R[d] Cn[t], P'[d+1] = q_t P[d]; step t
// scales by q_t before its Adam update.  The tables depend on the column rate
// through q: one set per decay class (distinct rate), after the Adam tables.
int build_lut_adamw_host(double b1, double b2, double lam, const float *rates, int nclass, int32_t T, int32_t K,
                         const double *sched, void *out, int64_t nbytes)
{
    Img im;
    if (nclass < 1 || nclass > kMaxDecayClasses || !rates) return -1;
    if (!open_image(out, nbytes, T, K, nclass, &im)) return -1;
    fill_adam(im, b1, b2, sched, kLutAdamw, nclass);
    for (int c = 0; c < nclass; ++c) {
        const double lr = (double)rates[c];
        for (int64_t t = 0; t <= (int64_t)T + 1; ++t) {
            im.qd(c)[t] = 1.0 - lr * (sched ? sched[t] : 1.0) * lam;
            im.qf(c)[t] = (float)im.qd(c)[t];
        }
        im.Pd(c, 1)[0] = 1.0;
        im.Pf(c, 1)[0] = 1.0f;
    }
    return 0;
}

int seek_lut_host(void *img, int64_t nbytes, int64_t step)
{
    if (!img || nbytes < (int64_t)sizeof(LutHeader)) return -1;
    const LutHeader *h = static_cast<const LutHeader *>(img);
    if (h->T < 1 || h->K < 0 || h->nclass < 0 || h->nclass > kMaxDecayClasses) return -1;
    if (nbytes < lut_total_bytes(h->T, h->K, h->nclass)) return -1;
    const int64_t cur = h->t_row[0] > h->t_row[1] ? h->t_row[0] : h->t_row[1];
    if (cur < 1 || step < cur || step > (int64_t)h->T + 1) return -1;
    Img im;
    im.b = static_cast<char *>(img);
    im.L = lut_layout(h->T, h->K);
    for (int64_t t = cur; t < step; ++t) advance_host(im, t);
    return 0;
}

}  // namespace gsdp
