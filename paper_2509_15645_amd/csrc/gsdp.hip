// libgsdp: HIP kernels and C ABI of the Gaussian-parameter hot path of
// GS-Scale-style 3DGS training (arXiv 2509.15645) for MI355X (gfx950).
//
// Build flags matter for exactness: -ffp-contract=off (no FMA contraction),
// correctly rounded FP32 division and square root, denormals preserved, and
// packed-FP32 instructions disabled.  Every floating-point expression that
// defines a result is written as the exact sequence of IEEE operations of its
// definition; only the band classifier's conservative bounds (which decide
// nothing near a boundary) use fused multiply-adds and the hardware
// reciprocal and square root, inside stated margins.
//
// Kernels
//   k_cull, k_tile_reduce, k_tile_ids
//               one block per 512-row tile stages the geometry through LDS
//               with 128-bit loads (non-temporal when the swept arrays exceed
//               the last-level cache), restores deferred rows (band classifier
//               first), culls and stores wave ballots and tile counts; group
//               sums of 64 tiles (skipped for small models); one block per
//               group writes the tile prefixes and the ids in order.
//               Deterministic, no global atomics, no waits.
//   k_rows      one wavefront per Gaussian row, lanes 0..9 = G columns,
//               lanes 10..10+dim = A columns; modes:
//                 gather  restore current values into compact buffers
//                 adam    restore + Adam (AdamW, SGD with momentum) with fused
//                         gradient scatter
//                 flush   catch up every deferred row
//                 max     FP8 first pass (block maxima of new moments)
//   k_fp8_rescale, k_dense_geo, k_scatter
//   k_cull_multi, k_multi_reduce, k_multi_offsets, k_multi_ids, k_grad_sum
//               batched form; a wavefront's box of rows is tested against
//               all cameras at once (one per lane) before the per-row tests
//   k_dens_plan, k_dens_scan, k_dens_apply                densification
//   k_synth     synthetic gradients (harness only)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "gsdp.h"
#include "gsdp_internal.h"

using u32 = uint32_t;
using u64 = unsigned long long;
using gsdp::kCullBlock;
using gsdp::kCullIpt;
using gsdp::kCullTile;
using gsdp::kChunkRows;
static_assert(kChunkRows == GS_CHUNK_ROWS, "chunk size of the public header");

namespace {

// ---------------------------------------------------------------------------
// exp for the cull.  Cody & Waite (1980) reduction x = k ln2 + r with ln2 split
// into 355/512 (exact products k*LN2_HI for |k| <= 128) and an FP32 tail, the
// degree-7 Taylor polynomial of e^r on |r| <= ln2/2 in Horner form, then 2^k
// by ldexp.  Each step is one correctly rounded operation, so the result is
// bit-reproducible on any IEEE machine.  Ordered comparisons let NaN through.
__device__ __forceinline__ float exp_cw(float x)
{
    if (x < -87.0f) x = -87.0f;
    if (x > 88.0f) x = 88.0f;
    const float k = rintf(x * 1.44269504088896341f);
    const float r = (x - k * 0.693359375f) - k * -2.12194440e-4f;
    float p = 1.98412698e-4f;
    p = p * r + 1.38888889e-3f;
    p = p * r + 8.33333333e-3f;
    p = p * r + 4.16666667e-2f;
    p = p * r + 1.66666667e-1f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return ldexpf(p, (int)k);
}

struct CamK {
    float R[9], T[3];
    float fx, fy, cx, cy, W, H, zn, zf;
};

// Cull of one Gaussian g = (mean, log-scale, quaternion wxyz) against the
// camera: the 3-sigma EWA footprint (projected covariance + 0.3 px dilation,
// largest eigenvalue, radius rounded up) around the projected centre must
// overlap the image, and the centre must lie strictly between near and far
// (Sec. 2.4 step 1).  All comparisons are positive, so a NaN anywhere culls.
__device__ __forceinline__ bool cull_v1(const float *g, const CamK &c)
{
    const float x = ((c.R[0] * g[0] + c.R[1] * g[1]) + c.R[2] * g[2]) + c.T[0];
    const float y = ((c.R[3] * g[0] + c.R[4] * g[1]) + c.R[5] * g[2]) + c.T[1];
    const float z = ((c.R[6] * g[0] + c.R[7] * g[1]) + c.R[8] * g[2]) + c.T[2];

    float qw = g[6], qx = g[7], qy = g[8], qz = g[9];
    const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    const float inv = 1.0f / sqrtf(n2);
    qw = qw * inv;
    qx = qx * inv;
    qy = qy * inv;
    qz = qz * inv;
    const float Q0 = 1.0f - 2.0f * (qy * qy + qz * qz);
    const float Q1 = 2.0f * (qx * qy - qw * qz);
    const float Q2 = 2.0f * (qx * qz + qw * qy);
    const float Q3 = 2.0f * (qx * qy + qw * qz);
    const float Q4 = 1.0f - 2.0f * (qx * qx + qz * qz);
    const float Q5 = 2.0f * (qy * qz - qw * qx);
    const float Q6 = 2.0f * (qx * qz - qw * qy);
    const float Q7 = 2.0f * (qy * qz + qw * qx);
    const float Q8 = 1.0f - 2.0f * (qx * qx + qy * qy);

    const float s0 = exp_cw(g[3]), s1 = exp_cw(g[4]), s2 = exp_cw(g[5]);
    const float M0 = Q0 * s0, M1 = Q1 * s1, M2 = Q2 * s2;
    const float M3 = Q3 * s0, M4 = Q4 * s1, M5 = Q5 * s2;
    const float M6 = Q6 * s0, M7 = Q7 * s1, M8 = Q8 * s2;
    // world covariance, symmetric: S_ab = M_a . M_b
    const float S00 = (M0 * M0 + M1 * M1) + M2 * M2;
    const float S01 = (M0 * M3 + M1 * M4) + M2 * M5;
    const float S02 = (M0 * M6 + M1 * M7) + M2 * M8;
    const float S10 = (M3 * M0 + M4 * M1) + M5 * M2;
    const float S11 = (M3 * M3 + M4 * M4) + M5 * M5;
    const float S12 = (M3 * M6 + M4 * M7) + M5 * M8;
    const float S20 = (M6 * M0 + M7 * M1) + M8 * M2;
    const float S21 = (M6 * M3 + M7 * M4) + M8 * M5;
    const float S22 = (M6 * M6 + M7 * M7) + M8 * M8;

    const float rz = 1.0f / z;
    const float limx = 1.3f * ((0.5f * c.W) / c.fx);
    const float limy = 1.3f * ((0.5f * c.H) / c.fy);
    float tx = x * rz, ty = y * rz;
    if (tx < -limx) tx = -limx;
    if (tx > limx) tx = limx;
    if (ty < -limy) ty = -limy;
    if (ty > limy) ty = limy;
    const float J00 = c.fx * rz, J02 = -(c.fx * tx) * rz;
    const float J11 = c.fy * rz, J12 = -(c.fy * ty) * rz;

    // T = J R (2x3)
    const float A0 = J00 * c.R[0] + J02 * c.R[6];
    const float A1 = J00 * c.R[1] + J02 * c.R[7];
    const float A2 = J00 * c.R[2] + J02 * c.R[8];
    const float B0 = J11 * c.R[3] + J12 * c.R[6];
    const float B1 = J11 * c.R[4] + J12 * c.R[7];
    const float B2 = J11 * c.R[5] + J12 * c.R[8];
    // U = T S
    const float U00 = (A0 * S00 + A1 * S10) + A2 * S20;
    const float U01 = (A0 * S01 + A1 * S11) + A2 * S21;
    const float U02 = (A0 * S02 + A1 * S12) + A2 * S22;
    const float U10 = (B0 * S00 + B1 * S10) + B2 * S20;
    const float U11 = (B0 * S01 + B1 * S11) + B2 * S21;
    const float U12 = (B0 * S02 + B1 * S12) + B2 * S22;
    const float a = ((U00 * A0 + U01 * A1) + U02 * A2) + 0.3f;
    const float b = (U00 * B0 + U01 * B1) + U02 * B2;
    const float cc = ((U10 * B0 + U11 * B1) + U12 * B2) + 0.3f;

    const float det = a * cc - b * b;
    const float mid = 0.5f * (a + cc);
    float disc = mid * mid - det;
    if (!(disc > 0.1f)) disc = 0.1f;
    const float lam = mid + sqrtf(disc);
    const float r = ceilf(3.0f * sqrtf(lam));

    const float u = (c.fx * x) * rz + c.cx;
    const float v = (c.fy * y) * rz + c.cy;
    return (z > c.zn) & (z < c.zf) & (det > 0.0f) & (u + r > 0.0f) & (u - r < c.W) & (v + r > 0.0f) &
           (v - r < c.H);
}

// Restore of one element deferred d > 0 steps (Eq. 3 with eps factored out):
// q = m / (sqrt(v) + eps) with the stored (old) moments, clamped to [-rb, rb],
// then w - (W[d] lr) q.  rb is 1.03x the Cauchy-Schwarz bound of |m|/sqrt(v)
// for Adam moments grown from zero, so the clamp never acts on a reachable
// FP32 state; it bounds the restore for any stored moments (quantised ones too).
__device__ __forceinline__ float restore1(float w, float m, float v, float wd, float lr, float eps, float rb)
{
    const float den = sqrtf(v) + eps;
    float q = m / den;
    // selects, not branches: a NaN stays NaN
    q = q > rb ? rb : q;
    q = q < -rb ? -rb : q;
    const float wsc = wd * lr;
    return w - wsc * q;
}

// AdamW restore of one element (d > 0): (P[d] w) - (Wl[d] lr) q with q the
// clamped m/(sqrt(v)+eps): Eq. 3 with every skipped update shrunk by the
// decoupled weight decays that follow it.
__device__ __forceinline__ float restore_w(float w, float m, float v, float wd, float pd, float lr, float eps, float rb)
{
    const float den = sqrtf(v) + eps;
    float q = m / den;
    q = q > rb ? rb : q;
    q = q < -rb ? -rb : q;
    const float a = pd * w;
    const float b = (wd * lr) * q;
    return a - b;
}

// SplitMix64 (Steele, Lea & Flood 2014): output k of the stream seeded s.
__device__ __forceinline__ u64 mix64(u64 z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ u64 sm_at(u64 s, u64 i) { return mix64(s + (i + 1ull) * 0x9E3779B97F4A7C15ull); }

// Moment storage.
//   F32 : plain FP32.
//   BF16: the upper 16 bits of the FP32 pattern; stores round stochastically by
//         adding 16 random bits before truncation (Inf kept, NaN quieted).
//   FP8 : OCP E4M3FN codes times one FP32 power-of-two scale per block of 128
//         rows (per group, per moment); the second moment is stored as its
//         square root.  Stores round stochastically (see e4m3_sr).
constexpr int kFp8Block = 128;

struct MomRef {
    void *p;            // [n][ld] elements
    const float *s;     // FP8 block scales (FP8 only)
    int64_t ld;
};

__device__ __forceinline__ float e4m3_dec(u32 b)
{
    const int e = (int)((b >> 3) & 0xfu), m = (int)(b & 7u);
    if (e == 15 && m == 7) return __uint_as_float(0x7fc00000u);
    const float a = e == 0 ? ldexpf((float)m, -9) : ldexpf((float)(8 + m), e - 10);
    return (b & 0x80u) ? -a : a;
}

// Stochastic rounding of y to E4M3 (saturating at 448): in a binade of
// quantum q, y = k q + f q rounds up when f * 65536 > r16.
__device__ __forceinline__ u32 e4m3_sr(float y, u32 r16)
{
    if (__builtin_isnan(y)) return 0x7fu;
    const u32 sign = (__float_as_uint(y) >> 31) << 7;
    float a = fabsf(y);
    if (a > 448.0f) a = 448.0f;
    const int e = a < 0.015625f ? -6 : (int)((__float_as_uint(a) >> 23) & 0xffu) - 127;
    const float quantum = ldexpf(1.0f, e - 3);
    const float yq = a / quantum;
    float k = floorf(yq);
    const float f = yq - k;
    if (f * 65536.0f > (float)r16) k = k + 1.0f;
    const float val = k * quantum;
    if (val == 0.0f) return sign;
    if (val < 0.015625f) return sign | (u32)(val / ldexpf(1.0f, -9));
    const int ev = (int)((__float_as_uint(val) >> 23) & 0xffu) - 127;
    const int mant = (int)(val / ldexpf(1.0f, ev) * 8.0f) - 8;
    return sign | ((u32)(ev + 7) << 3) | (u32)mant;
}

// Smallest power of two p with amax / p <= 448 (0 for amax <= 0 or non-finite).
__device__ __forceinline__ float fp8_scale_for(float amax)
{
    if (!(amax > 0.0f) || !(amax < __builtin_huge_valf())) return 0.0f;
    const float r = amax / 448.0f;
    int e;
    const float fr = frexpf(r, &e);
    return fr == 0.5f ? ldexpf(1.0f, e - 1) : ldexpf(1.0f, e);
}

template <int ST> __device__ __forceinline__ float mom_load(const MomRef &q, int64_t row, int64_t col, bool is_v);
template <> __device__ __forceinline__ float mom_load<GS_F32>(const MomRef &q, int64_t row, int64_t col, bool)
{
    return static_cast<const float *>(q.p)[row * q.ld + col];
}
template <> __device__ __forceinline__ float mom_load<GS_BF16>(const MomRef &q, int64_t row, int64_t col, bool)
{
    return __uint_as_float((u32) static_cast<const uint16_t *>(q.p)[row * q.ld + col] << 16);
}
template <> __device__ __forceinline__ float mom_load<GS_FP8E4M3>(const MomRef &q, int64_t row, int64_t col,
                                                                  bool is_v)
{
    const float x = e4m3_dec(static_cast<const uint8_t *>(q.p)[row * q.ld + col]) * q.s[row / kFp8Block];
    return is_v ? x * x : x;
}

template <int ST>
__device__ __forceinline__ void mom_store(const MomRef &q, int64_t row, int64_t col, float x, u32 r16, bool is_v);
template <>
__device__ __forceinline__ void mom_store<GS_F32>(const MomRef &q, int64_t row, int64_t col, float x, u32, bool)
{
    static_cast<float *>(q.p)[row * q.ld + col] = x;
}
template <>
__device__ __forceinline__ void mom_store<GS_BF16>(const MomRef &q, int64_t row, int64_t col, float x, u32 r16, bool)
{
    const u32 u = __float_as_uint(x);
    uint16_t h;
    if ((u & 0x7f800000u) == 0x7f800000u) h = (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x0040u : 0u));
    else h = (uint16_t)((u + r16) >> 16);
    static_cast<uint16_t *>(q.p)[row * q.ld + col] = h;
}

// Byte address of row r (stride s bytes) of the array at p, as a value the
// compiler cannot see through: it then addresses the lanes' columns as this
// scalar base plus a 32-bit lane offset, instead of re-associating the sum
// into per-lane 64-bit arithmetic.
typedef __attribute__((address_space(1))) char gchar;
// A 32-bit lane offset, zero-extended where it is used: the hardware adds it
// to a scalar base (no 64-bit lane address), but only if the extension is in
// the same block as the access, so it is not left for the compiler to hoist.
__device__ __forceinline__ u64 lane_off(u32 o)
{
    asm volatile("" : "+v"(o));
    return (u64)o;
}
__device__ __forceinline__ gchar *srow(const void *p, u64 r, u32 s)
{
    // rows and strides fit 32 bits: one 32 x 32 -> 64-bit product
    gchar *q = (gchar *)p + (u64)(u32)r * (u64)s;
    asm("" : "+s"(q));
    return q;
}

// Loads of data that a launch reads exactly once (the cull's sweep over all
// rows): marked non-temporal, so they do not displace reused lines from the
// caches.  A one-pass read of the geometry array runs about 11 % faster this
// way on this part.
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_once(const float4 *q)
{
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(q));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int ld_once(const int *q) { return __builtin_nontemporal_load(q); }
// non-temporal when NT, an ordinary load otherwise
template <bool NT, typename T>
__device__ __forceinline__ T ld_sweep(const T *q)
{
    if (NT) return ld_once(q);
    return *q;
}

// Loads and stores of one moment element at an element address (the row's
// base computed once per row on the scalar unit, plus the lane's column);
// same arithmetic as mom_load / mom_store.  s is the row's FP8 block scale.
// A load is split into the raw storage word and its decoding, so that the
// decoding of a row's moments does not wait for them before the next row's
// loads are issued.
// A register value the compiler takes as defined but that no instruction sets
// (for values that are never used where no load wrote them).
template <typename T> __device__ __forceinline__ T undef_v()
{
    u32 t;
    asm volatile("" : "=v"(t));
    return (T)t;
}
template <int ST> struct RawT { typedef u32 T; };
template <> struct RawT<GS_BF16> { typedef uint16_t T; };
template <> struct RawT<GS_FP8E4M3> { typedef uint8_t T; };
template <int ST> __device__ __forceinline__ typename RawT<ST>::T mraw(const char *e)
{
    return *reinterpret_cast<const typename RawT<ST>::T *>(e);
}
template <int ST> __device__ __forceinline__ float mdec(u32 raw, float s, bool is_v)
{
    if (ST == GS_F32) return __uint_as_float(raw);
    if (ST == GS_BF16) return __uint_as_float(raw << 16);
    const float x = e4m3_dec(raw) * s;
    return is_v ? x * x : x;
}
template <int ST> __device__ __forceinline__ void mstore(char *e, float s, float x, u32 r16, bool is_v)
{
    if (ST == GS_F32) {
        *reinterpret_cast<float *>(e) = x;
    } else if (ST == GS_BF16) {
        const u32 u = __float_as_uint(x);
        uint16_t h;
        if ((u & 0x7f800000u) == 0x7f800000u) h = (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x0040u : 0u));
        else h = (uint16_t)((u + r16) >> 16);
        *reinterpret_cast<uint16_t *>(e) = h;
    } else {
        const float y = is_v ? sqrtf(x) : x;
        *reinterpret_cast<uint8_t *>(e) = s > 0.0f ? (uint8_t)e4m3_sr(y / s, r16) : (uint8_t)0;
    }
}
template <int ST> constexpr int msize() { return ST == GS_F32 ? 4 : (ST == GS_BF16 ? 2 : 1); }

// Adam step of one element, (st m1) / (sqrt(v1)/bc + eps), clamped to
// st bc rb: moments grown from zero keep |m1|/sqrt(v1) below 7.27 < rb, so the
// clamp never acts on an FP32 state; it bounds the step when quantised
// moments lose the second moment to underflow.
__device__ __forceinline__ float adam_step(float m1, float v1, float st, float bc, float eps, float rb)
{
    const float den = sqrtf(v1) / bc + eps;
    float upd = (st * m1) / den;
    const float lim = (st * bc) * rb;
    upd = upd > lim ? lim : upd;
    upd = upd < -lim ? -lim : upd;
    return upd;
}

// Per-camera constants of the band classifier (host-computed, rounded up).
struct BandK {
    float rs0, rs1, rs2;   // |R_i0| + |R_i1| + |R_i2|, rows of the camera rotation
    float jf2;             // fx^2 (1 + limx^2) + fy^2 (1 + limy^2): bound of |J|_F^2 z^2
    float kpos, kscl, kq;  // B * max lr over position / log-scale / quaternion columns
};

// Per-camera constants of side_out (host-computed in FP64, margins rounded
// up): the four side planes in world coordinates, n . p + k, with
// n_l = fx R_0 + cl R_2, k_l = fx T_0 + cl T_2 (cl = cx + 3.93), the right
// side -fx and cr = W - cx + 3.93, the top fy, R_1, T_1 and ct = cy + 3.93,
// the bottom -fy and cb = H - cy + 3.93; n1 their 1-norms.
struct SideK {
    float n[4][3], k[4], n1[4];
    float ksig;            // 3.003 sqrt(1.001 jf2)
    float sa, sb;          // slack: 1e-5 (sa (mu + dp) + sb + ksig sig) covers every rounding
};

// One camera with its classifier constants: the records of gs_camera_pack,
// read by the batched cull and by the single-camera cull from a device table.
struct CamPack {
    CamK cam;
    BandK band;
    SideK side;
    float pad[14];
};
static_assert(sizeof(CamPack) == 256, "camera records are 256 bytes");

// Conservative classification of one Gaussian whose stored geometry g may be
// stale by a restore of at most B*W[d]*lr per column.  B is the clamp of the
// restore factor (1.03x the Cauchy-Schwarz bound (1-b1)/sqrt((1-b2)(1-b1^2/b2))
// of |m|/sqrt(v) for Adam moments grown from zero, 7.27 for b = (0.9, 0.999)).
// classify_cam returns 0 when every admissible restored geometry is culled by
// cull_v1, 1 when every one is kept, 2 when undecided (run the exact test).
// Bounds, all with generous margins for FP32 rounding of the exact test:
//   camera-space centre moves by <= |R_i|_1 * position drift;
//   projected covariance trace <= |J|_F^2 sigma_max^2, |J|_F^2 <= jf2 / z^2 since
//   |tan| is clamped, and the radius of cull_v1 is <= ceil(3 sqrt(trace + 0.92));
//   the radius is >= 3 and det > 0 holds when the trace bound is <= 1000.
// classify_pre holds the camera-independent part of one row.
struct RowPre {
    float dp;       // position drift bound incl. rounding of the restore
    float sig;      // bound of sigma_max after the restore
    float sig2;     // its square
    float mu;       // largest |position coordinate|
    int ok;         // 0: undecidable (non-finite, huge scale); bit 1: quaternion stays away from 0
};

__device__ __forceinline__ RowPre classify_pre(const float *g, float wd, const BandK &b)
{
    RowPre p;
    // one finiteness test of a sum: a NaN or an infinity anywhere (or a sum that
    // overflows) makes it non-finite, which only sends the row to the exact path
    const float fsum = (((fabsf(g[0]) + fabsf(g[1])) + (fabsf(g[2]) + fabsf(g[3]))) +
                        ((fabsf(g[4]) + fabsf(g[5])) + (fabsf(g[6]) + fabsf(g[7])))) + (fabsf(g[8]) + fabsf(g[9]));
    const bool fin = __builtin_isfinite(fsum);
    const float dpos = b.kpos * wd, dscl = b.kscl * wd, dq = b.kq * wd;
    const float mu = fmaxf(fmaxf(fabsf(g[0]), fabsf(g[1])), fabsf(g[2]));
    p.dp = dpos + 1e-6f * mu;
    p.mu = mu;
    const float smax = fmaxf(fmaxf(g[3], g[4]), g[5]) + dscl + 1e-6f * fmaxf(fmaxf(fabsf(g[3]), fabsf(g[4])), fabsf(g[5]));
    const float sig = __expf(fminf(smax, 80.0f)) * 1.001f;
    p.sig = sig;
    p.sig2 = sig * sig;
    // |q| > 2.002 dq + 1e-6, compared squared (the 0.1% margin covers the rounding)
    const float qn2 = fmaf(g[9], g[9], fmaf(g[8], g[8], fmaf(g[7], g[7], g[6] * g[6])));
    const float qmin = 2.002f * dq + 1e-6f;
    p.ok = (fin && smax < 80.0f) ? (qn2 > 1.001f * (qmin * qmin) ? 3 : 1) : 0;
    return p;
}

// Decision of one row against one camera: 0 sure-out, 1 sure-in, 2 exact
// path.  Evaluated without branches: every bound is computed and the tests are
// combined in their order of precedence (a row of a wavefront rarely leaves
// early together with all 63 others, so branching would only add mask work).
// Camera-space centre of the stored row and the half-widths of the interval
// in which the exact test's camera-space coordinates of every admissible
// restored geometry lie (drift and the exact path's rounding).
struct CamBox {
    float x, y, z, ex, ey, ez;
};

__device__ __forceinline__ CamBox cam_box(const float *g, const RowPre &p, const CamK &c, const BandK &b)
{
    CamBox q;
    const float dp = p.dp;
    // The bounds below are evaluated with fused multiply-adds: any evaluation
    // order of these short sums differs from the exact path's by a few ulp of
    // the terms' magnitude, far inside the 1e-6 relative slack.
    q.x = fmaf(c.R[2], g[2], fmaf(c.R[1], g[1], fmaf(c.R[0], g[0], c.T[0])));
    q.y = fmaf(c.R[5], g[2], fmaf(c.R[4], g[1], fmaf(c.R[3], g[0], c.T[1])));
    q.z = fmaf(c.R[8], g[2], fmaf(c.R[7], g[1], fmaf(c.R[6], g[0], c.T[2])));
    // magnitude of the terms of each transform row, bounded by |R_i|_1 max|mu| + |T_i|
    // (rounds up by far less than the 1e-6 relative slack it feeds)
    const float sx = fmaf(b.rs0, p.mu, fabsf(c.T[0]));
    const float sy = fmaf(b.rs1, p.mu, fabsf(c.T[1]));
    const float sz = fmaf(b.rs2, p.mu, fabsf(c.T[2]));
    const float dx = b.rs0 * dp, dy = b.rs1 * dp, dz = b.rs2 * dp;
    q.ex = fmaf(1e-6f, sx + dx, dx) + 1e-6f;
    q.ey = fmaf(1e-6f, sy + dy, dy) + 1e-6f;
    q.ez = fmaf(1e-6f, sz + dz, dz) + 1e-6f;
    return q;
}

// Sure-out test of the summary cull, without divisions or square roots: true
// only when every admissible restored geometry is culled by cull_v1 (for a
// row whose RowPre is decidable, ok != 0).  The exact test keeps a row only
// if z' > zn > 0 and u + r > 0 (and the other three sides), with u its
// rounded projected centre fx x'/z' + cx (within 2.5e-7 relative of the
// exact value) and r its radius, r <= 3.003 sqrt(1.001 |J|_F^2 sigma'^2 +
// 0.95) + 1 (the bound classify_cam uses) with |J|_F^2 <= jf2 / z'^2.  As
// z' > 0, multiplying by z' and using sqrt(a + b) <= sqrt(a) + sqrt(b):
//   fx x' + (cx + 3.93) z' + ksig sigma' + 2.5e-7 (fx |x'| + |cx| z') > 0,
// where x', z' are the exact test's rounded camera coordinates of the
// restored centre p': x' = R_0 p' + T_0 within 2.5e-7 (|R_0| |p'| + |T_0|).
// So fx x' + cl z' <= n_l . p' + k_l plus rounding terms, and
// n_l . p' <= n_l . p + n1_l dp for a drift of at most dp per coordinate.
// With sigma' <= sig, keeping the row needs n_l . p + k_l + n1_l dp +
// ksig sig + slack > 0, slack covering the rounding terms (at most 2.5e-7
// (2 fx |R_0|_1 + (|cl| + |cx|) |R_2|_1) (mu + dp) plus the same with |T|)
// and this evaluation's own rounding (1e-6 of its terms' magnitudes); the
// host folds all of it into sa and sb with a tenfold margin.  A value <= 0
// means no kept geometry: the row is out on that side.  The same for the
// other three sides; out_z is classify_cam's own test.  NaN bounds make
// every comparison false (not out).
__device__ __forceinline__ bool side_out(const float4 &v, const RowPre &p, const CamK &c, const BandK &b,
                                         const SideK &k)
{
    const float z = fmaf(c.R[8], v.z, fmaf(c.R[7], v.y, fmaf(c.R[6], v.x, c.T[2])));
    const float sz = fmaf(b.rs2, p.mu, fabsf(c.T[2]));
    const float dz = b.rs2 * p.dp;
    const float ez = fmaf(1e-6f, sz + dz, dz) + 1e-6f;
    const bool out_z = (z + ez <= c.zn) | (z - ez >= c.zf);
    const float ks = k.ksig * p.sig;
    const float base = ks + 1e-5f * fmaf(k.sa, p.mu + p.dp, k.sb + ks);
    bool out = out_z;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float e = fmaf(k.n1[i], p.dp, k.k[i] + base);
        const float l = fmaf(k.n[i][2], v.z, fmaf(k.n[i][1], v.y, fmaf(k.n[i][0], v.x, e)));
        out |= l <= 0.0f;
    }
    return out;
}

__device__ __forceinline__ int classify_box(const CamBox &q, const RowPre &p, const CamK &c, const BandK &b)
{
    const float x = q.x, y = q.y, z = q.z, ex = q.ex, ey = q.ey, ez = q.ez;
    const float zlo = z - ez, zhi = z + ez;
    // bitwise, not short-circuit, combinations: no branches
    const bool out_z = (zhi <= c.zn) | (zlo >= c.zf);
    const bool z_pos = zlo > 0.0f;
    // the hardware reciprocal and square root (about 1 ulp) suffice: every
    // bound below carries a margin of 1e-5 relative or more (their values
    // are ignored when zlo <= 0)
    const float izl = __builtin_amdgcn_rcpf(zlo), izh = __builtin_amdgcn_rcpf(zhi);
    const float S = ((b.jf2 * izl) * izl) * p.sig2;
    const float lam = fmaf(1.001f, S, 0.95f);
    const float rup = fmaf(3.003f, __builtin_amdgcn_sqrtf(lam), 1.0f);
    const float xlo = x - ex, xhi = x + ex, ylo = y - ey, yhi = y + ey;
    const float qxlo = fminf(xlo * izl, xlo * izh), qxhi = fmaxf(xhi * izl, xhi * izh);
    const float qylo = fminf(ylo * izl, ylo * izh), qyhi = fmaxf(yhi * izl, yhi * izh);
    const float eu = fmaf(1e-5f, fmaf(c.fx, fmaxf(fabsf(qxlo), fabsf(qxhi)), fabsf(c.cx)), 1e-3f);
    const float ev = fmaf(1e-5f, fmaf(c.fy, fmaxf(fabsf(qylo), fabsf(qyhi)), fabsf(c.cy)), 1e-3f);
    const float ulo = fmaf(c.fx, qxlo, c.cx) - eu, uhi = fmaf(c.fx, qxhi, c.cx) + eu;
    const float vlo = fmaf(c.fy, qylo, c.cy) - ev, vhi = fmaf(c.fy, qyhi, c.cy) + ev;
    const bool out_uv = (uhi + rup <= 0.0f) | (ulo - rup >= c.W) | (vhi + rup <= 0.0f) | (vlo - rup >= c.H);
    const bool in = ((p.ok & 2) != 0) & (zlo > c.zn) & (zhi < c.zf) & (ulo > -1.5f) & (uhi < c.W + 1.5f) &
                    (vlo > -1.5f) & (vhi < c.H + 1.5f) & (lam <= 1000.0f);
    const int cls = out_z ? 0 : (!z_pos ? 2 : (out_uv ? 0 : (in ? 1 : 2)));
    return p.ok ? cls : 2;
}

__device__ __forceinline__ int classify_cam(const float *g, const RowPre &p, const CamK &c, const BandK &b)
{
    return classify_box(cam_box(g, p, c, b), p, c, b);
}

__device__ __forceinline__ int classify(const float *g, float wd, const CamK &c, const BandK &b)
{
    return classify_cam(g, classify_pre(g, wd, b), c, b);
}

// The squared quaternion norm above which a row's summary allows a sure-in
// decision.  A deferred row's quaternion may drift by up to 2 qd in norm (qd
// = kq W, W up to the tables' bound of every restore coefficient, about 9 for
// Adam), and the exact cull keeps a row only if its quaternion is not zero;
// with |q|^2 >= 0.64 a sure-in decision holds while qd stays below about
// 0.4 (rotation rates up to about 5.8e-3).
constexpr float kSumQn2 = 0.64f;

// Cull summary of one geometry row, 16 bytes: its centre (x, y, z) and one
// word w.  Bits 31..17 of w are those of s, the largest log-scale plus the
// classifier's rounding slack, rounded up to 7 significand bits (so s_up = w
// & 0xfffe0000, read as a float, is >= s), or of a quiet NaN (0x7fc0 in the
// high 16 bits) when the band classifier must leave the row to the exact
// test: a non-finite value or s of 80 or more.  Bit 16 is set when the
// quaternion's squared norm is at least kSumQn2: only then may the row be
// classified as surely kept (a sure-out decision needs no quaternion).  The
// low 16 bits hold the row's last update step modulo 2^16, from which the
// cull recovers the defer count while the steps fit 16 bits.  The band cull
// reads these 16 bytes instead of the 40-byte row and the last step; it
// loads the row only for the rows the classifier leaves undecided.
// (Rows whose quaternion is small are not sent to the exact test outright:
// after long deferrals the catch-up of Adam's momentum moves quaternion
// components by a tenth or more, and such rows would keep whole chunks from
// being skipped.)
__device__ __forceinline__ float4 cull_summary(const float *g, int last)
{
    const float fsum = (((fabsf(g[0]) + fabsf(g[1])) + (fabsf(g[2]) + fabsf(g[3]))) +
                        ((fabsf(g[4]) + fabsf(g[5])) + (fabsf(g[6]) + fabsf(g[7])))) + (fabsf(g[8]) + fabsf(g[9]));
    const float sm = fmaxf(fmaxf(g[3], g[4]), g[5]) + 1e-6f * fmaxf(fmaxf(fabsf(g[3]), fabsf(g[4])), fabsf(g[5]));
    const float qn2 = fmaf(g[9], g[9], fmaf(g[8], g[8], fmaf(g[7], g[7], g[6] * g[6])));
    const bool ok = __builtin_isfinite(fsum) && sm < 80.0f;
    // round toward +infinity: a positive value's magnitude up, a negative one's down
    u32 b = __float_as_uint(sm);
    if (b >> 31) b &= 0xfffe0000u;
    else if (b & 0x1ffffu) b = (b & 0xfffe0000u) + 0x20000u;
    const u32 hi = ok ? ((b & 0xfffe0000u) | ((u32)(qn2 >= kSumQn2) << 16)) : 0x7fc00000u;
    return make_float4(g[0], g[1], g[2], __uint_as_float(hi | ((u32)last & 0xffffu)));
}

// classify_pre from a summary.  The bounds are those of classify_pre: the
// centre is the row's, s already holds the slack that classify_pre adds after
// the drift (the sum differs by at most an ulp, far inside the 0.1% margin
// on sigma), a NaN s makes the row undecidable, and with the summary's
// quaternion bit (qok: squared norm at least kSumQn2) the sure-in condition
// on the quaternion holds whenever 1.001 qmin^2 < kSumQn2; without it the row
// can be decided out but not in.  v.w: s_up.
__device__ __forceinline__ RowPre classify_pre_sum(const float4 &v, float wd, const BandK &b, u32 qok)
{
    RowPre p;
    const float dpos = b.kpos * wd, dscl = b.kscl * wd, dq = b.kq * wd;
    const float mu = fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fabsf(v.z));
    p.dp = dpos + 1e-6f * mu;
    p.mu = mu;
    const float smax = v.w + dscl;
    const float sig = __expf(fminf(smax, 80.0f)) * 1.001f;
    p.sig = sig;
    p.sig2 = sig * sig;
    const float qmin = 2.002f * dq + 1e-6f;
    p.ok = smax < 80.0f ? ((qok != 0u && 1.001f * (qmin * qmin) < kSumQn2) ? 3 : 1) : 0;
    return p;
}

// Store the summary of a row whose new geometric values sit in lanes 0..9 of
// the wavefront (value x of this lane) and whose last step becomes `last`;
// every lane of the wavefront takes part, lane 0 stores.
__device__ __forceinline__ float4 cull_summary_store_wave(float4 *sum, u32 row, float x, int last)
{
    float g[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) g[j] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
    const float4 v = cull_summary(g, last);
    if ((threadIdx.x & 63) == 0) sum[row] = v;
    return v;
}

// Chunk records: rows [c * kChunkRows, (c + 1) * kChunkRows) share record c
// of 8 floats (lo x, y, z, s, hi x, y, z, 0): the box of their summary
// centres and the largest summary s (a NaN when some row's is).  Writers of
// summaries widen records with float minima and maxima taken through integer
// atomics: non-negative floats order as their bits read as signed integers,
// negative ones in reverse as unsigned integers; a positive NaN (the
// summaries' 0x7fc0 code) is above every float as a signed integer and below
// every negative one as an unsigned integer, so a NaN s stays once stored.
// -0 is stored as +0.
__device__ __forceinline__ void fatomic_min(float *p, float v)
{
    v = v == 0.0f ? 0.0f : v;
    if (v >= 0.0f) atomicMin(reinterpret_cast<int *>(p), __float_as_int(v));
    else atomicMax(reinterpret_cast<unsigned int *>(p), __float_as_uint(v));
}
__device__ __forceinline__ void fatomic_max(float *p, float v)
{
    v = v == 0.0f ? 0.0f : v;
    if (!(v < 0.0f)) atomicMax(reinterpret_cast<int *>(p), __float_as_int(v));
    else atomicMin(reinterpret_cast<unsigned int *>(p), __float_as_uint(v));
}

// Element lane & 7 of the chunk record of `row` (every lane loads; lanes
// past 7 repeat the first eight, so the wavefront reads one 32-byte record).
__device__ __forceinline__ float chunk_rec_lane(const float *chunk, u32 row)
{
    return chunk[(size_t)(row / (u32)kChunkRows) * 8u + (threadIdx.x & 7u)];
}

// Widen the chunk record of `row` to hold its new summary v (uniform over the
// wavefront); rec: this lane's element from chunk_rec_lane, loaded earlier in
// the same launch (records only grow, so an older value is never too wide).
// Lane j < 7 checks element j and widens it only when v lies outside.
__device__ __forceinline__ void chunk_widen(float *chunk, u32 row, const float4 &v, float rec)
{
    const u32 lane = threadIdx.x & 63u;
    const float sv = __uint_as_float(__float_as_uint(v.w) & 0xfffe0000u);
    const u32 e = lane < 3u ? lane : (lane < 4u ? 3u : lane - 4u);
    const float x = lane == 3u ? sv : (e == 0u ? v.x : (e == 1u ? v.y : v.z));
    const bool low = lane < 3u;
    const bool need = lane < 7u && (low ? !(x >= rec) : !(x <= rec));
    if (need) {
        float *p = chunk + (size_t)(row / (u32)kChunkRows) * 8u + lane;
        if (low) fatomic_min(p, x);
        else fatomic_max(p, x);
    }
}

// Bounds of a group of rows (a wavefront's) that classify_cam evaluates:
// the box of their stored centres and the largest mu, position drift and
// sigma_max^2 of their RowPre.  wave_sure_out(box, camera) is true only when
// classify_cam returns 0 for every row of the group, so every one is culled.
// It bounds the quantities classify_cam computes per row, over the group,
// with twice its rounding margins:
//   camera-space x, y, z over the box: the centre transform's range, each
//     coordinate's term at the end of the box that minimises / maximises it;
//   1/z between 1/zhi and 1/zlo of the group, so x/z is bounded at the
//     group's z ends by the sign of x (x/z rises with x and, for x >= 0,
//     falls with z; for x < 0 it rises with z);
//   the footprint radius at the group's smallest z and largest sigma.
// A group that may reach z <= 0 is not decided, as classify_cam leaves such
// a row to the exact test.
struct WaveBox {
    float lo[3], hi[3];
    float mu, dp, sig2;
};

__device__ __forceinline__ bool wave_sure_out(const WaveBox &w, const CamK &c, const BandK &b)
{
    float rlo[3], rhi[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float lo = c.T[i], hi = c.T[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float e0 = c.R[3 * i + j] * w.lo[j], e1 = c.R[3 * i + j] * w.hi[j];
            lo += fminf(e0, e1);
            hi += fmaxf(e0, e1);
        }
        const float rs = i == 0 ? b.rs0 : (i == 1 ? b.rs1 : b.rs2);
        const float sx = fmaf(rs, w.mu, fabsf(c.T[i]));
        const float dx = rs * w.dp;
        const float ex = fmaf(3e-6f, sx + dx, dx) + 2e-6f;
        rlo[i] = lo - ex;
        rhi[i] = hi + ex;
    }
    if ((rhi[2] <= c.zn) | (rlo[2] >= c.zf)) return true;
    if (!(rlo[2] > 0.0f)) return false;
    // 1/z of every row lies in [izh, izl] (hardware reciprocal, widened)
    const float izl = __builtin_amdgcn_rcpf(rlo[2]) * 1.00001f, izh = __builtin_amdgcn_rcpf(rhi[2]) * 0.99999f;
    const float S = ((b.jf2 * izl) * izl) * w.sig2;
    const float lam = fmaf(1.002f, S, 0.96f);
    const float rup = fmaf(3.004f, __builtin_amdgcn_sqrtf(lam) * 1.00001f, 1.001f);
    const float qxhi = rhi[0] >= 0.0f ? rhi[0] * izl : rhi[0] * izh;
    const float qxlo = rlo[0] < 0.0f ? rlo[0] * izl : rlo[0] * izh;
    const float qyhi = rhi[1] >= 0.0f ? rhi[1] * izl : rhi[1] * izh;
    const float qylo = rlo[1] < 0.0f ? rlo[1] * izl : rlo[1] * izh;
    const float eu = fmaf(2e-5f, fmaf(c.fx, fmaxf(fabsf(qxlo), fabsf(qxhi)), fabsf(c.cx)), 2e-3f);
    const float ev = fmaf(2e-5f, fmaf(c.fy, fmaxf(fabsf(qylo), fabsf(qyhi)), fabsf(c.cy)), 2e-3f);
    const float ulo = fmaf(c.fx, qxlo, c.cx) - eu, uhi = fmaf(c.fx, qxhi, c.cx) + eu;
    const float vlo = fmaf(c.fy, qylo, c.cy) - ev, vhi = fmaf(c.fy, qyhi, c.cy) + ev;
    return (uhi + rup <= 0.0f) | (ulo - rup >= c.W) | (vhi + rup <= 0.0f) | (vlo - rup >= c.H);
}

__device__ __forceinline__ float wave_min(float x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ float wave_max(float x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ u32 lane_rank(u64 mask)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

__device__ __forceinline__ u64 wave_sum_u64(u64 x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Step of a launch: the kernel argument, or (graph replay) the value at
// t_dev clamped to [1, T]; returns the table row of step t (+1 for a flush)
// and the largest defer count that row holds.
struct StepK {
    int32_t t, T, K, nrow;           // nrow: entries of a restore row
    const int32_t *t_dev;
    const float *lut;                // the two FP32 restore rows (slot 0, slot 1)
    gsdp::LutHeader *hdr;            // step held by each slot, error word
};

// The step of a launch (from the device counter when t_dev is set) and the
// restore row of step + extra: slot (step + extra) & 1 of the tables, whose
// header says which step it holds.  *err (uniform over the grid) is nonzero
// when the step lies outside [1, T] (bit 1) or the slot holds another step
// (bit 0); the step is then clamped for indexing, callers that store state
// skip their stores, and step_flag records the error in the header.
__device__ __forceinline__ int resolve_step(const StepK &s, int extra, const float **wrow, int *dmax, int *err)
{
    int t = s.t;                     // an explicit step was checked against [1, T] by the host
    int e = 0;
    if (s.t_dev) {
        t = *s.t_dev;
        if (t < 1 || t > s.T) {
            e = 2;
            t = t < 1 ? 1 : s.T;
        }
    }
    const int tr = t + extra;
    const int slot = tr & 1;
    if (s.hdr->t_row[slot] != tr) e |= 1;
    *err = e;
    *wrow = s.lut + (int64_t)slot * s.nrow;
    int64_t dm = tr - 1;
    if (s.K > 0 && dm > s.K) dm = s.K;
    *dmax = (int)dm;
    return t;
}

// Records a step error in the header's error word.  Kernels call it after
// their last load of model data: a store or atomic that may precede a load
// keeps the compiler from reading uniform data through the scalar cache.
__device__ __forceinline__ void step_flag(const StepK &s, int err)
{
    if (err) atomicOr(&s.hdr->error, err);
}

// ---------------------------------------------------------------------------
// cull + ordered compaction, in three launches without inter-block waits:
//   k_cull         one block per 512-row tile: cull every row, store the keep
//                  (and saturated) ballots and the tile's counts
//   k_tile_reduce  one wavefront per group of 64 tiles: the group's sums
//   k_tile_ids     one block per group: tile prefixes from the earlier
//                  groups' sums, then ids from ballots + tile prefix
// No same-address atomics and no spin-waits: on this multi-die part a
// device-scope atomic on one word serialises across all dies, which costs
// more than the two extra launches.
// ---------------------------------------------------------------------------
struct CullArgs {
    const float *gw;                 // [n][10]
    MomRef gm, gv;                   // G moments (restore), storage type gst
    int32_t gst, pad2;
    float rb, pad3;
    const int32_t *last;
    int64_t n;
    StepK step;
    float lr[10];
    float eps;
    CamK cam;
    BandK band;
    int32_t mode;                    // 0 exact restoring, 1 band
    int32_t geo_dense;               // geometry updated densely every step: never restore G
    int32_t K;                       // max_defer
    int32_t sgd;                     // SGD with momentum: restore w - (W lr) buf
    int32_t adamw, pad7;             // AdamW: decayed restore with the column's class tables
    const float *aw_base;
    int64_t aw_per, aw_nW;
    uint8_t cls[16];                 // rate class of G columns 0..9
    u64 *keep_bits;                  // [tiles][8] keep ballots of the tile's 64-row slabs
    u64 *sat_bits;                   // [tiles][8] saturated ballots (K > 0)
    u64 *tile_vs;                    // [tiles] visible << 32 | saturated
    u32 *tile_rest;                  // [tiles] restored rows
    int64_t tiles;
    const float4 *sum;               // [n] cull summaries (k_cull_sum)
    SideK side;                      // side_out constants (k_cull_sum)
    const CamPack *cams;             // camera table (k_cull_sum<..., true>): record (t - 1) % n_cams
    int32_t n_cams, pad9;
    const float4 *chunk;             // [chunks][2] chunk records (k_chunk_scan), or null
    u32 *chunk_flags;                // [chunks] k_chunk_scan's decisions (k_cull_sum), or null
    u64 *grp_vs, *grp_rest;          // group sums that k_chunk_scan clears and k_cull_sum adds to, or null
};

// Seven blocks per CU (the LDS tiles allow seven): the register budget this
// implies (72) keeps one more tile's loads in flight per CU than the six the
// kernel's natural register count allows; it spills a few registers of the
// rarely taken exact path.  NT: the sweep's loads are non-temporal (chosen
// when the swept arrays exceed the last-level cache; below that, the lines
// the sweep leaves cached serve the gather and the update that follow).
// the last-level (Infinity) cache of the part
constexpr int64_t kLastLevelCacheBytes = 256ll << 20;
template <bool NT>
__global__ __launch_bounds__(kCullBlock, 7) void k_cull(CullArgs a)
{
    __shared__ float4 sG4[kCullTile * 10 / 4];
    __shared__ u32 sCntV[kCullIpt * 4], sCntS[kCullIpt * 4];
    __shared__ u32 sRestored;
    float *sG = reinterpret_cast<float *>(sG4);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = blockIdx.x;
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    const int K = a.K;
    if (tid == 0) sRestored = 0;
    const int64_t row0 = tile * kCullTile;
    const int rows = (int)min((int64_t)kCullTile, a.n - row0);

    // stage the tile's geometry (rows x 40 B, contiguous) through LDS
    const int nf = rows * 10, nf4 = nf >> 2;
    const float *src = a.gw + row0 * 10;
    const float4 *src4 = reinterpret_cast<const float4 *>(src);
    int lastv[kCullIpt], dv[kCullIpt];
    float wdv[kCullIpt];
    // the rows' gaps and step-table entries (the table loads depend only on
    // the last steps, so on a full tile they are issued behind the geometry
    // loads and their latency hides under it)
    auto gaps = [&]() {
#pragma unroll
        for (int k = 0; k < kCullIpt; ++k) {
            int d = t - 1 - lastv[k];
            d = d < 0 ? 0 : (d > dmax ? dmax : d);
            dv[k] = d;
            // with dense geometry the stored G is always current
            wdv[k] = (d > 0 && !a.geo_dense) ? Wrow[d] : 0.0f;
        }
    };
    if (rows == kCullTile) {
        // full tile: every load of the thread is issued before the first one
        // is waited for (the tile is a few round trips of latency otherwise);
        // the last steps first, so waiting for them waits for nothing else
        constexpr int P = kCullTile * 10 / 4 / kCullBlock;
        static_assert(P * kCullBlock * 4 == kCullTile * 10, "tile is a whole number of float4 per thread");
#pragma unroll
        for (int k = 0; k < kCullIpt; ++k) lastv[k] = ld_sweep<NT>(a.last + row0 + k * kCullBlock + tid);
        __builtin_amdgcn_sched_barrier(0);
        float4 x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = ld_sweep<NT>(src4 + k * kCullBlock + tid);
        gaps();
#pragma unroll
        for (int k = 0; k < P; ++k) sG4[k * kCullBlock + tid] = x[k];
    } else {
        for (int j = tid; j < nf4; j += kCullBlock) sG4[j] = src4[j];
        for (int j = nf4 * 4 + tid; j < nf; j += kCullBlock) sG[j] = src[j];
#pragma unroll
        for (int k = 0; k < kCullIpt; ++k) {
            const int r = k * kCullBlock + tid;
            lastv[k] = r < rows ? a.last[row0 + r] : 0;
        }
        gaps();
    }
    __syncthreads();

    u32 nrest = 0;
#pragma unroll
    for (int k = 0; k < kCullIpt; ++k) {
        const int r = k * kCullBlock + tid;
        bool keep = false, sat = false;
        if (r < rows) {
            float g[10];
            const float2 *p2 = reinterpret_cast<const float2 *>(sG + r * 10);
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const float2 q = p2[j];
                g[2 * j] = q.x;
                g[2 * j + 1] = q.y;
            }
            const int d = dv[k];
            const float wd = wdv[k];
            const int cls = a.mode == 1 ? classify(g, wd, a.cam, a.band) : 2;
            if (cls == 2) {
                if (d > 0 && !a.geo_dense) {
                    const int64_t row = row0 + r;
                    float mv[10], vv[10];
                    if (a.sgd) {
                        // SGD with momentum (FP32 or BF16 buffer): w - (W lr) buf
                        if (a.gst == GS_F32) {
#pragma unroll
                            for (int j = 0; j < 10; ++j) g[j] = g[j] - (wd * a.lr[j]) * mom_load<GS_F32>(a.gm, row, j, false);
                        } else {
#pragma unroll
                            for (int j = 0; j < 10; ++j) g[j] = g[j] - (wd * a.lr[j]) * mom_load<GS_BF16>(a.gm, row, j, false);
                        }
                    } else {
                        if (a.gst == GS_F32) {
#pragma unroll
                            for (int j = 0; j < 10; ++j) {
                                mv[j] = mom_load<GS_F32>(a.gm, row, j, false);
                                vv[j] = mom_load<GS_F32>(a.gv, row, j, true);
                            }
                        } else if (a.gst == GS_BF16) {
#pragma unroll
                            for (int j = 0; j < 10; ++j) {
                                mv[j] = mom_load<GS_BF16>(a.gm, row, j, false);
                                vv[j] = mom_load<GS_BF16>(a.gv, row, j, true);
                            }
                        } else {
#pragma unroll
                            for (int j = 0; j < 10; ++j) {
                                mv[j] = mom_load<GS_FP8E4M3>(a.gm, row, j, false);
                                vv[j] = mom_load<GS_FP8E4M3>(a.gv, row, j, true);
                            }
                        }
                        if (a.adamw) {
                            const int64_t ro = (Wrow - a.step.lut) + d;
#pragma unroll
                            for (int j = 0; j < 10; ++j) {
                                const float *cb = a.aw_base + (int64_t)a.cls[j] * a.aw_per + ro;
                                g[j] = restore_w(g[j], mv[j], vv[j], cb[0], cb[a.aw_nW], a.lr[j], a.eps, a.rb);
                            }
                        } else {
#pragma unroll
                            for (int j = 0; j < 10; ++j)
                                g[j] = restore1(g[j], mv[j], vv[j], wd, a.lr[j], a.eps, a.rb);
                        }
                    }
                    ++nrest;
                }
                keep = cull_v1(g, a.cam);
            } else {
                keep = cls == 1;
            }
            sat = (K > 0) && !keep && d == K;
        }
        const u64 bv = __ballot(keep);
        const u64 bs = __ballot(sat);
        if (lane == 0) {
            const int slab = k * 4 + wave;   // rows row0 + slab*64 .. +63
            sCntV[slab] = (u32)__popcll(bv);
            sCntS[slab] = (u32)__popcll(bs);
            a.keep_bits[tile * gsdp::kWordsPerTile + slab] = bv;
            if (K > 0) a.sat_bits[tile * gsdp::kWordsPerTile + slab] = bs;
        }
    }
    if (nrest) atomicAdd(&sRestored, nrest);
    __syncthreads();
    if (tid == 0) {
        u32 sv = 0, ss = 0;
        for (int e = 0; e < kCullIpt * 4; ++e) {
            sv += sCntV[e];
            ss += sCntS[e];
        }
        a.tile_vs[tile] = ((u64)sv << 32) | (u64)ss;
        a.tile_rest[tile] = sRestored;
    }
    step_flag(a.step, step_err);
}

// The band cull from the cull summaries (Adam, geometry deferred).  A block
// takes TPB consecutive 512-row tiles, kCullIpt * TPB rows a thread: every
// row's summary (and, unless PACKED, its last step) is loaded first
// (coalesced, no LDS staging), then the rows are classified, a deferred one
// with the tables' bound of every restore coefficient.  The undecided rows
// (near a decision
// boundary, or flagged by their summary) are rare: one loop, not unrolled,
// loads each one's geometry row, restores it when deferred and takes the
// exact test.  Same outputs as k_cull, tile by tile.
constexpr int kCullSumTiles = 2;      // tiles of a k_cull_sum block (of 1, 2, 4, 8 the fastest at 40M rows)
// with chunk records (four tiles, two chunks, a block were slower: 21.2
// against 19.4 us at 40M rows in Morton order)
constexpr int kCullSumChunkTiles = 2;
static_assert(kCullSumTiles * kCullTile == kChunkRows, "a chunk is the tiles of a k_cull_sum block");

// True only when every row of a chunk is culled: classify_box returns 0 for
// each row with the RowPre of its summary at any defer count.  The record's
// box holds each row's centre, so each |coordinate| is at most the box's mu;
// each row's drift bound (kpos W + 1e-6 mu, W <= wbound) is at most the one
// formed from wbound and the box's mu; each row's largest log-scale after the
// restore (s + kscl W) is at most the record's s + kscl wbound, below 79 (so
// no row is undecidable) and widened by 1e-4 before the exponential.
// wave_sure_out then bounds what classify_box computes for each row.
__device__ __forceinline__ bool chunk_sure_out(const float4 &c0, const float4 &c1, float wbound, const CamK &cam,
                                               const BandK &band)
{
    const float smax = c0.w + band.kscl * wbound;
    if (!(smax < 79.0f)) return false;
    WaveBox w;
    w.lo[0] = c0.x;
    w.lo[1] = c0.y;
    w.lo[2] = c0.z;
    w.hi[0] = c1.x;
    w.hi[1] = c1.y;
    w.hi[2] = c1.z;
    w.mu = fmaxf(fmaxf(fmaxf(fabsf(c0.x), fabsf(c1.x)), fmaxf(fabsf(c0.y), fabsf(c1.y))),
                 fmaxf(fabsf(c0.z), fabsf(c1.z)));
    w.dp = band.kpos * wbound + 1e-6f * w.mu;
    const float sig = __expf(smax + 1e-4f) * 1.001f;
    w.sig2 = sig * sig;
    return wave_sure_out(w, cam, band);
}
// PACKED (steps up to 2^16): each row's defer count comes from the low 16
// bits of its summary word, and the last-step array is not read.  CAMDEV:
// the camera is record (t - 1) % n_cams of a device table (graph replay).
template <bool NT, int TPB, bool PACKED, bool CAMDEV>
__global__ __launch_bounds__(kCullBlock) void k_cull_sum(CullArgs a)
{
    constexpr int RPT = kCullIpt * TPB;
    static_assert(RPT <= 32, "row bits of a thread fit a word");
    __shared__ u32 sCntV[TPB][kCullIpt * 4], sCntS[TPB][kCullIpt * 4];
    __shared__ u32 sRestored[TPB];
    // chunks that k_chunk_scan skipped (it wrote their ballots and counts,
    // and records a step error) are neither loaded nor classified; a block
    // whose chunks are all skipped has nothing to do.  Tested first, so the
    // rows' loads wait for one load only.
    constexpr int CT = kChunkRows / kCullTile;      // tiles of a chunk
    static_assert(TPB % CT == 0, "a block covers whole chunks");
    constexpr int CPB = TPB / CT;                   // chunks of a block
    u32 live = (1u << CPB) - 1u;
    if (a.chunk_flags) {
        const int64_t nch = (a.tiles + CT - 1) / CT;
        live = 0;
#pragma unroll
        for (int h = 0; h < CPB; ++h) {
            const int64_t c = (int64_t)blockIdx.x * CPB + h;
            if (c < nch && !a.chunk_flags[c]) live |= 1u << h;
        }
        if (!live) return;
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile0 = (int64_t)blockIdx.x * TPB;
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    const int K = a.K;
    CamK cam;
    BandK band;
    SideK side;
    if (CAMDEV) {
        const CamPack &cp = a.cams[(t - 1) % a.n_cams];
        cam = cp.cam;
        band = cp.band;
        side = cp.side;
    } else {
        cam = a.cam;
        band = a.band;
        side = a.side;
    }
    if (tid < TPB) sRestored[tid] = 0;
    // row of slot q = j * kCullIpt + i: tile tile0 + j, rows i * kCullBlock + tid
    auto row_of = [&](int q) -> int64_t {
        return (tile0 + q / kCullIpt) * kCullTile + (int64_t)(q % kCullIpt) * kCullBlock + tid;
    };
    int lastv[RPT];
    float4 sv[RPT];
    u32 valid = 0;
    // every block but the last lies inside the model: no per-row clamps
    const bool full = (tile0 + TPB) * kCullTile <= a.n;
    const float4 *sb = a.sum + tile0 * kCullTile;
    const int32_t *lb = a.last + tile0 * kCullTile;
    if (full) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int o = (q / kCullIpt) * kCullTile + (q % kCullIpt) * kCullBlock + tid;
            lastv[q] = 0;
            sv[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if ((live >> (q / kCullIpt / CT)) & 1u) {
                valid |= 1u << q;
                if (!PACKED) lastv[q] = ld_sweep<NT>(lb + o);
                sv[q] = ld_sweep<NT>(sb + o);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t row = row_of(q);
            lastv[q] = 0;
            sv[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if ((live >> (q / kCullIpt / CT)) & 1u) {
                valid |= (u32)(row < a.n) << q;
                const int64_t rc = row < a.n ? row : a.n - 1;
                if (!PACKED) lastv[q] = ld_sweep<NT>(a.last + rc);
                sv[q] = ld_sweep<NT>(a.sum + rc);
            }
        }
    }
    // A deferred row is classified with the tables' bound of every restore
    // coefficient instead of its own W[d] (a looser band, no dependent load);
    // the exact test below uses the row's own W[d].
    const float wbound = a.step.hdr->wbound;
    int dv[RPT];
    float wdv[RPT];
    u32 qok = 0;                                          // the summaries' quaternion bits
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const u32 wb = __float_as_uint(sv[q].w);
        // t - 1 - last is in [0, 2^16) while the steps fit 16 bits
        int d = PACKED ? (int)(((u32)(t - 1) - wb) & 0xffffu) : t - 1 - lastv[q];
        d = d < 0 ? 0 : (d > dmax ? dmax : d);
        dv[q] = d;
        wdv[q] = d > 0 ? wbound : 0.0f;
        qok |= ((wb >> 16) & 1u) << q;
        sv[q].w = __uint_as_float(wb & 0xfffe0000u);      // s rounded up (or NaN)
    }
    // classification: keep bits and undecided bits of this thread's rows.
    // side_out settles most rows; the full classification runs for a slot
    // only where some lane's row is left (a uniform branch).
    u32 keepm = 0, und = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const RowPre pre = classify_pre_sum(sv[q], wdv[q], band, (qok >> q) & 1u);
        const bool left = !(pre.ok != 0 && side_out(sv[q], pre, cam, band, side)) && ((valid >> q) & 1u);
        if (__ballot(left) != 0ull) {
            const float c3[3] = {sv[q].x, sv[q].y, sv[q].z};
            const int cls = left ? classify_box(cam_box(c3, pre, cam, band), pre, cam, band) : 0;
            keepm |= (u32)(cls == 1) << q;
            und |= (u32)(cls == 2) << q;
        }
    }
    und &= valid;
    keepm &= valid;
    u32 nrest[TPB];
#pragma unroll
    for (int j = 0; j < TPB; ++j) nrest[j] = 0;
    // the exact test of the undecided rows
    u32 left = und;
#pragma unroll 1
    while (left) {
        const int q = __builtin_ctz(left);
        left &= left - 1u;
        const int64_t row = row_of(q);
        float g[10];
        const float2 *p2 = reinterpret_cast<const float2 *>(a.gw + row * 10);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const float2 v = p2[j];
            g[2 * j] = v.x;
            g[2 * j + 1] = v.y;
        }
        int d = t - 1 - a.last[row];
        d = d < 0 ? 0 : (d > dmax ? dmax : d);
        if (d > 0) {
            const float wd = Wrow[d];
            float mv[10], vv[10];
            if (a.gst == GS_F32) {
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    mv[j] = mom_load<GS_F32>(a.gm, row, j, false);
                    vv[j] = mom_load<GS_F32>(a.gv, row, j, true);
                }
            } else if (a.gst == GS_BF16) {
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    mv[j] = mom_load<GS_BF16>(a.gm, row, j, false);
                    vv[j] = mom_load<GS_BF16>(a.gv, row, j, true);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    mv[j] = mom_load<GS_FP8E4M3>(a.gm, row, j, false);
                    vv[j] = mom_load<GS_FP8E4M3>(a.gv, row, j, true);
                }
            }
#pragma unroll
            for (int j = 0; j < 10; ++j) g[j] = restore1(g[j], mv[j], vv[j], wd, a.lr[j], a.eps, a.rb);
#pragma unroll
            for (int j = 0; j < TPB; ++j) nrest[j] += (u32)(q / kCullIpt == j);
        }
        keepm |= (u32)cull_v1(g, cam) << q;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int j = q / kCullIpt, i = q % kCullIpt;
        const bool keep = (keepm >> q) & 1u;
        const u64 bv = __ballot(keep);
        u64 bs = 0;
        if (K > 0) bs = __ballot(((valid >> q) & 1u) && !keep && dv[q] == K);
        const int64_t tile = tile0 + j;
        if (lane == 0) {
            const int slab = i * 4 + wave;
            sCntV[j][slab] = (u32)__popcll(bv);
            sCntS[j][slab] = (u32)__popcll(bs);
            if (tile < a.tiles) {
                a.keep_bits[tile * gsdp::kWordsPerTile + slab] = bv;
                if (K > 0) a.sat_bits[tile * gsdp::kWordsPerTile + slab] = bs;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < TPB; ++j)
        if (nrest[j]) atomicAdd(&sRestored[j], nrest[j]);
    __syncthreads();
    if (tid < TPB && tile0 + tid < a.tiles) {
        u32 v = 0, ss = 0;
        for (int e = 0; e < kCullIpt * 4; ++e) {
            v += sCntV[tid][e];
            ss += sCntS[tid][e];
        }
        a.tile_vs[tile0 + tid] = ((u64)v << 32) | (u64)ss;
        a.tile_rest[tile0 + tid] = sRestored[tid];
        // with the chunk scan the group sums are added here (skipped chunks
        // add nothing), not summed by k_tile_reduce
        if (a.grp_vs) {
            const int64_t grp = (tile0 + tid) / gsdp::kGroupTiles;
            if (v | ss) atomicAdd(a.grp_vs + grp, ((u64)v << 32) | (u64)ss);
            if (sRestored[tid]) atomicAdd(a.grp_rest + grp, (u64)sRestored[tid]);
        }
    }
    step_flag(a.step, step_err);
}

// Summaries of rows [0, n) from the stored geometry (grid-stride, one row a
// thread).
__global__ __launch_bounds__(256) void k_cull_summary_build(const float *gw, const int32_t *last, float4 *sum,
                                                            int64_t n)
{
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
        float g[10];
        const float2 *p2 = reinterpret_cast<const float2 *>(gw + r * 10);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const float2 q = p2[j];
            g[2 * j] = q.x;
            g[2 * j + 1] = q.y;
        }
        sum[r] = cull_summary(g, last[r]);
    }
}

// Chunk records of the summaries, tight: one block per chunk, four rows a
// thread; the box of the centres and the largest s, a NaN s when any row's
// summary s is a NaN (then its centre may be anything, and is left out).
__global__ __launch_bounds__(256) void k_cull_chunk_build(const float4 *sum, int64_t n, float *chunk)
{
    __shared__ float sRed[4][8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kChunkRows;
    const float inf = __builtin_huge_valf();
    float lo[3] = {inf, inf, inf}, hi[3] = {-inf, -inf, -inf}, smax = -inf;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kChunkRows / 256; ++k) {
        const int64_t r = r0 + k * 256 + tid;
        if (r < n) {
            const float4 v = sum[r];
            const float sv = __uint_as_float(__float_as_uint(v.w) & 0xfffe0000u);
            if (sv == sv) {
                lo[0] = fminf(lo[0], v.x);
                lo[1] = fminf(lo[1], v.y);
                lo[2] = fminf(lo[2], v.z);
                hi[0] = fmaxf(hi[0], v.x);
                hi[1] = fmaxf(hi[1], v.y);
                hi[2] = fmaxf(hi[2], v.z);
                smax = fmaxf(smax, sv);
            } else {
                bad = true;
            }
        }
    }
    const bool any_bad = __ballot(bad) != 0ull;
    float red[8];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        red[i] = wave_min(lo[i]);
        red[4 + i] = wave_max(hi[i]);
    }
    red[3] = any_bad ? __builtin_nanf("") : wave_max(smax);
    red[7] = 0.0f;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 8; ++i) sRed[wave][i] = red[i];
    __syncthreads();
    if (tid < 8) {
        float x = sRed[0][tid];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
            const float y = sRed[w][tid];
            if (tid == 3) x = (x != x || y != y) ? __builtin_nanf("") : fmaxf(x, y);
            else if (tid < 3) x = fminf(x, y);
            else if (tid < 7) x = fmaxf(x, y);
        }
        chunk[blockIdx.x * 8ull + tid] = x;
    }
}

// The summary cull's chunk decisions, one thread a chunk, launched before
// k_cull_sum (with max_defer 0 and chunk records): flags[c] = 1 when chunk
// c's record shows every row culled; this thread then writes the zero
// ballots and counts of the chunk's tiles, and block c of k_cull_sum returns
// at once.  (One launch over the chunks costs less than the test in every
// k_cull_sum block, which would hold back the block's loads.)
template <bool CAMDEV>
__global__ __launch_bounds__(256) void k_chunk_scan(CullArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t chunks = (a.n + kChunkRows - 1) / kChunkRows;
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    CamK cam;
    BandK band;
    if (CAMDEV) {
        const CamPack &cp = a.cams[(t - 1) % a.n_cams];
        cam = cp.cam;
        band = cp.band;
    } else {
        cam = a.cam;
        band = a.band;
    }
    const float wbound = a.step.hdr->wbound;
    if (c >= chunks) return;
    // the group sums k_cull_sum adds to start at zero (fewer groups than chunks)
    if (a.grp_vs && c < (a.tiles + gsdp::kGroupTiles - 1) / gsdp::kGroupTiles) {
        a.grp_vs[c] = 0ull;
        a.grp_rest[c] = 0ull;
    }
    const bool skip = chunk_sure_out(a.chunk[2 * c], a.chunk[2 * c + 1], wbound, cam, band);
    a.chunk_flags[c] = skip ? 1u : 0u;
    // (the error is the same in every thread; k_cull_sum's skipped blocks do
    // not record it)
    if (c == 0) step_flag(a.step, step_err);
    if (!skip) return;
#pragma unroll
    for (int j = 0; j < kChunkRows / kCullTile; ++j) {
        const int64_t tile = c * (kChunkRows / kCullTile) + j;
        if (tile < a.tiles) {
            ulonglong2 *kb = reinterpret_cast<ulonglong2 *>(a.keep_bits + tile * gsdp::kWordsPerTile);
#pragma unroll
            for (int w = 0; w < gsdp::kWordsPerTile / 2; ++w) kb[w] = make_ulonglong2(0ull, 0ull);
            a.tile_vs[tile] = 0ull;
            a.tile_rest[tile] = 0u;
        }
    }
}

// flags[c] = 1 when the summary cull skips chunk c for this camera (the
// decision k_chunk_scan takes), one thread a chunk.
__global__ __launch_bounds__(256) void k_chunk_flags(const float4 *chunk, int64_t chunks,
                                                     const gsdp::LutHeader *hdr, CamK cam, BandK band,
                                                     uint8_t *flags)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= chunks) return;
    flags[c] = (uint8_t)chunk_sure_out(chunk[2 * c], chunk[2 * c + 1], hdr->wbound, cam, band);
}

// Block scans used by the one-block counter scans of the batched cull and of
// densification.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 7;           // 56 KB of LDS per chunk
constexpr int kScanChunk = kScanThreads * kScanPer;

__device__ __forceinline__ u64 block_excl_scan_u64(u64 x, u64 *sWave, u64 *total)
{
    // inclusive scan within the wave, then over the 16 wave totals
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u64 inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = (u64)__shfl_up((long long)inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sWave[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 run = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            const u64 v = sWave[w];
            sWave[w] = run;
            run += v;
        }
        sWave[kScanThreads / 64] = run;
    }
    __syncthreads();
    *total = sWave[kScanThreads / 64];
    const u64 r = sWave[wave] + inc - x;
    __syncthreads();                 // sWave may be reused by the caller's next scan
    return r;
}

// Exclusive prefix of one u32 count per tile, by the whole block, through LDS
// in chunks (coalesced loads and stores); returns the total.  sV holds
// kScanChunk entries, sWave kScanThreads/64 + 1.
__device__ u64 scan_counts_u32(const u32 *cnt, u32 *off, int64_t tiles, u64 *sV, u64 *sWave)
{
    const int tid = threadIdx.x;
    u64 carry = 0;
    for (int64_t c0 = 0; c0 < tiles; c0 += kScanChunk) {
        const int64_t nc = min((int64_t)kScanChunk, tiles - c0);
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const int64_t i = (int64_t)q * kScanThreads + tid;
            sV[i] = i < nc ? (u64)cnt[c0 + i] : 0ull;
        }
        __syncthreads();
        u64 v[kScanPer], sum = 0;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            v[q] = sV[tid * kScanPer + q];
            sum += v[q];
        }
        u64 tot = 0;
        u64 run = carry + block_excl_scan_u64(sum, sWave, &tot);
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            sV[tid * kScanPer + q] = run;
            run += v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const int64_t i = (int64_t)q * kScanThreads + tid;
            if (i < nc) off[c0 + i] = (u32)sV[i];
        }
        carry += tot;
        __syncthreads();
    }
    return carry;
}

// Prefix of the tile counts in two launches of many blocks.  k_tile_reduce:
// one wavefront per group of 64 tiles sums its (visible, saturated) and
// restored counts.  k_tile_ids: one block per group adds the sums of all
// earlier groups (read from L2), scans its 64 tiles in one wavefront, stores
// the tile prefixes, and then writes the visible (and saturated) ids of its
// tiles in ascending order from the ballots, one wavefront per tile; the last
// group's block writes the totals.  Up to kDirectTiles tiles (8M rows) the
// group sums are skipped: each k_tile_ids block sums the counts of all
// earlier tiles itself (at most 32 loads per thread, from L2), which costs
// less than the second launch.
constexpr int64_t kDirectTiles = 16384;
struct IdsArgs {
    const u64 *keep_bits, *sat_bits;
    const u64 *tile_vs;              // visible << 32 | saturated of each tile
    const u32 *tile_rest;
    u64 *tile_off;                   // visible << 32 | saturated before the tile
    u64 *grp_vs, *grp_rest;          // per group of 64 tiles
    int64_t tiles, groups, n;
    u32 *ids;
    u32 cap;
    int32_t direct;                  // sum earlier tiles directly (no group sums)
    u32 *sat_ids;
    u32 *count;
    gsdp::WsHeader *hdr;
};

__global__ __launch_bounds__(256) void k_tile_reduce(IdsArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= a.groups) return;
    const int64_t tile = g * gsdp::kGroupTiles + lane;
    u64 vs = 0, rest = 0;
    if (tile < a.tiles) {
        vs = a.tile_vs[tile];
        rest = a.tile_rest[tile];
    }
    vs = wave_sum_u64(vs);
    rest = wave_sum_u64(rest);
    if (lane == 0) {
        a.grp_vs[g] = vs;
        a.grp_rest[g] = rest;
    }
}

// one thread per 64-row ballot word of a group of 64 tiles
constexpr int kIdsThreads = gsdp::kGroupTiles * gsdp::kWordsPerTile;

// Store the ids of the set bits of this lane's word `m` (rows row0 + bit) at
// out[p ...] in ascending order, positions from `cap` on dropped.  Words with
// up to kIdsSerial bits are written by their own lane (the lanes in step, as
// long as the fullest of them); each word with more is written by the whole
// wavefront (lane b stores row b at p + the number of lower set bits), one
// word after another.  Rows in no order give words of a few bits (5.6 on
// average at 8.7 % visible), rows in a spatial order empty and full words.
// Every lane of the wavefront calls it.
constexpr int kIdsSerial = 16;
__device__ __forceinline__ void write_word_ids(u64 m, u32 p, int64_t row0, u32 *out, u32 cap, int lane)
{
    const bool dense = __popcll(m) > kIdsSerial;
    if (!dense)
        for (u64 r = m; r; r &= r - 1ull, ++p)
            if (p < cap) out[p] = (u32)(row0 + __builtin_ctzll(r));
    u64 dw = __ballot(dense);
    const u64 below = (1ull << lane) - 1ull;
    while (dw) {
        const int j = __builtin_ctzll(dw);
        dw &= dw - 1ull;
        const u64 wj = ((u64)(u32)__builtin_amdgcn_readlane((int)(u32)(m >> 32), j) << 32) |
                       (u64)(u32)__builtin_amdgcn_readlane((int)(u32)m, j);
        const u32 pj = (u32)__builtin_amdgcn_readlane((int)p, j);
        const int64_t rj = row0 + (int64_t)(j - lane) * 64;
        if ((wj >> lane) & 1ull) {
            const u32 q = pj + (u32)__popcll(wj & below);
            if (q < cap) out[q] = (u32)(rj + lane);
        }
    }
}

template <bool DIRECT>
__global__ __launch_bounds__(kIdsThreads) void k_tile_ids(IdsArgs a)
{
    constexpr int NW = kIdsThreads / 64;
    __shared__ u64 sRed[3][NW];
    __shared__ u64 sWave[NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t g = blockIdx.x;
    const bool last = g == (a.groups > 0 ? a.groups - 1 : 0);
    // this thread's word (keep and saturated ballots of 64 rows), loaded
    // first: it does not depend on the prefix, so its latency overlaps the
    // sums below
    const int64_t t0 = g * gsdp::kGroupTiles;
    const int64_t word = t0 * gsdp::kWordsPerTile + tid;
    const bool has = g < a.groups && word < a.tiles * gsdp::kWordsPerTile;
    u64 kw = 0ull, sw = 0ull;
    if (has) {
        kw = a.keep_bits[word];
        if (a.sat_ids) sw = a.sat_bits[word];
    }
    u64 base = 0, rest = 0, own = 0;
    if (DIRECT) {
        // sums of the earlier tiles (the last block: of all tiles, its own
        // group's apart), sixteen independent loads per thread per round (one
        // round up to 8192 tiles)
        const int64_t upto = last ? a.tiles : t0;
        for (int64_t i0 = tid; i0 < upto; i0 += 16 * kIdsThreads) {
            u64 c[16];
            u32 r[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int64_t i = i0 + (int64_t)k * kIdsThreads;
                const int64_t ic = i < upto ? i : 0;
                c[k] = a.tile_vs[ic];
                r[k] = last ? a.tile_rest[ic] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int64_t i = i0 + (int64_t)k * kIdsThreads;
                if (i < upto) {
                    if (i < t0) base += c[k];
                    else own += c[k];
                    rest += r[k];
                }
            }
        }
    } else {
        // sums of the earlier groups (and, for the last block, of all groups)
        const int64_t upto = last ? a.groups : g;
        for (int64_t i = tid; i < upto; i += kIdsThreads) {
            if (i < g) base += a.grp_vs[i];
            if (last) rest += a.grp_rest[i];
        }
    }
    base = wave_sum_u64(base);
    rest = wave_sum_u64(rest);
    own = wave_sum_u64(own);
    // inclusive scan of the words' (visible << 32 | saturated) counts
    const u64 c = ((u64)__popcll(kw) << 32) | (u64)__popcll(sw);
    u64 inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = (u64)__shfl_up((long long)inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 0) {
        sRed[0][wave] = base;
        sRed[1][wave] = rest;
        sRed[2][wave] = own;
    }
    if (lane == 63) sWave[wave] = inc;
    __syncthreads();
    base = 0;
    u64 rsum = 0, osum = 0, before = 0, gsum = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        base += sRed[0][w];
        rsum += sRed[1][w];
        osum += sRed[2][w];
        before += w < wave ? sWave[w] : 0ull;
        gsum += sWave[w];
    }
    if (last && tid == 0) {
        // the last block also knows every total
        const u64 tot = base + (DIRECT ? osum : (g < a.groups ? a.grp_vs[g] : 0ull));
        const u32 vis = (u32)(tot >> 32);
        *a.count = vis;
        a.hdr->vis_total = vis;
        a.hdr->sat_total = (u32)tot;
        a.hdr->restored_last = (u32)rsum;
        a.hdr->vis_accum += vis;
        a.hdr->restored_accum += rsum;
    }
    (void)gsum;
    // exclusive prefix of this word: earlier groups + earlier words of the
    // group (lanes past the last word have no bits and store nothing, but
    // stay: the wavefront writes dense words together)
    const u64 pre = base + before + inc - c;
    if (has && (tid % gsdp::kWordsPerTile) == 0) a.tile_off[t0 + tid / gsdp::kWordsPerTile] = pre;
    // ids of the word's set bits, ascending: a word with a few bits by its
    // own thread, a word with many (rows in a spatial order, close views)
    // by the whole wavefront, one lane a row, so the stores are contiguous
    const int64_t row0 = word * 64;
    const u32 pv0 = (u32)(pre >> 32), ps0 = (u32)pre;
    write_word_ids(kw, pv0, row0, a.ids, a.cap, lane);
    if (a.sat_ids) write_word_ids(sw, ps0, row0, a.sat_ids, 0xffffffffu, lane);
}

// ---------------------------------------------------------------------------
// row kernels: gather / adam / flush
// ---------------------------------------------------------------------------
enum RowMode { kGather = 0, kAdam = 1, kFlush = 2, kAdamMax = 3 };
// rows per wavefront iteration: the gather (fewer loads a row, fewer
// registers) runs faster with two, the update passes with four
template <int MODE>
constexpr int row_unroll() { return MODE == kGather ? 2 : 4; }

// The update of step t also moves the tables' restore rows to step t + 1:
// every row deferred d steps at t is deferred d + 1 steps at t + 1 and has
// also skipped step t, so (entries d = 0 .. min(t, Dn) - 1)
//   W'[d+1] = W[d] + R[d] Cn[t]                      W'[0] = 0
//   Wl'[d+1] = q[t] Wl[d] + R[d] Cn[t],  P'[d+1] = q[t] P[d]   (AdamW classes)
// in FP64 from the FP64 rows of slot t & 1 into slot (t+1) & 1, each entry
// rounded once to FP32 beside it.  The update kernel reads slot t & 1 only,
// so its threads do this (entries i0, i0 + stride, ...) beside their rows.
struct LutAdv {
    double *Wd;                      // [2][nrow]
    float *Wf;                       // [2][nrow]
    const double *R, *Cn;
    char *cls;                       // first AdamW class block
    int64_t cls_bytes, cWlf, cPf, cWld, cPd, cqd;
    int32_t nclass, on;              // on: this launch advances the tables
};

__device__ __forceinline__ void lut_advance_slice(const LutAdv &a, const StepK &s, int t, int64_t i0,
                                                  int64_t stride)
{
    const int64_t nrow = s.nrow;
    const int64_t so = (int64_t)(t & 1) * nrow, sn = (int64_t)((t + 1) & 1) * nrow;
    const int64_t dn = (int64_t)t < nrow - 1 ? (int64_t)t : nrow - 1;
    const double c = a.Cn[t];
    for (int64_t i = i0; i <= dn; i += stride) {
        double w = 0.0;
        if (i > 0) w = a.Wd[so + i - 1] + a.R[i - 1] * c;
        a.Wd[sn + i] = w;
        a.Wf[sn + i] = (float)w;
        for (int cl = 0; cl < a.nclass; ++cl) {
            char *b = a.cls + cl * a.cls_bytes;
            double *Wl = reinterpret_cast<double *>(b + a.cWld), *P = reinterpret_cast<double *>(b + a.cPd);
            const double q = reinterpret_cast<const double *>(b + a.cqd)[t];
            double l = 0.0, p = 1.0;
            if (i > 0) {
                l = q * Wl[so + i - 1] + a.R[i - 1] * c;
                p = q * P[so + i - 1];
            }
            Wl[sn + i] = l;
            P[sn + i] = p;
            reinterpret_cast<float *>(b + a.cWlf)[sn + i] = (float)l;
            reinterpret_cast<float *>(b + a.cPf)[sn + i] = (float)p;
        }
    }
    if (i0 == 0) s.hdr->t_row[(t + 1) & 1] = t + 1;
}

struct RowArgs {
    float *gw, *aw;
    int64_t gw_ld, aw_ld;
    MomRef gm, gv, am, av;
    int32_t adim, pad3;
    StepK step;
    float lr[64];                    // lane-indexed: 0..9 G, 10.. A
    float eps, omb1, omb2, rb;       // rb: clamp of the restore factor and of the Adam step
    u64 sr_seed;
    int32_t geo_dense, pad6;
    // the optimizer is a template parameter of the kernel; for AdamW:
    const float *aw_base;            // first class's tables
    int64_t aw_per, aw_nW;           // floats per class, floats of one W layout
    uint8_t cls[64];                 // rate class of each lane
    int32_t *last;
    int64_t n;
    const float *Mf, *Vf, *SS, *BC;
    const u32 *ids, *count;
    u32 cap, pad1;
    const u32 *sat_ids, *sat_count;
    const float *g_geo, *g_app;      // compact gradients
    float *gd_geo, *gd_app;          // dense gradients (read and cleared)
    float *out_geo, *out_app;        // gather outputs
    u32 *fp8max[4];                  // per-block max |m'|, sqrt(v') that outgrew the scale (G m, G v, A m, A v)
    u32 *fp8list, *fp8count;         // tasks (moment * nb + block) that outgrew their scale, and their count
    int64_t nb;
    // fused layout: A w, A m, A v, G m and G v of a row lie in one byte row of
    // fz_s bytes starting at aw (offsets in bytes); the kernel then addresses
    // them all from one row base
    u32 fz_s, fz_ogm, fz_ogv, fz_oam, fz_oav, pad8;
    LutAdv adv;                      // kAdam: the tables' advance to the next step
    float4 *cull_sum;                // [n] cull summaries kept current (or null)
    float *cull_chunk;               // their chunk records, widened (or null)
};

// One wavefront per Gaussian row: lane c < 10 owns G column c, lane 10+c owns
// A column c.  GST / AST are the moment storage types of G and A.
//   kGather   current values into compact buffers (read-only)
//   kAdam     restore + Adam step + stores, last_step = t
//   kFlush    catch-up of deferred rows
//   kAdamMax  first pass for FP8 moments: new moments only, recording per
//             block the largest magnitude that no longer fits the block scale
// FZ: the fused layout with one storage type for both groups; the moments of
// every lane are then one access from the row's single base.
template <int MODE, int GST, int AST, int OPT, bool FZ>
__device__ __forceinline__ void rows_work(const RowArgs &a, const int t, const float *const Wrow, const int dmax)
{
    constexpr int kRU = row_unroll<MODE>();
    const int lane = threadIdx.x & 63;
    // the wavefront index is uniform: keep it (and so every row index and row
    // id below) in scalar registers
    // Row counts, positions and ids fit 31 bits (checked with the model) and
    // are kept 32-bit: comparisons and products of them then stay on the
    // scalar unit.
    const u32 wid = blockIdx.x * 4u + (u32)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const u32 nw = gridDim.x * 4u;
    const bool isG = lane < 10;
    // with dense geometry, G columns are updated elsewhere and never deferred
    const bool act = lane < 10 + a.adim && !(isG && a.geo_dense && MODE != kGather);
    const bool grest = !(isG && a.geo_dense);
    constexpr bool sgd = OPT == GS_OPT_SGD_MOMENTUM;
    constexpr bool adamw = OPT == GS_OPT_ADAMW;
    const int ca = lane - 10;
    // Lanes past the last column load (but never store) the last column, so
    // that the loads need no lane mask: a row's loads are then one uniform
    // branch, not a mask of lanes.
    const int col = isG ? lane : (ca < a.adim ? ca : a.adim - 1);
    // Addressing: a row's base in each array is wave-uniform (scalar
    // registers); each lane adds a 32-bit byte offset of its column that is
    // fixed for the whole launch.  G and A lanes take their loads and stores
    // in two exec-masked halves, so no per-lane 64-bit address arithmetic.
    const u32 off4 = (u32)col * 4u;
    const u32 offm = (u32)col * (u32)(isG ? msize<GST>() : msize<AST>());
    // row strides in bytes (a row is at most a few KB)
    const u32 sGW = (u32)a.gw_ld * 4u, sAW = (u32)a.aw_ld * 4u;
    const u32 sGM = (u32)a.gm.ld * msize<GST>(), sGV = (u32)a.gv.ld * msize<GST>();
    const u32 sAM = (u32)a.am.ld * msize<AST>(), sAV = (u32)a.av.ld * msize<AST>();
    const u32 sAG = (u32)a.adim * 4u;
    static_assert(!FZ || GST == AST, "the fused single access needs one storage type");
    const u32 fzm = isG ? a.fz_ogm + (u32)col * msize<GST>() : a.fz_oam + (u32)col * msize<AST>();
    const u32 fzv = isG ? a.fz_ogv + (u32)col * msize<GST>() : a.fz_oav + (u32)col * msize<AST>();
    // element of row r (stride s bytes) at this lane's byte offset o; the row
    // base goes through srow, so it stays a scalar base of the access
    auto elem = [](const void *p, u64 r, u32 s, u32 o) { return (char *)(srow(p, r, s) + lane_off(o)); };
    // the same at a row base already computed
    auto at = [](gchar *b, u32 o) { return (char *)(b + lane_off(o)); };
    const float lr = a.lr[lane];
    // AdamW: this lane's rate class tables, same row offset as Wrow
    const float *WlRow = Wrow, *PRow = Wrow;
    float qdec = 1.0f;
    if (adamw) {
        const float *cb = a.aw_base + (int64_t)a.cls[lane] * a.aw_per;
        const int64_t ro = Wrow - a.step.lut;
        WlRow = cb + ro;
        PRow = cb + a.aw_nW + ro;
        qdec = cb[2 * a.aw_nW + t];
    }

    // an empty model has no row 0 for the clamped loads below
    if (a.n <= 0) return;
    const u32 n = (u32)a.n;
    u32 nvis, total;
    if (MODE == kFlush) {
        nvis = n;
        total = n;
    } else {
        const u32 c = *a.count;
        nvis = c < a.cap ? c : a.cap;
        total = nvis + (((MODE == kAdam || MODE == kAdamMax) && a.sat_count) ? *a.sat_count : 0u);
    }
    float ss = 0.0f, bc = 1.0f;
    if (MODE == kAdam) {
        ss = a.SS[t];
        bc = a.BC[t];
    }
    const float step = lr * ss;
    // the rescale (previous launch) has consumed the task list of this step
    if (MODE == kAdam && a.fp8count && blockIdx.x == 0 && threadIdx.x == 0) *a.fp8count = 0u;
    const bool quant = (GST != GS_F32) || (AST != GS_F32);
    const u64 s_step = quant ? sm_at(a.sr_seed, (u64)t) : 0ull;

    // Software pipeline over iterations of kRU rows: while one
    // iteration's state is loaded, the next iteration's last steps and the
    // ids of the one after are loaded too, so an iteration waits for one
    // round of memory latency instead of three (ids -> last step -> state).
    // The prefetched words are loaded at an index plus a zero that the
    // compiler must treat as per-lane, so they stay in vector registers and
    // are waited for where they are moved to scalar registers, at the end of
    // the iteration, not right after the load.  Positions past the end give
    // ok = false and row 0 / the last position (clamped indices: no load sits
    // behind a branch).  Rows are unique within a launch, so reading a later
    // row's last step before this iteration's stores is safe.
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    const u32 stride = nw * kRU;
    // positions past nvis index the saturated list (only rows in range are
    // ever read through it)
    const u32 *sat_base = a.sat_ids ? a.sat_ids - nvis : a.ids;
    auto fetch_raw = [&](u32 b, u32 *rid) {
        if (MODE == kFlush) return;
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            const u32 i = min(b + u, total - 1u);
            rid[u] = (i < nvis ? a.ids : sat_base)[i + vzero];
        }
    };
    auto decode = [&](u32 b, const u32 *rid, u32 *idv, bool *okv) {
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            const u32 r = MODE == kFlush ? b + u : (u32)__builtin_amdgcn_readfirstlane((int)rid[u]);
            okv[u] = b + u < total && r < n;
            idv[u] = okv[u] ? r : 0u;
        }
    };
    auto gap = [&](int lastv, bool okv) {
        const int l = __builtin_amdgcn_readfirstlane(lastv);
        int dd = (MODE == kFlush) ? t - l : t - 1 - l;
        dd = dd < 0 ? 0 : (dd > dmax ? dmax : dd);
        return okv ? dd : 0;
    };
    u32 id[kRU], idn[kRU];
    bool ok[kRU], okn[kRU];
    int d[kRU];
    u32 rid[kRU], ridn[kRU];
    u32 base = wid * kRU;
    if (base < total) {
        fetch_raw(base, rid);
        decode(base, rid, id, ok);
        int lastv[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) lastv[u] = a.last[id[u] + vzero];
        fetch_raw(base + stride, ridn);
#pragma unroll
        for (int u = 0; u < kRU; ++u) d[u] = gap(lastv[u], ok[u]);
        decode(base + stride, ridn, idn, okn);
    }
    for (; base < total; base += stride) {
        int lastn[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) lastn[u] = a.last[idn[u] + vzero];
        u32 ridnn[kRU];
        fetch_raw(base + 2 * stride, ridnn);
        // Raw words first (every row's loads in flight), selected and decoded
        // afterwards.  The G and A halves load into separate registers that
        // start undefined: a write of a default value to a register with a
        // load of the other half still pending would have to wait for it.
        u32 Gw[kRU], Gg[kRU], Aw[kRU], Ag[kRU];
        typename RawT<GST>::T Gm[kRU], Gv[kRU];
        typename RawT<AST>::T Am[kRU], Av[kRU];
        float ms[kRU], vs[kRU];
        // Row bases of the weight rows (the fused rows too: their stride is
        // the A row's), computed once and kept for the stores; the compact
        // gradient rows of the iteration are consecutive, at constant offsets
        // from the first.
        gchar *rA[kRU], *rG[kRU];
        float crec[kRU];                 // chunk record elements (summary writers)
        gchar *const cG = srow(a.g_geo, base, 40u), *const cA = srow(a.g_app, base, sAG);
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            Gw[u] = undef_v<u32>();
            Gg[u] = undef_v<u32>();
            Aw[u] = undef_v<u32>();
            Ag[u] = undef_v<u32>();
            Gm[u] = undef_v<typename RawT<GST>::T>();
            Gv[u] = undef_v<typename RawT<GST>::T>();
            Am[u] = undef_v<typename RawT<AST>::T>();
            Av[u] = undef_v<typename RawT<AST>::T>();
            const u64 ru = (u64)id[u];
            rA[u] = srow(a.aw, ru, sAW);
            rG[u] = srow(a.gw, ru, sGW);
            float gms = 0.0f, gvs = 0.0f, ams = 0.0f, avs = 0.0f;
            if (GST == GS_FP8E4M3 || AST == GS_FP8E4M3) {
                const u64 b = ru / kFp8Block;
                if (GST == GS_FP8E4M3) {
                    gms = a.gm.s[b];
                    gvs = a.gv.s[b];
                }
                if (AST == GS_FP8E4M3) {
                    ams = a.am.s[b];
                    avs = a.av.s[b];
                }
            }
            ms[u] = isG ? gms : ams;
            vs[u] = isG ? gvs : avs;
            const bool need = ok[u] && (MODE != kFlush || d[u] > 0);
            // the gather and Adam read the moments of every row (most visible
            // rows are deferred); the flush only those it catches up
            const bool ldm = MODE == kAdam || MODE == kAdamMax || MODE == kGather || d[u] > 0;
            const bool ldg = (MODE == kAdam || MODE == kAdamMax) && base + u < nvis;
            crec[u] = 0.0f;
            if (!need) continue;
            if ((MODE == kAdam || MODE == kFlush) && a.cull_chunk) crec[u] = chunk_rec_lane(a.cull_chunk, id[u]);
            // (with dense geometry the G moments are current: loading them is
            // harmless, and no lane mask is needed)
            if (FZ && ldm) {
                Gm[u] = mraw<GST>(at(rA[u], fzm));
                if (!sgd) Gv[u] = mraw<GST>(at(rA[u], fzv));
            }
            if (isG) {
                if (MODE != kAdamMax) Gw[u] = *reinterpret_cast<const u32 *>(at(rG[u], off4));
                if (!FZ && ldm && !a.geo_dense) {
                    Gm[u] = mraw<GST>(elem(a.gm.p, ru, sGM, offm));
                    if (!sgd) Gv[u] = mraw<GST>(elem(a.gv.p, ru, sGV, offm));
                }
                if (ldg)
                    Gg[u] = a.g_geo ? *reinterpret_cast<const u32 *>(at(cG + 40u * u, off4))
                                    : *reinterpret_cast<const u32 *>(elem(a.gd_geo, ru, 40u, off4));
                // distinct markers end the two halves: otherwise the compiler
                // merges their accesses into one with a per-lane address
                asm volatile("; G columns");
            } else {
                if (MODE != kAdamMax) Aw[u] = *reinterpret_cast<const u32 *>(at(rA[u], off4));
                if (!FZ && ldm) {
                    Am[u] = mraw<AST>(elem(a.am.p, ru, sAM, offm));
                    if (!sgd) Av[u] = mraw<AST>(elem(a.av.p, ru, sAV, offm));
                }
                if (ldg)
                    Ag[u] = a.g_app ? *reinterpret_cast<const u32 *>(at(cA + sAG * u, off4))
                                    : *reinterpret_cast<const u32 *>(elem(a.gd_app, ru, sAG, off4));
                asm volatile("; A columns");
            }
        }
        // no instruction that waits for a load may be moved between the loads
        __builtin_amdgcn_sched_barrier(0);
        // values of lanes or rows that loaded nothing are never stored; a
        // saturated row (no compact gradient) takes g = 0
        float w[kRU], m[kRU], v[kRU], g[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            w[u] = __uint_as_float(isG ? Gw[u] : Aw[u]);
            const bool ldg = (MODE == kAdam || MODE == kAdamMax) && base + u < nvis;
            g[u] = ldg ? __uint_as_float(isG ? Gg[u] : Ag[u]) : 0.0f;
            if (FZ) {
                m[u] = mdec<GST>((u32)Gm[u], ms[u], false);
                v[u] = mdec<GST>((u32)Gv[u], vs[u], true);
            } else if (GST == AST) {
                m[u] = mdec<GST>(isG ? (u32)Gm[u] : (u32)Am[u], ms[u], false);
                v[u] = mdec<GST>(isG ? (u32)Gv[u] : (u32)Av[u], vs[u], true);
            } else {
                m[u] = isG ? mdec<GST>(Gm[u], ms[u], false) : mdec<AST>(Am[u], ms[u], false);
                v[u] = isG ? mdec<GST>(Gv[u], vs[u], true) : mdec<AST>(Av[u], vs[u], true);
            }
        }
        // table entries of each row's gap (issued after the state loads, which
        // do not depend on them)
        float Wd[kRU], Mfd[kRU], Vfd[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            Wd[u] = Wrow[d[u]];
            Mfd[u] = Vfd[u] = 0.0f;
            if (MODE == kAdam || MODE == kAdamMax || MODE == kFlush) {
                const int j = MODE == kFlush ? (d[u] > 0 ? d[u] - 1 : 0) : d[u];
                Mfd[u] = a.Mf[j];
                Vfd[u] = a.Vf[j];
            }
        }
        // FP8 max pass: tasks this iteration's rows list first (one
        // same-address atomic per iteration, not one per task)
        u32 newt[kRU][4];
#pragma unroll
        for (int u = 0; u < kRU; ++u)
#pragma unroll
            for (int k = 0; k < 4; ++k) newt[u][k] = 0xffffffffu;
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            if (!ok[u]) continue;
            const u32 r = id[u];
            if (MODE == kGather) {
                float x = w[u];
                if (d[u] > 0 && grest) {
                    if (sgd) x = x - (Wd[u] * lr) * m[u];
                    else if (adamw) x = restore_w(x, m[u], v[u], WlRow[d[u]], PRow[d[u]], lr, a.eps, a.rb);
                    else x = restore1(x, m[u], v[u], Wd[u], lr, a.eps, a.rb);
                }
                if (act) {
                    const u64 cp = (u64)(base + u);
                    if (isG) {
                        if (a.out_geo) *reinterpret_cast<float *>(elem(a.out_geo, cp, 40u, off4)) = x;
                    } else if (a.out_app) {
                        *reinterpret_cast<float *>(elem(a.out_app, cp, sAG, off4)) = x;
                    }
                }
                continue;
            }
            const int dd = d[u];
            if (MODE == kAdamMax) {
                const bool fp8 = isG ? GST == GS_FP8E4M3 : AST == GS_FP8E4M3;
                const u32 b = r / kFp8Block;
                u32 xm = 0u, xv = 0u;
                if (act && fp8) {
                    const float m1 = Mfd[u] * m[u] + a.omb1 * g[u];
                    const float v1 = Vfd[u] * v[u] + (a.omb2 * g[u]) * g[u];
                    const float r1 = sqrtf(v1);
                    const float am = fabsf(m1);
                    if (am > 448.0f * ms[u]) xm = __float_as_uint(am);
                    if (r1 > 448.0f * vs[u]) xv = __float_as_uint(r1);
                }
                // maxima over the group's lanes (non-negative floats order as
                // their bit patterns), then at most four atomics per row
                u32 mx[4] = {isG ? xm : 0u, isG ? xv : 0u, isG ? 0u : xm, isG ? 0u : xv};
#pragma unroll
                for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const u32 y = (u32)__shfl_xor((int)mx[k], o);
                        mx[k] = y > mx[k] ? y : mx[k];
                    }
                if (lane == 0)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (mx[k]) {
                            // the first record of a task this step lists it for the
                            // rescale (listed after the iteration's rows, below)
                            const u32 old = atomicMax(&a.fp8max[k][b], mx[k]);
                            if (old == 0u) newt[u][k] = (u32)(k * a.nb + b);
                        }
                continue;
            }
            if (MODE == kFlush && dd == 0) continue;
            float xs = 0.0f;                 // this lane's new value (for the summary)
            if (act) {
                float x, m1, v1;
                if (MODE == kAdam && sgd) {
                    // SGD with momentum: catch up, buf = mu^(d+1) buf + g, w -= (lr s_t) buf
                    x = w[u];
                    if (dd > 0) x = x - (Wd[u] * lr) * m[u];
                    m1 = Mfd[u] * m[u] + g[u];
                    v1 = 0.0f;
                    x = x - step * m1;
                } else if (MODE == kAdam && adamw) {
                    // AdamW: decayed catch-up, Adam moments, w = q_t w - step
                    x = w[u];
                    if (dd > 0) x = restore_w(x, m[u], v[u], WlRow[dd], PRow[dd], lr, a.eps, a.rb);
                    m1 = Mfd[u] * m[u] + a.omb1 * g[u];
                    v1 = Vfd[u] * v[u] + (a.omb2 * g[u]) * g[u];
                    const float xq = qdec * x;
                    x = xq - adam_step(m1, v1, step, bc, a.eps, a.rb);
                } else if (MODE == kAdam) {
                    x = w[u];
                    if (dd > 0) x = restore1(x, m[u], v[u], Wd[u], lr, a.eps, a.rb);
                    m1 = Mfd[u] * m[u] + a.omb1 * g[u];
                    v1 = Vfd[u] * v[u] + (a.omb2 * g[u]) * g[u];
                    x = x - adam_step(m1, v1, step, bc, a.eps, a.rb);
                } else if (adamw) {
                    x = restore_w(w[u], m[u], v[u], WlRow[dd], PRow[dd], lr, a.eps, a.rb);
                    m1 = Mfd[u] * m[u];
                    v1 = Vfd[u] * v[u];
                } else if (sgd) {
                    x = w[u] - (Wd[u] * lr) * m[u];
                    m1 = Mfd[u] * m[u];
                    v1 = 0.0f;
                } else {
                    x = restore1(w[u], m[u], v[u], Wd[u], lr, a.eps, a.rb);
                    m1 = Mfd[u] * m[u];
                    v1 = Vfd[u] * v[u];
                }
                u32 rm = 0, rv = 0;
                if (quant) {
                    // the row's part of the random stream is the same on every
                    // lane: compute it once, on the scalar unit
                    const u64 h = sm_at(sm_at(s_step, (u64)r), (u64)lane);
                    rm = (u32)(h & 0xffffull);
                    rv = (u32)((h >> 16) & 0xffffull);
                }
                const u64 ru = (u64)r;
                const bool clr = MODE == kAdam && !a.g_geo && base + u < nvis;
                if (FZ) {
                    mstore<GST>(at(rA[u], fzm), ms[u], m1, rm, false);
                    if (!sgd) mstore<GST>(at(rA[u], fzv), vs[u], v1, rv, true);
                }
                xs = x;
                if (isG) {
                    *reinterpret_cast<float *>(at(rG[u], off4)) = x;
                    if (!FZ) {
                        mstore<GST>(elem(a.gm.p, ru, sGM, offm), ms[u], m1, rm, false);
                        if (!sgd) mstore<GST>(elem(a.gv.p, ru, sGV, offm), vs[u], v1, rv, true);
                    }
                    if (clr) *reinterpret_cast<float *>(elem(a.gd_geo, ru, 40u, off4)) = 0.0f;
                    asm volatile("; G columns");
                } else {
                    *reinterpret_cast<float *>(at(rA[u], off4)) = x;
                    if (!FZ) {
                        mstore<AST>(elem(a.am.p, ru, sAM, offm), ms[u], m1, rm, false);
                        if (!sgd) mstore<AST>(elem(a.av.p, ru, sAV, offm), vs[u], v1, rv, true);
                    }
                    if (clr) *reinterpret_cast<float *>(elem(a.gd_app, ru, sAG, off4)) = 0.0f;
                    asm volatile("; A columns");
                }
            }
            if (a.cull_sum) {
                const float4 sv = cull_summary_store_wave(a.cull_sum, r, xs, t);
                if (a.cull_chunk) chunk_widen(a.cull_chunk, r, sv, crec[u]);
            }
            if (lane == 0) a.last[r] = t;
        }
        if (MODE == kAdamMax && lane == 0) {
            u32 nn = 0;
#pragma unroll
            for (int u = 0; u < kRU; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) nn += newt[u][k] != 0xffffffffu;
            if (nn) {
                u32 at = atomicAdd(a.fp8count, nn);
#pragma unroll
                for (int u = 0; u < kRU; ++u)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (newt[u][k] != 0xffffffffu) {
                            if ((int64_t)at < 4 * a.nb) a.fp8list[at] = newt[u][k];
                            ++at;
                        }
            }
        }
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            d[u] = gap(lastn[u], okn[u]);
            id[u] = idn[u];
            ok[u] = okn[u];
        }
        decode(base + 2 * stride, ridnn, idn, okn);
    }
}

// The step, the rows, then the tables' advance to the next step: its stores
// follow every load of the rows, so the rows' uniform loads stay scalar.
template <int MODE, int GST, int AST, int OPT, bool FZ>
__global__ __launch_bounds__(256) void k_rows(RowArgs a)
{
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, MODE == kFlush ? 1 : 0, &Wrow, &dmax, &step_err);
    // the tables do not hold this step: nothing is stored (the gather still
    // writes its outputs; the header's error word says they are not valid)
    if (step_err && MODE != kGather) {
        step_flag(a.step, step_err);
        return;
    }
    rows_work<MODE, GST, AST, OPT, FZ>(a, t, Wrow, dmax);
    if (MODE == kAdam && a.adv.on)
        lut_advance_slice(a.adv, a.step, t, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
    step_flag(a.step, step_err);
}

// ---------------------------------------------------------------------------
// Row kernels of the common configuration: Adam, one moment storage type
// (FP32 or BF16) for both groups, the fused layout with the moments of the
// two groups contiguous (A w | G m, A m | G v, A v), compact gradients and
// deferred geometry.  Same arithmetic and lane mapping as k_rows (lane c < 10
// is G column c, lane 10 + c is A column c), with far fewer instructions a
// row:
//  - each lane's weight, gradient and output element is one per-lane 64-bit
//    address, a 32 x 32 + 64-bit multiply-add of the wave-uniform row index
//    with the lane's stride and base (G lanes: the [n][10] array; A lanes: the
//    fused row), so G and A lanes load and store together, with no exec-mask
//    halves and no per-row scalar bases of either group;
//  - the moments of all lanes are one run each in the fused row: the row's
//    scalar base plus the lane's 32-bit offset.
// ---------------------------------------------------------------------------
struct FastArgs {
    const float *gw;                 // [n][10] G weights
    char *fz;                        // fused rows (A w at offset 0)
    int32_t *last;
    const u32 *ids, *count;
    const u32 *sat_ids, *sat_count;  // saturated rows (max_defer > 0)
    const float *g_geo, *g_app;      // compact gradients (update)
    float *out_geo, *out_app;        // compact outputs (gather)
    const float *Mf, *Vf, *SS, *BC;
    StepK step;
    float lr[64];                    // lane-indexed: 0..9 G, 10.. A
    float eps, omb1, omb2, rb;
    u64 sr_seed;
    u32 n, cap, adim, fz_s;          // rows, id capacity, A columns, fused row bytes
    u32 om, ov, pad0, pad1;          // byte offsets of the G m and G v runs in the fused row
    LutAdv adv;                      // kAdam: the tables' advance to the next step
    float4 *cull_sum;                // [n] cull summaries kept current (or null)
    float *cull_chunk;               // their chunk records, widened (or null)
};

// Pointers into the global and the constant address space: global loads and
// stores need no flat-address checks, and uniform loads of read-only tables
// through a constant-space pointer become scalar loads.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) u32 gu32;
typedef __attribute__((address_space(4))) const float cfloat;
__device__ __forceinline__ gfloat *gptr(u64 a) { return (gfloat *)a; }
__device__ __forceinline__ const cfloat *cptr(const float *p) { return (const cfloat *)(uintptr_t)p; }

template <int MODE, int ST, int RU>
__device__ __forceinline__ void rows_fz_work(const FastArgs &a, const int t, const float *const Wrow, const int dmax)
{
    static_assert(MODE == kGather || MODE == kAdam, "gather and update only");
    static_assert(ST == GS_F32 || ST == GS_BF16, "FP32 or BF16 moments");
    static_assert(RU >= 1 && RU <= 8 && (RU & (RU - 1)) == 0, "rows per iteration: a power of two up to 8");
    constexpr u32 MS = (u32)msize<ST>();
    const int lane = threadIdx.x & 63;
    const u32 wid = blockIdx.x * 4u + (u32)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const u32 nw = gridDim.x * 4u;
    const u32 adim = a.adim;
    const bool isG = lane < 10;
    const bool act = (u32)lane < 10u + adim;
    // lanes past the last column load (never store) the last column
    const u32 col = isG ? (u32)lane : min((u32)lane - 10u, adim - 1u);
    const u32 mcol = isG ? (u32)lane : 10u + col;
    const u32 mo = a.om + mcol * MS, vo = a.ov + mcol * MS;
    const u64 wb = isG ? (u64)(a.gw + lane) : (u64)(a.fz + 4u * col);
    const u32 wst = isG ? 40u : a.fz_s;
    const u64 cb = MODE == kAdam ? (isG ? (u64)(a.g_geo + lane) : (u64)(a.g_app + col))
                                 : (isG ? (u64)(a.out_geo + lane) : (u64)(a.out_app + col));
    const u32 cst = isG ? 40u : 4u * adim;
    const float lr = a.lr[lane];
    const cfloat *W4 = cptr(Wrow), *Mf4 = cptr(a.Mf), *Vf4 = cptr(a.Vf);
    if (a.n == 0) return;
    const u32 n = a.n;
    u32 nvis, total;
    {
        const u32 c = *a.count;
        nvis = c < a.cap ? c : a.cap;
        total = nvis + ((MODE == kAdam && a.sat_count) ? *a.sat_count : 0u);
    }
    float ss = 0.0f, bc = 1.0f;
    if (MODE == kAdam) {
        ss = cptr(a.SS)[t];
        bc = cptr(a.BC)[t];
    }
    const float step = lr * ss;
    const u64 s_step = ST == GS_BF16 ? sm_at(a.sr_seed, (u64)t) : 0ull;

    // Row bookkeeping in vector registers, lane u (mod RU) holding row u of an
    // iteration: the iteration's ids and last steps are one load each, read
    // into scalar registers lane by lane.  Software pipeline: the ids two
    // iterations ahead and the last steps one iteration ahead are in flight
    // while an iteration's rows load; positions past the end read the last
    // position and give row 0, which is loaded but never stored.
    const u32 stride = nw * RU;
    const u32 lu = (u32)lane & (RU - 1u);
    auto fetch_id = [&](u32 b) -> u32 {
        const u32 i = min(b + lu, total - 1u);
        const u32 *p = i < nvis ? a.ids + i : a.sat_ids + (i - nvis);
        return *(const gu32 *)p;
    };
    auto valid_id = [&](u32 b, u32 raw) -> u32 { return (b + lu < total && raw < n) ? raw : 0xffffffffu; };
    auto fetch_last = [&](u32 idv) -> int { return a.last[idv < n ? idv : 0u]; };
    u32 base = wid * RU;
    if (base >= total) return;
    u32 idc = valid_id(base, fetch_id(base));
    int lastc = fetch_last(idc);
    u32 idn = fetch_id(base + stride);
    for (; base < total; base += stride) {
        // rows of this iteration (scalar)
        u32 id[RU];
        bool ok[RU];
        int d[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const u32 r = (u32)__builtin_amdgcn_readlane((int)idc, u);
            ok[u] = r != 0xffffffffu;
            id[u] = ok[u] ? r : 0u;
            int dd = t - 1 - __builtin_amdgcn_readlane(lastc, u);
            dd = dd < 0 ? 0 : (dd > dmax ? dmax : dd);
            d[u] = ok[u] ? dd : 0;
        }
        // next iteration's last steps and the ids after it
        const u32 idnv = valid_id(base + stride, idn);
        const int lastn = fetch_last(idnv);
        const u32 idnn = fetch_id(base + 2 * stride);
        u32 wr[RU], gr[RU];
        typename RawT<ST>::T mr[RU], vr[RU];
        gfloat *wa[RU];
        gchar *fb[RU];
        float crec[RU];                  // chunk record elements (the update)
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            crec[u] = 0.0f;
            if (MODE == kAdam && a.cull_chunk) crec[u] = chunk_rec_lane(a.cull_chunk, id[u]);
            wa[u] = gptr(wb + (u64)id[u] * (u64)wst);
            fb[u] = srow(a.fz, id[u], a.fz_s);
            wr[u] = __float_as_uint(*wa[u]);
            mr[u] = mraw<ST>((const char *)(fb[u] + lane_off(mo)));
            vr[u] = mraw<ST>((const char *)(fb[u] + lane_off(vo)));
            gr[u] = 0u;
            if (MODE == kAdam && base + u < nvis) gr[u] = *(const gu32 *)(cb + (u64)(base + u) * (u64)cst);
        }
        float Wd[RU], Mfd[RU], Vfd[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            Wd[u] = W4[d[u]];
            if (MODE == kAdam) {
                Mfd[u] = Mf4[d[u]];
                Vfd[u] = Vf4[d[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const float w = __uint_as_float(wr[u]);
            const float m = mdec<ST>((u32)mr[u], 0.0f, false);
            const float v = mdec<ST>((u32)vr[u], 0.0f, true);
            if (MODE == kGather) {
                float x = w;
                if (d[u] > 0) x = restore1(x, m, v, Wd[u], lr, a.eps, a.rb);
                if (ok[u] && act) *gptr(cb + (u64)(base + u) * (u64)cst) = x;
                continue;
            }
            const float g = __uint_as_float(gr[u]);
            float x = w;
            if (d[u] > 0) x = restore1(x, m, v, Wd[u], lr, a.eps, a.rb);
            const float m1 = Mfd[u] * m + a.omb1 * g;
            const float v1 = Vfd[u] * v + (a.omb2 * g) * g;
            x = x - adam_step(m1, v1, step, bc, a.eps, a.rb);
            u32 rm = 0, rv = 0;
            if (ST == GS_BF16) {
                const u64 h = sm_at(sm_at(s_step, (u64)id[u]), (u64)lane);
                rm = (u32)(h & 0xffffull);
                rv = (u32)((h >> 16) & 0xffffull);
            }
            if (ok[u]) {
                if (act) {
                    *wa[u] = x;
                    mstore<ST>((char *)(fb[u] + lane_off(mo)), 0.0f, m1, rm, false);
                    mstore<ST>((char *)(fb[u] + lane_off(vo)), 0.0f, v1, rv, true);
                }
                if (a.cull_sum) {
                    const float4 sv = cull_summary_store_wave(a.cull_sum, id[u], x, t);
                    if (a.cull_chunk) chunk_widen(a.cull_chunk, id[u], sv, crec[u]);
                }
                if (lane == 0) a.last[id[u]] = t;
            }
        }
        idc = idnv;
        lastc = lastn;
        idn = idnn;
    }
}

// The step, the rows, then the tables' advance (after every load of the rows).
template <int MODE, int ST, int RU>
__global__ __launch_bounds__(256) void k_rows_fz(FastArgs a)
{
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    if (step_err && MODE == kAdam) {
        step_flag(a.step, step_err);
        return;
    }
    rows_fz_work<MODE, ST, RU>(a, t, Wrow, dmax);
    if (MODE == kAdam && a.adv.on)
        lut_advance_slice(a.adv, a.step, t, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
    step_flag(a.step, step_err);
}

// FP8 scale growth between the two Adam passes: every 128-row block whose
// recorded max outgrew its scale gets the smallest power-of-two scale that
// fits, and all its rows are re-encoded (random column = column + 64); the
// recorded max is cleared.  One wavefront per block and moment.
struct RescaleArgs {
    uint8_t *q[4];                   // G m, G v, A m, A v codes
    float *s[4];                     // their block scales
    int64_t ld[4];
    int32_t dim[4], col0[4];
    u32 *maxb[4];
    int32_t fp8[4];                  // which of the four are FP8
    int64_t n, nb;
    u64 sr_seed;
    StepK step;
    const u32 *list, *count;         // tasks that outgrew their scale this step
};

// One workgroup per listed task (moment, 128-row block): grow the scale to the
// smallest power of two that fits the recorded max and re-encode the block.
__global__ __launch_bounds__(256) void k_fp8_rescale(RescaleArgs a)
{
    constexpr int kIlp = 8;          // codes per thread in flight (a 49-column block: 3 rounds)
    __shared__ float sOld;
    const int tid = threadIdx.x;
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    if (step_err) {
        step_flag(a.step, step_err);
        return;
    }
    const u64 s_step = sm_at(a.sr_seed, (u64)t);
    const u32 ntask = (u32)min((int64_t)*a.count, 4 * a.nb);
    for (u32 i = blockIdx.x; i < ntask; i += gridDim.x) {
        const u32 task = a.list[i];
        const int wq = (int)(task / (u32)a.nb);
        const int64_t bq = (int64_t)(task - (u32)wq * (u32)a.nb);
        const float amax = __uint_as_float(a.maxb[wq][bq]);
        if (tid == 0) sOld = a.s[wq][bq];
        __syncthreads();
        const float sold = sOld;
        const float snew = fp8_scale_for(amax);
        // A block still at scale 0 holds only 0x00 codes (stores under scale 0
        // write 0x00 and scales only grow), which re-encode to 0x00: its rows
        // are not touched, only its scale is set.
        if (snew > sold && sold > 0.0f) {
            const int dim = a.dim[wq];
            const int64_t r0 = bq * kFp8Block;
            const int64_t nrow = min((int64_t)kFp8Block, a.n - r0);
            const int64_t nel = nrow * dim;
            const bool is_v = wq & 1;
            uint8_t *q = a.q[wq];
            const int64_t ld = a.ld[wq];
            // scales are powers of two: a normal code that stays normal only loses
            // kshift from its exponent field (the stochastic rounding of an exactly
            // representable value returns it); the rest take the full rounding
            int eo = 0, en = 0;
            frexpf(sold, &eo);
            frexpf(snew, &en);
            const int kshift = en - eo;
            for (int64_t e0 = 0; e0 < nel; e0 += 256 * kIlp) {
                uint8_t code[kIlp];
                int64_t off[kIlp], row[kIlp];
                int col[kIlp];
#pragma unroll
                for (int k = 0; k < kIlp; ++k) {
                    const int64_t e = e0 + k * 256 + tid;
                    const u32 rr = (u32)e / (u32)dim;     // e < 128 * 54: 32-bit division
                    row[k] = r0 + rr;
                    col[k] = (int)((u32)e - rr * (u32)dim);
                    off[k] = e < nel ? row[k] * ld + col[k] : -1;
                    code[k] = off[k] >= 0 ? q[off[k]] : (uint8_t)0;
                }
#pragma unroll
                for (int k = 0; k < kIlp; ++k) {
                    if (off[k] < 0) continue;
                    const int ef = (code[k] >> 3) & 15, mf = code[k] & 7;
                    if (ef >= 1 && !(ef == 15 && mf == 7) && ef - kshift >= 1) {
                        q[off[k]] = (uint8_t)((code[k] & 0x80) | ((ef - kshift) << 3) | mf);
                        continue;
                    }
                    const float x = e4m3_dec(code[k]) * sold;
                    const u64 h = sm_at(sm_at(s_step, (u64)row[k]), (u64)(a.col0[wq] + col[k] + 64));
                    const u32 rr = (u32)((is_v ? h >> 16 : h) & 0xffffull);
                    q[off[k]] = (uint8_t)e4m3_sr(x / snew, rr);
                }
            }
        }
        __syncthreads();              // every thread has read sold and the codes
        if (tid == 0) {
            if (snew > sold) a.s[wq][bq] = snew;
            a.maxb[wq][bq] = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// dense geometric Adam (geo_mode = 1): every row's 10 G columns, every step
// ---------------------------------------------------------------------------
struct DenseArgs {
    float *w;
    MomRef m, v;
    int64_t n;
    StepK step;
    float lr[10];
    float eps, omb1, omb2, b1f, b2f, rb;
    const float *SS, *BC;
    u64 sr_seed;
    const float *g_geo;              // compact gradients of the cull's visible rows, or NULL
    const u64 *keep_bits;            // the cull's keep ballots
    const u64 *tile_off;             // the cull's tile prefixes (visible << 32 | saturated)
    int64_t tiles;
    u32 cap, pad2;
    float *gd_geo;                   // dense [n][10] gradients (read and cleared) when g_geo is NULL
};

// One block per cull tile (512 rows x 10 columns, element-parallel and
// coalesced).  The compact index of a visible row is the tile's exclusive
// prefix (from the cull's tile scan) + the keep bits before it.
template <int GST>
__global__ __launch_bounds__(256) void k_dense_geo(DenseArgs a)
{
    __shared__ u64 sBits[gsdp::kWordsPerTile];
    __shared__ u32 sOff[gsdp::kWordsPerTile];
    __shared__ u32 sExcl;
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t row0 = tile * kCullTile;
    const int rows = (int)min((int64_t)kCullTile, a.n - row0);
    if (a.g_geo) {
        if (tid < gsdp::kWordsPerTile) sBits[tid] = a.keep_bits[tile * gsdp::kWordsPerTile + tid];
        if (tid == 0) sExcl = (u32)(a.tile_off[tile] >> 32);
        __syncthreads();
        if (tid == 0) {
            u32 o = 0;
            for (int j = 0; j < gsdp::kWordsPerTile; ++j) {
                sOff[j] = o;
                o += (u32)__popcll(sBits[j]);
            }
        }
        __syncthreads();
    }
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    if (step_err) {
        step_flag(a.step, step_err);
        return;
    }
    const float ss = a.SS[t], bc = a.BC[t];
    const u64 s_step = GST != GS_F32 ? sm_at(a.sr_seed, (u64)t) : 0ull;
    for (int e = tid; e < rows * 10; e += 256) {
        const int r = e / 10, c = e - r * 10;
        const int64_t row = row0 + r;
        float g = 0.0f;
        if (a.g_geo) {
            const int word = (r >> 8) * 4 + ((r & 255) >> 6), bit = r & 63;
            const u64 bw = sBits[word];
            if ((bw >> bit) & 1ull) {
                const u32 rank = sExcl + sOff[word] + (u32)__popcll(bw & ((1ull << bit) - 1ull));
                if (rank < a.cap) g = a.g_geo[(int64_t)rank * 10 + c];
            }
        } else {
            g = a.gd_geo[row * 10 + c];
            a.gd_geo[row * 10 + c] = 0.0f;
        }
        const float mm = mom_load<GST>(a.m, row, c, false), vv = mom_load<GST>(a.v, row, c, true);
        const float m1 = a.b1f * mm + a.omb1 * g;
        const float v1 = a.b2f * vv + (a.omb2 * g) * g;
        const float lr = a.lr[c];
        a.w[row * 10 + c] = a.w[row * 10 + c] - adam_step(m1, v1, lr * ss, bc, a.eps, a.rb);
        u32 rm = 0, rv = 0;
        if (GST != GS_F32) {
            const u64 h = sm_at(sm_at(s_step, (u64)row), (u64)c);
            rm = (u32)(h & 0xffffull);
            rv = (u32)((h >> 16) & 0xffffull);
        }
        mom_store<GST>(a.m, row, c, m1, rm, false);
        mom_store<GST>(a.v, row, c, v1, rv, true);
    }
}

// ---------------------------------------------------------------------------
// scatter and synthetic gradients
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(const u32 *ids, const u32 *count, u32 cap, int dim,
                                                 const float *gc, float *gd, int acc)
{
    const u32 c = *count;
    const int64_t total = (int64_t)(c < cap ? c : cap) * dim;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / dim;
        const int col = (int)(e - i * dim);
        float *dst = gd + (int64_t)ids[i] * dim + col;
        const float val = gc[e];
        *dst = acc ? *dst + val : val;
    }
}

__global__ __launch_bounds__(256) void k_synth(u64 seed, u64 step, const u32 *ids, const u32 *count, u32 cap,
                                               int dim, int col0, double scale, float *out)
{
    const u32 c = *count;
    const int64_t total = (int64_t)(c < cap ? c : cap) * dim;
    const u64 s1 = sm_at(seed, step);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / dim;
        const int col = (int)(e - i * dim);
        const u64 key = ids ? (u64)ids[i] : (u64)i;
        const u64 h = sm_at(sm_at(s1, key), (u64)(col0 + col));
        const long long s = (long long)((h & 0xffffull) + ((h >> 16) & 0xffffull) + ((h >> 32) & 0xffffull) + (h >> 48));
        out[e] = (float)((double)(2 * s - 4 * 65535) * scale);
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
thread_local char g_err[512] = "";

int hip_fail(hipError_t e, const char *what)
{
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
    return GS_EHIP;
}

int launched(const char *what)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : hip_fail(e, what);
}

std::atomic<int> g_cu[64];

int cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int v = g_cu[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        g_cu[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Clamp of the restore factor: 1.03 x (1-b1)/sqrt((1-b2)(1-b1^2/b2)) in FP32
// (+inf when b1^2 >= b2, where Adam moments have no such bound).
float restore_bound(double b1, double b2)
{
    if (!(b1 * b1 < b2)) return INFINITY;
    return (float)((1.0 - b1) / std::sqrt((1.0 - b2) * (1.0 - b1 * b1 / b2)) * 1.03);
}

size_t mom_bytes(int state) { return state == GS_F32 ? 4 : (state == GS_BF16 ? 2 : 1); }

bool has_fp8(const gs_model *m) { return m->geo.state == GS_FP8E4M3 || m->app.state == GS_FP8E4M3; }

int check_group(const gs_group &g, int64_t n, bool geo)
{
    if (geo && g.dim != 10) return GS_EINVAL;
    if (!geo && (g.dim < 1 || g.dim > 54)) return GS_EINVAL;
    if (g.w_ld < g.dim || g.m_ld < g.dim || g.v_ld < g.dim) return GS_EINVAL;
    if (g.state != GS_F32 && g.state != GS_BF16 && g.state != GS_FP8E4M3) return GS_EUNSUPPORTED;
    if (n > 0 && (!g.w || !g.m || !g.v)) return GS_EINVAL;
    if (n > 0 && g.state == GS_FP8E4M3 && (!g.m_scale || !g.v_scale)) return GS_EINVAL;
    if (!aligned(g.w, 4) || !aligned(g.m, mom_bytes(g.state)) || !aligned(g.v, mom_bytes(g.state)))
        return GS_EINVAL;
    return GS_OK;
}

int decay_classes(const gs_model *m, float *rates, uint8_t *cls);

int check_model(const gs_model *m)
{
    if (!m) return GS_EINVAL;
    if (m->n < 0 || m->n > 0x7fffffffLL) return GS_EINVAL;
    int rc = check_group(m->geo, m->n, true);
    if (rc) return rc;
    rc = check_group(m->app, m->n, false);
    if (rc) return rc;
    if (m->geo.w_ld != 10 || !aligned(m->geo.w, 16)) return GS_EINVAL;
    if (m->n > 0 && !m->last_step) return GS_EINVAL;
    if (!m->lut || m->lut_max_steps < 1 || m->max_defer < 0) return GS_EINVAL;
    if (!(m->beta1 > 0.0 && m->beta1 < 1.0 && m->beta2 > 0.0 && m->beta2 < 1.0 && m->eps >= 0.0)) return GS_EINVAL;
    if (m->cull_mode != 0 && m->cull_mode != 1) return GS_EINVAL;
    if (m->geo_mode != 0 && m->geo_mode != 1) return GS_EINVAL;
    if (m->geo_mode == 1 && m->geo.state == GS_FP8E4M3) return GS_EUNSUPPORTED;
    if (m->optimizer != GS_OPT_ADAM && m->optimizer != GS_OPT_SGD_MOMENTUM && m->optimizer != GS_OPT_ADAMW)
        return GS_EINVAL;
    if (m->optimizer != GS_OPT_ADAM &&
        (m->geo_mode != 0 || m->geo.state == GS_FP8E4M3 || m->app.state == GS_FP8E4M3))
        return GS_EUNSUPPORTED;
    if (m->optimizer == GS_OPT_ADAMW) {
        float rates[gsdp::kMaxDecayClasses];
        if (decay_classes(m, rates, nullptr) < 0) return GS_EUNSUPPORTED;
    }
    // summaries stay current only where the row kernels store the geometry
    if (m->cull_sum && !aligned(m->cull_sum, 16)) return GS_EINVAL;
    if (m->cull_sum && m->geo_mode != 0) return GS_EUNSUPPORTED;
    if (m->cull_chunk && (!m->cull_sum || !aligned(m->cull_chunk, 32))) return GS_EINVAL;
    return GS_OK;
}

// The tables that do not move with the step: b^(d+1), step sizes and bias terms.
struct LutPtrs {
    const float *Mf, *Vf, *SS, *BC;
};

LutPtrs lut_ptrs(const gs_model *m)
{
    const gsdp::LutLayout L = gsdp::lut_layout(m->lut_max_steps, m->max_defer);
    const char *base = static_cast<const char *>(m->lut);
    auto f = [&](int64_t o) { return reinterpret_cast<const float *>(base + o); };
    return {f(L.oMf), f(L.oVf), f(L.oSS), f(L.oBC)};
}

// AdamW class tables in the kernels' float units: the first class's restore
// rows, floats per class block, and the distance from the restore rows to
// the decay-product rows (the step decays follow at twice that).
// The tables' advance of `m` (on = 1).
LutAdv lut_adv(const gs_model *m)
{
    const gsdp::LutLayout L = gsdp::lut_layout(m->lut_max_steps, m->max_defer);
    char *base = static_cast<char *>(m->lut);
    LutAdv a;
    memset(&a, 0, sizeof a);
    a.Wd = reinterpret_cast<double *>(base + L.oWd);
    a.Wf = reinterpret_cast<float *>(base + L.oWf);
    a.R = reinterpret_cast<const double *>(base + L.oR);
    a.Cn = reinterpret_cast<const double *>(base + L.oC);
    a.cls = base + L.oCls;
    a.cls_bytes = L.cls_bytes;
    a.cWlf = L.cWlf;
    a.cPf = L.cPf;
    a.cWld = L.cWld;
    a.cPd = L.cPd;
    a.cqd = L.cqd;
    if (m->optimizer == GS_OPT_ADAMW) {
        float rates[gsdp::kMaxDecayClasses];
        a.nclass = decay_classes(m, rates, nullptr);
    }
    a.on = 1;
    return a;
}

void adamw_ptrs(const gs_model *m, const float **base, int64_t *per, int64_t *nW)
{
    const gsdp::LutLayout L = gsdp::lut_layout(m->lut_max_steps, m->max_defer);
    *base = reinterpret_cast<const float *>(static_cast<const char *>(m->lut) + L.oCls + L.cWlf);
    *per = L.cls_bytes / 4;
    *nW = 2 * L.nrow;
}

// step >= 1: that step; step == 0: the step is read from *step_dev when the
// kernels run (graph replay), clamped to [1, lut_max_steps]
bool step_ok(const gs_model *m, int64_t step)
{
    if (step == 0) return m->step_dev != nullptr;
    return step >= 1 && step <= m->lut_max_steps;
}

StepK step_k(const gs_model *m, int64_t step)
{
    StepK k;
    memset(&k, 0, sizeof k);
    const gsdp::LutLayout L = gsdp::lut_layout(m->lut_max_steps, m->max_defer);
    k.t = (int32_t)step;
    k.T = m->lut_max_steps;
    k.K = m->max_defer;
    k.nrow = (int32_t)L.nrow;
    k.t_dev = step == 0 ? m->step_dev : nullptr;
    k.hdr = static_cast<gsdp::LutHeader *>(m->lut);
    k.lut = reinterpret_cast<const float *>(static_cast<const char *>(m->lut) + L.oWf);
    return k;
}

// AdamW decay classes: the distinct column rates in order of first
// appearance (G columns 0..9, then A columns); cls[lane] is the class of the
// column lane (0..9 G, 10.. A).  Returns the number of classes, -1 if > 8.
int decay_classes(const gs_model *m, float *rates, uint8_t *cls)
{
    int nc = 0;
    for (int lane = 0; lane < 64; ++lane) {
        if (cls) cls[lane] = 0;
        float r;
        if (lane < 10) r = m->geo.lr[lane];
        else if (lane - 10 < m->app.dim) r = m->app.lr[lane - 10];
        else continue;
        int c = 0;
        while (c < nc && memcmp(&rates[c], &r, sizeof r) != 0) ++c;
        if (c == nc) {
            if (nc == gsdp::kMaxDecayClasses) return -1;
            rates[nc++] = r;
        }
        if (cls) cls[lane] = (uint8_t)c;
    }
    return nc;
}

// Byte offset of p inside the row of the fused block at base, or -1.
int64_t fused_off(const void *base, const void *p, int64_t row_bytes)
{
    const int64_t o = static_cast<const char *>(p) - static_cast<const char *>(base);
    return (o >= 0 && o < row_bytes) ? o : -1;
}

// The fused layout: every state array of a row but G w in one byte row.
bool fused_layout(const gs_model *m, u32 *S, u32 *ogm, u32 *ogv, u32 *oam, u32 *oav)
{
    const int64_t gs = (int64_t)mom_bytes(m->geo.state), as = (int64_t)mom_bytes(m->app.state);
    const int64_t row = (int64_t)m->app.w_ld * 4;
    if (row <= 0 || row > 0xffff) return false;
    if ((int64_t)m->app.m_ld * as != row || (int64_t)m->app.v_ld * as != row || (int64_t)m->geo.m_ld * gs != row ||
        (int64_t)m->geo.v_ld * gs != row)
        return false;
    const int64_t o[4] = {fused_off(m->app.w, m->geo.m, row), fused_off(m->app.w, m->geo.v, row),
                          fused_off(m->app.w, m->app.m, row), fused_off(m->app.w, m->app.v, row)};
    for (int k = 0; k < 4; ++k)
        if (o[k] < 0) return false;
    *S = (u32)row;
    *ogm = (u32)o[0];
    *ogv = (u32)o[1];
    *oam = (u32)o[2];
    *oav = (u32)o[3];
    return true;
}

void fill_rows(RowArgs &a, const gs_model *m)
{
    memset(&a, 0, sizeof a);
    if (!fused_layout(m, &a.fz_s, &a.fz_ogm, &a.fz_ogv, &a.fz_oam, &a.fz_oav)) a.fz_s = 0;
    a.gw = m->geo.w;
    a.gw_ld = m->geo.w_ld;
    a.gm = {m->geo.m, m->geo.m_scale, m->geo.m_ld};
    a.gv = {m->geo.v, m->geo.v_scale, m->geo.v_ld};
    a.aw = m->app.w;
    a.aw_ld = m->app.w_ld;
    a.am = {m->app.m, m->app.m_scale, m->app.m_ld};
    a.av = {m->app.v, m->app.v_scale, m->app.v_ld};
    a.adim = m->app.dim;
    for (int c = 0; c < 10; ++c) a.lr[c] = m->geo.lr[c];
    for (int c = 0; c < m->app.dim; ++c) a.lr[10 + c] = m->app.lr[c];
    a.eps = (float)m->eps;
    a.omb1 = (float)(1.0 - m->beta1);
    a.omb2 = (float)(1.0 - m->beta2);
    a.rb = restore_bound(m->beta1, m->beta2);
    a.sr_seed = m->sr_seed;
    a.geo_dense = m->geo_mode == 1;
    if (m->optimizer == GS_OPT_ADAMW) {
        float rates[gsdp::kMaxDecayClasses];
        decay_classes(m, rates, a.cls);
        adamw_ptrs(m, &a.aw_base, &a.aw_per, &a.aw_nW);
    }
    a.last = m->last_step;
    a.n = m->n;
    a.cull_sum = reinterpret_cast<float4 *>(m->cull_sum);
    a.cull_chunk = m->cull_sum ? m->cull_chunk : nullptr;
}

// The configuration of k_rows_fz: Adam, both groups' moments in FP32 or both
// in BF16, deferred geometry, G w dense, and the fused layout with the G and
// A moment runs adjacent (A m right after G m, A v right after G v).  Fills
// everything but the per-call pointers; false when the model does not qualify.
bool fill_fast(FastArgs &f, const gs_model *m)
{
    memset(&f, 0, sizeof f);
    if (m->optimizer != GS_OPT_ADAM || m->geo_mode != 0) return false;
    const int st = m->geo.state;
    if (st != m->app.state || (st != GS_F32 && st != GS_BF16)) return false;
    if (m->geo.w_ld != 10 || m->n <= 0 || m->n > 0x7fffffff) return false;
    u32 S, ogm, ogv, oam, oav;
    if (!fused_layout(m, &S, &ogm, &ogv, &oam, &oav)) return false;
    const u32 ms = (u32)mom_bytes(st);
    if (oam != ogm + 10u * ms || oav != ogv + 10u * ms) return false;
    f.gw = m->geo.w;
    f.fz = reinterpret_cast<char *>(m->app.w);
    f.last = m->last_step;
    for (int c = 0; c < 10; ++c) f.lr[c] = m->geo.lr[c];
    for (int c = 0; c < m->app.dim; ++c) f.lr[10 + c] = m->app.lr[c];
    f.eps = (float)m->eps;
    f.omb1 = (float)(1.0 - m->beta1);
    f.omb2 = (float)(1.0 - m->beta2);
    f.rb = restore_bound(m->beta1, m->beta2);
    f.sr_seed = m->sr_seed;
    f.n = (u32)m->n;
    f.adim = (u32)m->app.dim;
    f.fz_s = S;
    f.om = ogm;
    f.ov = ogv;
    f.cull_sum = reinterpret_cast<float4 *>(m->cull_sum);
    f.cull_chunk = m->cull_sum ? m->cull_chunk : nullptr;
    return true;
}

template <int MODE, int RU>
void launch_fast(int st, int grid, hipStream_t s, const FastArgs &f)
{
    if (st == GS_F32) hipLaunchKernelGGL((k_rows_fz<MODE, GS_F32, RU>), dim3(grid), dim3(256), 0, s, f);
    else hipLaunchKernelGGL((k_rows_fz<MODE, GS_BF16, RU>), dim3(grid), dim3(256), 0, s, f);
}

// Camera constants of cull_v1 and of the band classifier (bounds rounded up).
void pack_camera(const gs_model *model, const gs_camera *cam, CamK &k, BandK &b)
{
    for (int i = 0; i < 9; ++i) k.R[i] = cam->R[i];
    for (int i = 0; i < 3; ++i) k.T[i] = cam->t[i];
    k.fx = cam->fx;
    k.fy = cam->fy;
    k.cx = cam->cx;
    k.cy = cam->cy;
    k.W = (float)cam->width;
    k.H = (float)cam->height;
    k.zn = cam->near_plane;
    k.zf = cam->far_plane;
    const double B = (double)restore_bound(model->beta1, model->beta2) * 1.001;
    auto mx = [&](int lo, int hi) {
        double v = 0.0;
        for (int c = lo; c < hi; ++c) v = std::max(v, (double)std::fabs(model->geo.lr[c]));
        return (float)(B * v * (1.0 + 1e-6));
    };
    b.kpos = mx(0, 3);
    b.kscl = mx(3, 6);
    b.kq = mx(6, 10);
    auto rs = [&](int r) {
        return (float)((std::fabs((double)cam->R[3 * r]) + std::fabs((double)cam->R[3 * r + 1]) +
                        std::fabs((double)cam->R[3 * r + 2])) * (1 + 1e-6));
    };
    b.rs0 = rs(0);
    b.rs1 = rs(1);
    b.rs2 = rs(2);
    const float limx = 1.3f * ((0.5f * (float)cam->width) / cam->fx);
    const float limy = 1.3f * ((0.5f * (float)cam->height) / cam->fy);
    const double fx = cam->fx, fy = cam->fy;
    b.jf2 = (float)((fx * fx * (1.0 + (double)limx * limx) + fy * fy * (1.0 + (double)limy * limy)) * (1.0 + 1e-4));
}

// Constants of side_out (a larger margin only keeps more rows).
void pack_side(const gs_camera *cam, const BandK &b, SideK &k)
{
    const double up = 1.0 + 1e-6;
    k.ksig = (float)(3.003 * std::sqrt(1.001 * (double)b.jf2) * up);
    const double fx = cam->fx, fy = cam->fy;
    const double cx = cam->cx, cy = cam->cy, W = cam->width, H = cam->height;
    const double c4[4] = {cx + 3.93, W - cx + 3.93, cy + 3.93, H - cy + 3.93};
    const double f4[4] = {fx, -fx, fy, -fy};
    const int row[4] = {0, 0, 1, 1};
    double R[9], T[3];
    for (int i = 0; i < 9; ++i) R[i] = cam->R[i];
    for (int i = 0; i < 3; ++i) T[i] = cam->t[i];
    auto r1 = [&](int r) { return std::fabs(R[3 * r]) + std::fabs(R[3 * r + 1]) + std::fabs(R[3 * r + 2]); };
    double sa = 0.0, sb = 0.0;
    for (int s = 0; s < 4; ++s) {
        const int r = row[s];
        double n1 = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double nj = f4[s] * R[3 * r + j] + c4[s] * R[6 + j];
            k.n[s][j] = (float)nj;
            n1 += std::fabs(nj);
        }
        const double kk = f4[s] * T[r] + c4[s] * T[2];
        k.k[s] = (float)kk;
        k.n1[s] = (float)(n1 * up + 1e-30);
        // rounding of the exact test's coordinates (2 |f| |R_r|_1 + (|c| + |c0|) |R_2|_1 per unit of
        // mu + dp, the same with |T|) and of this test (|n|_1 per unit of mu + dp, |k|)
        const double c0 = s < 2 ? std::fabs(cx) : std::fabs(cy);
        sa = std::max(sa, 2.0 * std::fabs(f4[s]) * r1(r) + (std::fabs(c4[s]) + c0) * r1(2) + n1);
        sb = std::max(sb, 2.0 * std::fabs(f4[s]) * std::fabs(T[r]) + (std::fabs(c4[s]) + c0) * std::fabs(T[2]) +
                              std::fabs(kk));
    }
    k.sa = (float)(sa * up);
    k.sb = (float)(sb * up + 1e-6);
}

// Launch k_rows<MODE> for the moment storage types and the optimizer of the
// model's groups.
template <int MODE, int G, int OPT>
void launch_rows_a(int ast, int grid, hipStream_t st, const RowArgs &a)
{
    // the fused single access when both groups share the storage type
    const bool fz = a.fz_s != 0 && ast == G;
    if (ast == GS_F32) {
        if (fz && G == GS_F32) hipLaunchKernelGGL((k_rows<MODE, G, GS_F32, OPT, G == GS_F32>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_rows<MODE, G, GS_F32, OPT, false>), dim3(grid), dim3(256), 0, st, a);
    } else if (ast == GS_BF16) {
        if (fz && G == GS_BF16) hipLaunchKernelGGL((k_rows<MODE, G, GS_BF16, OPT, G == GS_BF16>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_rows<MODE, G, GS_BF16, OPT, false>), dim3(grid), dim3(256), 0, st, a);
    } else if constexpr (OPT == GS_OPT_ADAM) {
        if (fz && G == GS_FP8E4M3)
            hipLaunchKernelGGL((k_rows<MODE, G, GS_FP8E4M3, OPT, G == GS_FP8E4M3>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_rows<MODE, G, GS_FP8E4M3, OPT, false>), dim3(grid), dim3(256), 0, st, a);
    }
}

// FP8 moments are Adam only (checked with the model)
template <int MODE, int OPT>
void launch_rows_o(const gs_model *m, int grid, hipStream_t st, const RowArgs &a)
{
    const int g = m->geo.state, p = m->app.state;
    if (g == GS_F32) launch_rows_a<MODE, GS_F32, OPT>(p, grid, st, a);
    else if (g == GS_BF16) launch_rows_a<MODE, GS_BF16, OPT>(p, grid, st, a);
    else if constexpr (OPT == GS_OPT_ADAM) launch_rows_a<MODE, GS_FP8E4M3, OPT>(p, grid, st, a);
}

template <int MODE>
void launch_rows(const gs_model *m, int grid, hipStream_t st, const RowArgs &a)
{
    if (m->optimizer == GS_OPT_SGD_MOMENTUM) launch_rows_o<MODE, GS_OPT_SGD_MOMENTUM>(m, grid, st, a);
    else if (m->optimizer == GS_OPT_ADAMW) launch_rows_o<MODE, GS_OPT_ADAMW>(m, grid, st, a);
    else launch_rows_o<MODE, GS_OPT_ADAM>(m, grid, st, a);
}

constexpr int kRowBlocksGather = 8, kRowBlocksUpdate = 16;
// rows per wavefront iteration of k_rows_fz
constexpr int kFastGatherRows = 2, kFastUpdateRows = 4;
// blocks of a row launch: one iteration's rows per wavefront at least, at most
// `per_cu` blocks per CU (the gather runs best at 8, the update passes at 16,
// where short and long wavefronts even out)
int row_grid(int64_t rows, int per_cu)
{
    const int cu = cu_count();
    int64_t want = (rows + 4 * row_unroll<kAdam>() - 1) / (4 * row_unroll<kAdam>());
    int64_t cap = (int64_t)(cu > 0 ? cu : 256) * per_cu;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)want;
}

// ---------------------------------------------------------------------------
// batched form: many scenes x many cameras in one pass
// ---------------------------------------------------------------------------
// The scenes are row ranges of one model (each starting at a multiple of
// kMultiAlign rows).  One tile of one scene is loaded once and culled against
// all C <= 32 cameras of that scene.  One global ordered compaction produces
//   union_ids : rows visible to at least one camera of their scene (ascending)
//   cam_pos[c]: for camera slot c, the union positions of the rows it sees
//               (ascending, all scenes back to back; scene_start gives each
//               scene's first entry in every list)
// from per-tile counts of 33 counters (union and 32 camera slots).
constexpr int kMaxCams = 32;
constexpr int kNCnt = kMaxCams + 1;
constexpr int kMultiMinTile = 64;


// union positions per chunk of the batched gradient sum
constexpr int kSumRows = 128;

struct MultiArgs {
    const float *gw;
    MomRef gm, gv;
    int32_t gst, mode;
    float rb, eps;
    const int32_t *last;
    int64_t n;
    StepK step;
    float lr[10];
    int32_t S, C, n_sets, pad0;
    const int64_t *scene_row0;       // [S+1]
    const CamPack *cams;             // [n_sets][S][C]
    u32 *union_ids, *union_count;
    u32 *cam_pos, *cam_count;
    u32 cap_union, cap_cam;
    u32 *scene_start;                // [S][1+C]
    u32 *chunk_start;                // [ceil(cap_union / kSumRows) + 1][C] or null
    u32 *cnt;                        // [kNCnt][stride] per-tile counts (union, camera slots)
    u32 *off;                        // [kNCnt][stride] exclusive prefixes over tiles
    u32 *grp;                        // [kNCnt][gstride] sums over groups of 64 tiles
    int64_t gstride;
    u32 *mask;                       // [n] camera bits of every row
    int64_t tiles;                   // tiles of this launch
    int64_t stride;                  // tiles of the smallest tile size
    int32_t tile_rows, pad5;         // rows per tile of this launch
};

// Batched cull in four launches (as the single-camera cull): k_cull_multi
// writes every row's camera bits and the tile's counts, k_multi_reduce and
// k_multi_offsets take the exclusive prefixes over tiles for every counter,
// k_multi_ids writes the union ids, the per-camera union positions and the
// chunk starts of the gradient sum.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_cull_multi(MultiArgs a)
{
    constexpr int NW = BLOCK / 64;
    constexpr int TR = BLOCK * IPT;
    constexpr int NSLAB = IPT * NW;
    __shared__ float4 sG4[TR * 10 / 4];
    __shared__ u32 sCnt[NSLAB][kNCnt];
    __shared__ u32 sScene;
    float *sG = reinterpret_cast<float *>(sG4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *Wrow;
    int dmax, step_err;
    const int t = resolve_step(a.step, 0, &Wrow, &dmax, &step_err);
    const int C = a.C;
    const int set = (t - 1) % a.n_sets;
    const int64_t tile = blockIdx.x;
    const int64_t row0 = tile * TR;
    const int rows = (int)min((int64_t)TR, a.n - row0);
    if (tid == 0) {
        int sc = 0;
        while (sc + 1 < a.S && a.scene_row0[sc + 1] <= row0) ++sc;
        sScene = (u32)sc;
    }
    const int nf = rows * 10, nf4 = nf >> 2;
    const float *src = a.gw + row0 * 10;
    const float4 *src4 = reinterpret_cast<const float4 *>(src);
    for (int j = tid; j < nf4; j += BLOCK) sG4[j] = src4[j];
    for (int j = nf4 * 4 + tid; j < nf; j += BLOCK) sG[j] = src[j];
    int lastv[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int r = k * BLOCK + tid;
        lastv[k] = r < rows ? a.last[row0 + r] : 0;
    }
    __syncthreads();
    const int scene = (int)sScene;
    const bool in_scene = row0 < a.scene_row0[scene + 1];
    const CamPack *cams = a.cams + ((int64_t)set * a.S + scene) * C;

#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int r = k * BLOCK + tid;
        const bool valid = r < rows && in_scene;
        u32 mk = 0;
        // every lane reads a row (past the tile's rows: stale LDS, never used)
        float g[10];
        const float2 *p2 = reinterpret_cast<const float2 *>(sG + r * 10);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const float2 q = p2[j];
            g[2 * j] = q.x;
            g[2 * j + 1] = q.y;
        }
        int d = t - 1 - lastv[k];
        d = d < 0 ? 0 : (d > dmax ? dmax : d);
        const float wd = d > 0 ? Wrow[d] : 0.0f;
        const RowPre pre = classify_pre(g, wd, cams[0].band);
        // The wavefront's box, for the band classifier only and only when it
        // decides every row of the wavefront (none undecidable).  With rows
        // in spatial order a camera's frustum misses most wavefronts' boxes,
        // and the per-row classification is skipped for that camera.
        // Lane c tests camera c against the box (C <= 32); the ballot is the
        // set of cameras that cull the whole wavefront.
        const bool box = a.mode == 1 && __ballot(valid && pre.ok == 0) == 0ull && __ballot(valid) != 0ull;
        u32 out_mask = 0u;
        if (box) {
            WaveBox wb;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                wb.lo[i] = wave_min(valid ? g[i] : __builtin_huge_valf());
                wb.hi[i] = wave_max(valid ? g[i] : -__builtin_huge_valf());
            }
            wb.mu = wave_max(valid ? pre.mu : 0.0f);
            wb.dp = wave_max(valid ? pre.dp : 0.0f);
            wb.sig2 = wave_max(valid ? pre.sig2 : 0.0f);
            bool o = false;
            if (lane < C) o = wave_sure_out(wb, cams[lane].cam, cams[lane].band);
            out_mask = (u32)__ballot(o);
        }
        if (valid) {
            u32 undecided = 0;
            for (int c = 0; c < C; ++c) {
                if ((out_mask >> c) & 1u) continue;
                const int cls = a.mode == 1 ? classify_cam(g, pre, cams[c].cam, cams[c].band) : 2;
                mk |= (u32)(cls == 1) << c;
                undecided |= (u32)(cls == 2) << c;
            }
            if (undecided) {
                if (d > 0) {
                    const int64_t row = row0 + r;
                    float mv[10], vv[10];
                    if (a.gst == GS_F32) {
                        for (int j = 0; j < 10; ++j) {
                            mv[j] = mom_load<GS_F32>(a.gm, row, j, false);
                            vv[j] = mom_load<GS_F32>(a.gv, row, j, true);
                        }
                    } else if (a.gst == GS_BF16) {
                        for (int j = 0; j < 10; ++j) {
                            mv[j] = mom_load<GS_BF16>(a.gm, row, j, false);
                            vv[j] = mom_load<GS_BF16>(a.gv, row, j, true);
                        }
                    } else {
                        for (int j = 0; j < 10; ++j) {
                            mv[j] = mom_load<GS_FP8E4M3>(a.gm, row, j, false);
                            vv[j] = mom_load<GS_FP8E4M3>(a.gv, row, j, true);
                        }
                    }
                    for (int j = 0; j < 10; ++j) g[j] = restore1(g[j], mv[j], vv[j], wd, a.lr[j], a.eps, a.rb);
                }
                for (int c = 0; c < C; ++c)
                    if (((undecided >> c) & 1u) && cull_v1(g, cams[c].cam)) mk |= 1u << c;
            }
        }
        if (r < rows) a.mask[row0 + r] = mk;
        const int slab = k * NW + wave;
        const u64 ub = __ballot(mk != 0u);
        if (lane == 0) sCnt[slab][0] = (u32)__popcll(ub);
        for (int c = 0; c < C; ++c) {
            const u64 cb = __ballot((mk >> c) & 1u);
            if (lane == 0) sCnt[slab][1 + c] = (u32)__popcll(cb);
        }
    }
    __syncthreads();
    if (tid < 1 + C) {
        u32 o = 0;
        for (int sl = 0; sl < NSLAB; ++sl) o += sCnt[sl][tid];
        a.cnt[(int64_t)tid * a.stride + tile] = o;
    }
    step_flag(a.step, step_err);
}

// Exclusive prefixes over tiles of every counter in three launches:
// k_multi_reduce sums each group of 64 tiles (one wavefront per group);
// k_multi_gscan scans the group sums of each counter (one block per counter)
// and writes the totals; k_multi_offsets (one wavefront per group) scans the
// group's tiles on top of its group prefix.
__global__ __launch_bounds__(256) void k_multi_reduce(MultiArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t groups = (a.tiles + 63) / 64;
    if (g >= groups) return;
    const int64_t tile = g * 64 + lane;
    for (int j = 0; j < 1 + a.C; ++j) {
        const u64 c = tile < a.tiles ? (u64)a.cnt[(int64_t)j * a.stride + tile] : 0ull;
        const u64 sum = wave_sum_u64(c);
        if (lane == 0) a.grp[(int64_t)j * a.gstride + g] = (u32)sum;
    }
}

// Exclusive prefix over the groups of one counter (block j = counter j), in
// place, and that counter's total: linear in the number of groups.
__global__ __launch_bounds__(kScanThreads) void k_multi_gscan(MultiArgs a)
{
    __shared__ u64 sV[kScanChunk];
    __shared__ u64 sWave[kScanThreads / 64 + 1];
    const int j = blockIdx.x;
    const int64_t groups = (a.tiles + 63) / 64;
    u32 *g = a.grp + (int64_t)j * a.gstride;
    const u64 tot = scan_counts_u32(g, g, groups, sV, sWave);
    if (threadIdx.x == 0) {
        if (j == 0) *a.union_count = (u32)tot;
        else a.cam_count[j - 1] = (u32)tot;
    }
}

// One wavefront per group of 64 tiles: the group's prefix (from
// k_multi_gscan) plus the scan of its tiles' counts, for every counter.
__global__ __launch_bounds__(256) void k_multi_offsets(MultiArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t groups = (a.tiles + 63) / 64;
    if (g >= groups) return;
    const int64_t tile = g * 64 + lane;
    for (int j = 0; j < 1 + a.C; ++j) {
        const u64 base = a.grp[(int64_t)j * a.gstride + g];
        const u64 c = tile < a.tiles ? (u64)a.cnt[(int64_t)j * a.stride + tile] : 0ull;
        u64 inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const u64 y = (u64)__shfl_up((long long)inc, o);
            if (lane >= o) inc += y;
        }
        if (tile < a.tiles) a.off[(int64_t)j * a.stride + tile] = (u32)(base + inc - c);
    }
}

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_multi_ids(MultiArgs a)
{
    constexpr int NW = BLOCK / 64;
    constexpr int TR = BLOCK * IPT;
    constexpr int NSLAB = IPT * NW;
    __shared__ u32 sCnt[NSLAB][kNCnt];
    __shared__ u32 sOff[NSLAB][kNCnt];
    __shared__ u32 sScene;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int C = a.C;
    const int64_t tile = blockIdx.x;
    const int64_t row0 = tile * TR;
    const int rows = (int)min((int64_t)TR, a.n - row0);
    if (tid == 0) {
        int sc = 0;
        while (sc + 1 < a.S && a.scene_row0[sc + 1] <= row0) ++sc;
        sScene = (u32)sc;
    }
    u32 mask[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int r = k * BLOCK + tid;
        const u32 mk = r < rows ? a.mask[row0 + r] : 0u;
        mask[k] = mk;
        const int slab = k * NW + wave;
        const u64 ub = __ballot(mk != 0u);
        if (lane == 0) sCnt[slab][0] = (u32)__popcll(ub);
        for (int c = 0; c < C; ++c) {
            const u64 cb = __ballot((mk >> c) & 1u);
            if (lane == 0) sCnt[slab][1 + c] = (u32)__popcll(cb);
        }
    }
    __syncthreads();
    if (tid < 1 + C) {
        u32 o = a.off[(int64_t)tid * a.stride + tile];
        const int scene = (int)sScene;
        if (row0 == a.scene_row0[scene]) a.scene_start[(int64_t)scene * (1 + C) + tid] = o;
        for (int sl = 0; sl < NSLAB; ++sl) {
            sOff[sl][tid] = o;
            o += sCnt[sl][tid];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const u32 mk = mask[k];
        const int slab = k * NW + wave;
        const u64 ub = __ballot(mk != 0u);
        const u32 p = sOff[slab][0] + lane_rank(ub);
        if (mk && p < a.cap_union) a.union_ids[p] = (u32)(row0 + k * BLOCK + tid);
        // the union row at the start of a chunk of kSumRows positions records,
        // per camera slot, the index of that slot's first entry at or after it
        const bool chunk0 = a.chunk_start && mk && p < a.cap_union && (p % kSumRows) == 0;
        for (int c = 0; c < C; ++c) {
            const bool on = (mk >> c) & 1u;
            const u64 cb = __ballot(on);
            const u32 q = sOff[slab][1 + c] + lane_rank(cb);
            if (on && q < a.cap_cam) a.cam_pos[(size_t)c * a.cap_cam + q] = p;
            if (chunk0) a.chunk_start[(size_t)(p / kSumRows) * C + c] = q;
        }
    }
}

// Deterministic sum of the per-camera gradients onto the union rows:
// out[p] = (...((0 + g_c0) + g_c1) + ...) over the camera slots that see p, in
// slot order.  cam_pos[c] is ascending, so the entries of a block of union
// positions form one contiguous range per camera: read from the chunk starts
// the compaction records, or found by binary search without them.
struct GradSumArgs {
    const u32 *cam_pos, *cam_count, *union_count;
    const u32 *chunk_start;          // per chunk and camera slot: first entry index, or null
    u32 cap_cam, cap_union;
    int32_t C, adim;
    const float *g_cam;              // [C][cap_cam][10 + adim]
    float *out_geo, *out_app;        // [cap_union][10], [cap_union][adim]
};

constexpr int kGsRows = 8;           // rows of a wavefront summed together
constexpr int kGsSlots = 4;          // camera entries per row loaded up front

__device__ __forceinline__ u32 lower_bound_u32(const u32 *a, u32 n, u32 key)
{
    u32 lo = 0, hi = n;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One block per chunk of kSumRows union positions: (1) each camera's entries in
// the chunk (its range of the list) are scattered into an LDS table
// (row, camera) -> entry, with the row's camera bits; (2) one wavefront per
// row (lane = column) adds the row's camera gradients in slot order,
// (((0 + g_c0) + g_c1) + ...), so the sum is deterministic.
__global__ __launch_bounds__(256) void k_grad_sum(GradSumArgs a)
{
    __shared__ u32 sIdx[kSumRows][kMaxCams];
    __shared__ u32 sMask[kSumRows];
    __shared__ u32 sLo[kMaxCams], sOff[kMaxCams + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int D = 10 + a.adim;
    const int C = a.C;
    const u32 U = min(*a.union_count, a.cap_union);
    for (u32 p0 = blockIdx.x * kSumRows; p0 < U; p0 += gridDim.x * kSumRows) {
        for (int e = tid; e < kSumRows; e += 256) sMask[e] = 0u;
        if (tid < C) {
            const u32 nc = min(a.cam_count[tid], a.cap_cam);
            u32 lo, hi;
            if (a.chunk_start) {
                // the chunk's range of each list, recorded by the compaction
                const size_t q = p0 / kSumRows;
                lo = min(a.chunk_start[q * C + tid], nc);
                hi = p0 + kSumRows < U ? min(a.chunk_start[(q + 1) * C + tid], nc) : nc;
            } else {
                const u32 *lst = a.cam_pos + (size_t)tid * a.cap_cam;
                lo = lower_bound_u32(lst, nc, p0);
                hi = lower_bound_u32(lst, nc, p0 + kSumRows);
            }
            sLo[tid] = lo;
            sOff[tid + 1] = hi - lo;
        }
        __syncthreads();
        if (tid == 0) {
            sOff[0] = 0;
            for (int c = 0; c < C; ++c) sOff[c + 1] += sOff[c];
        }
        __syncthreads();
        const u32 total = sOff[C];
        // positions of this chunk: the union list may hold more rows than
        // cap_union (then the camera lists still name the positions past it,
        // and the last chunk's range reaches them); only p0 .. p0 + np - 1 are
        // summed, so entries outside that window are skipped
        const u32 np = min((u32)kSumRows, U - p0);
        for (u32 e = tid; e < total; e += 256) {
            int c = 0;
            while (e >= sOff[c + 1]) ++c;
            const u32 i = sLo[c] + (e - sOff[c]);
            const u32 p = a.cam_pos[(size_t)c * a.cap_cam + i] - p0;
            if (p < np) {
                sIdx[p][c] = i;
                atomicOr(&sMask[p], 1u << c);
            }
        }
        __syncthreads();
        // kGsRows rows of this wavefront at a time: the first kGsSlots camera
        // entries of each are loaded before the first add (rows rarely have
        // more; those take the rest one by one).  Entry addresses are uniform:
        // scalar bases plus the lane's column.  A missing slot adds +0, which
        // leaves the sum's bits unchanged (a sum started at +0 is never -0).
        for (u32 r0 = wave; r0 < np; r0 += 4 * kGsRows) {
            float v[kGsRows][kGsSlots];
            u32 rest[kGsRows];
#pragma unroll
            for (int q = 0; q < kGsRows; ++q) {
                const u32 r = r0 + 4 * q;
                u32 m = r < np ? (u32)__builtin_amdgcn_readfirstlane((int)sMask[r]) : 0u;
#pragma unroll
                for (int sl = 0; sl < kGsSlots; ++sl) {
                    // a zero the compiler cannot fold into the add below (it
                    // would then move the add next to the load and wait there)
                    asm volatile("v_mov_b32 %0, 0" : "=v"(v[q][sl]));
                    if (m) {
                        const int c = __builtin_ctz(m);
                        m &= m - 1u;
                        const u32 idx = (u32)__builtin_amdgcn_readfirstlane((int)sIdx[r][c]);
                        const float *src = a.g_cam + ((u64)c * a.cap_cam + idx) * (u64)D;
                        if (lane < D) v[q][sl] = src[lane];
                    }
                }
                rest[q] = m;
            }
#pragma unroll
            for (int q = 0; q < kGsRows; ++q) {
                const u32 r = r0 + 4 * q;
                float acc = 0.0f;
#pragma unroll
                for (int sl = 0; sl < kGsSlots; ++sl) acc = acc + v[q][sl];
                for (u32 m = rest[q]; m; m &= m - 1u) {
                    const int c = __builtin_ctz(m);
                    const u32 idx = (u32)__builtin_amdgcn_readfirstlane((int)sIdx[r][c]);
                    const float *src = a.g_cam + ((u64)c * a.cap_cam + idx) * (u64)D;
                    acc = acc + (lane < D ? src[lane] : 0.0f);
                }
                if (r < np) {
                    if (lane < 10) a.out_geo[(size_t)(p0 + r) * 10 + lane] = acc;
                    else if (lane < D) a.out_app[(size_t)(p0 + r) * a.adim + (lane - 10)] = acc;
                }
            }
        }
        __syncthreads();
    }
}

__global__ void k_step_advance(int32_t *t) { *t += 1; }

// The advance alone (gs_lut_seek: one launch per step).
__global__ __launch_bounds__(256) void k_lut_advance(StepK step, LutAdv adv)
{
    const float *wrow;
    int dmax, step_err;
    const int t = resolve_step(step, 0, &wrow, &dmax, &step_err);
    if (step_err) {
        step_flag(step, step_err);
        return;
    }
    lut_advance_slice(adv, step, t, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
}

// Read-bandwidth probe in the cull's own access pattern: one block per
// 20 KB tile (5 non-temporal 16-byte loads per thread, all issued before the
// first is used), seven blocks per CU; the last block's tail is guarded.  The
// sum is stored only if it equals a value finite data never sum to, so the
// loads cannot be dropped and nothing is written in practice.
constexpr int kProbeP = 5;
__global__ __launch_bounds__(256, 7) void k_stream_read(const float4 *p, int64_t n4, float *sink)
{
    const int64_t b = (int64_t)blockIdx.x * (kProbeP * 256) + threadIdx.x;
    float4 x[kProbeP];
    if (b + (kProbeP - 1) * 256 < n4) {
#pragma unroll
        for (int k = 0; k < kProbeP; ++k) x[k] = ld_once(p + b + k * 256);
    } else {
#pragma unroll
        for (int k = 0; k < kProbeP; ++k) x[k] = b + k * 256 < n4 ? p[b + k * 256] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < kProbeP; ++k) acc += (x[k].x + x[k].y) + (x[k].z + x[k].w);
    if (acc == -1.5e-38f) *sink = acc;
}

// Row-access probe in the row kernels' pattern: one wavefront per listed row
// (four rows an iteration, every row's loads issued before the first is
// used), 16 bytes a lane, rows of up to 1024 bytes.  RW: every loaded 16
// bytes are stored back unchanged (the same bits), so the probe moves the
// traffic of a read-modify-write of the rows without changing them.  Read
// only: the sum is stored only if it equals a value finite data never sum to.
template <bool RW>
__global__ __launch_bounds__(256) void k_row_probe(const u32 *ids, u32 count, u64 n_rows, float4 *base, u32 row_f4,
                                                   float *sink)
{
    const u32 lane = threadIdx.x & 63u;
    const u32 w = blockIdx.x * 4u + (threadIdx.x >> 6), nw = gridDim.x * 4u;
    float acc = 0.0f;
    for (u32 i = w * 4u; i < count; i += nw * 4u) {
        float4 v[4];
        u32 id[4];
        bool on[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            id[u] = ids[min(i + (u32)u, count - 1u)];
            // ids at or past n_rows are skipped
            on[u] = lane < row_f4 && (u64)id[u] < n_rows;
            v[u] = on[u] ? base[(u64)id[u] * row_f4 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (RW) {
                if (on[u] && i + (u32)u < count) base[(u64)id[u] * row_f4 + lane] = v[u];
            } else {
                acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
            }
        }
    }
    if (!RW && acc == -1.5e-38f) *sink = acc;
}

// ---------------------------------------------------------------------------
// densification: plan (codes + tile counts) -> scan -> apply (row copies)
// ---------------------------------------------------------------------------
struct DensArgs {
    const float *gw, *aw;            // source current values
    int64_t aw_ld;
    int32_t adim, big_on;
    const float *accum, *denom, *radii;
    float thr, log_dense, log_big, logit_min, max_screen, log_split;
    u64 seed;
    int64_t n, tiles;
    uint8_t *code;                   // [n] bit 0 original kept, 1 clone kept, 2 children kept
    u32 *cnt, *off;                  // [3][tiles]
    u32 *totals;                     // [4]
    // apply
    MomRef sgm, sgv, sam, sav;       // source moments
    int32_t gst, ast;
    float *dgw, *daw;
    int64_t daw_ld;
    MomRef dgm, dgv, dam, dav;       // destination moments
    int32_t *dlast;
    int64_t dn;
    int32_t step, pad;
};

__device__ __forceinline__ u32 dens_code(const DensArgs &a, int64_t i)
{
    const float *g = a.gw + i * 10;
    const float den = a.denom[i];
    const float gr = den > 0.0f ? a.accum[i] / den : 0.0f;
    const bool grad = gr >= a.thr;
    float smax = g[3];
    if (g[4] > smax) smax = g[4];
    if (g[5] > smax) smax = g[5];
    const bool clone = grad && (smax <= a.log_dense);
    const bool split = grad && (smax > a.log_dense);
    const bool low = a.aw[i * a.aw_ld] < a.logit_min;
    const bool big = a.big_on && (smax > a.log_big);
    const bool screen = a.radii && a.max_screen > 0.0f && a.radii[i] > a.max_screen;
    const float cmax = smax - a.log_split;
    const bool cbig = a.big_on && (cmax > a.log_big);
    u32 c = 0;
    if (!split && !low && !big && !screen) c |= 1u;
    if (clone && !low && !big) c |= 2u;
    if (split && !low && !cbig) c |= 4u;
    return c;
}

__global__ __launch_bounds__(kCullBlock) void k_dens_plan(DensArgs a)
{
    __shared__ u32 sCnt[kCullIpt * 4][3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = blockIdx.x, row0 = tile * kCullTile;
#pragma unroll
    for (int k = 0; k < kCullIpt; ++k) {
        const int64_t i = row0 + k * kCullBlock + tid;
        const u32 c = i < a.n ? dens_code(a, i) : 0u;
        if (i < a.n) a.code[i] = (uint8_t)c;
        const int slab = k * 4 + wave;
        const u64 b0 = __ballot(c & 1u), b1 = __ballot(c & 2u), b2 = __ballot(c & 4u);
        if (lane == 0) {
            sCnt[slab][0] = (u32)__popcll(b0);
            sCnt[slab][1] = (u32)__popcll(b1);
            sCnt[slab][2] = 2u * (u32)__popcll(b2);
        }
    }
    __syncthreads();
    if (tid < 3) {
        u32 o = 0;
        for (int sl = 0; sl < kCullIpt * 4; ++sl) o += sCnt[sl][tid];
        a.cnt[(int64_t)tid * a.tiles + tile] = o;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_dens_scan(DensArgs a)
{
    __shared__ u64 sV[kScanChunk];
    __shared__ u64 sWave[kScanThreads / 64 + 1];
    for (int j = 0; j < 3; ++j) {
        const u64 tot = scan_counts_u32(a.cnt + (int64_t)j * a.tiles, a.off + (int64_t)j * a.tiles, a.tiles, sV, sWave);
        if (threadIdx.x == 0) a.totals[j] = (u32)tot;
    }
}

// One block per tile: output positions of the tile's rows from ballots and
// the tile prefixes, then one wavefront per row copies it (lane c < 10: G
// column c, lane 10 + c: A column c).
template <int GST, int AST>
__global__ __launch_bounds__(kCullBlock) void k_dens_apply(DensArgs a)
{
    __shared__ u32 sCnt[kCullIpt * 4][3];
    __shared__ u32 sOff[kCullIpt * 4][3];
    __shared__ int64_t sPos[kCullTile][3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = blockIdx.x, row0 = tile * kCullTile;
    const int rows = (int)min((int64_t)kCullTile, a.n - row0);
    const u64 lt = (1ull << lane) - 1ull;
    u32 cv[kCullIpt];
    u64 bb[kCullIpt][3];
#pragma unroll
    for (int k = 0; k < kCullIpt; ++k) {
        const int r = k * kCullBlock + tid;
        cv[k] = r < rows ? (u32)a.code[row0 + r] : 0u;
        const int slab = k * 4 + wave;
        bb[k][0] = __ballot(cv[k] & 1u);
        bb[k][1] = __ballot(cv[k] & 2u);
        bb[k][2] = __ballot(cv[k] & 4u);
        if (lane == 0) {
            sCnt[slab][0] = (u32)__popcll(bb[k][0]);
            sCnt[slab][1] = (u32)__popcll(bb[k][1]);
            sCnt[slab][2] = 2u * (u32)__popcll(bb[k][2]);
        }
    }
    __syncthreads();
    if (tid < 3) {
        u32 o = a.off[(int64_t)tid * a.tiles + tile];
        if (tid >= 1) o += a.totals[0];
        if (tid == 2) o += a.totals[1];
        for (int sl = 0; sl < kCullIpt * 4; ++sl) {
            sOff[sl][tid] = o;
            o += sCnt[sl][tid];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCullIpt; ++k) {
        const int r = k * kCullBlock + tid;
        const int slab = k * 4 + wave;
        if (r < rows) {
            sPos[r][0] = (cv[k] & 1u) ? (int64_t)(sOff[slab][0] + (u32)__popcll(bb[k][0] & lt)) : -1;
            sPos[r][1] = (cv[k] & 2u) ? (int64_t)(sOff[slab][1] + (u32)__popcll(bb[k][1] & lt)) : -1;
            sPos[r][2] = (cv[k] & 4u) ? (int64_t)(sOff[slab][2] + 2u * (u32)__popcll(bb[k][2] & lt)) : -1;
        }
    }
    __syncthreads();

    const bool isG = lane < 10;
    const bool act = lane < 10 + a.adim;
    const int ca = lane - 10;
    for (int r = wave; r < rows; r += kCullBlock / 64) {
        const int64_t i = row0 + r;
        const int64_t p0 = sPos[r][0], p1 = sPos[r][1], p2 = sPos[r][2];
        if (p0 < 0 && p1 < 0 && p2 < 0) continue;
        float x = 0.0f, m = 0.0f, v = 0.0f;
        if (act) {
            x = isG ? a.gw[i * 10 + lane] : a.aw[i * a.aw_ld + ca];
            if (p0 >= 0) {
                if (isG) {
                    m = mom_load<GST>(a.sgm, i, lane, false);
                    v = mom_load<GST>(a.sgv, i, lane, true);
                } else {
                    m = mom_load<AST>(a.sam, i, ca, false);
                    v = mom_load<AST>(a.sav, i, ca, true);
                }
            }
        }
        // copies of the source row: the original keeps its moments, a clone starts at zero
        for (int kind = 0; kind < 2; ++kind) {
            const int64_t o = kind == 0 ? p0 : p1;
            if (o < 0 || o >= a.dn || !act) continue;
            const float mo = kind == 0 ? m : 0.0f, vo = kind == 0 ? v : 0.0f;
            if (isG) {
                a.dgw[o * 10 + lane] = x;
                mom_store<GST>(a.dgm, o, lane, mo, 0u, false);
                mom_store<GST>(a.dgv, o, lane, vo, 0u, true);
            } else {
                a.daw[o * a.daw_ld + ca] = x;
                mom_store<AST>(a.dam, o, ca, mo, 0u, false);
                mom_store<AST>(a.dav, o, ca, vo, 0u, true);
            }
        }
        if (lane == 0) {
            if (p0 >= 0 && p0 < a.dn) a.dlast[p0] = a.step;
            if (p1 >= 0 && p1 < a.dn) a.dlast[p1] = a.step;
        }
        if (p2 < 0) continue;
        // two split children: scales s - log 1.6, positions mu + Q (exp(s) z)
        float cx = x;
        if (isG && lane < 6) {
            const float *g = a.gw + i * 10;
            float qw = g[6], qx = g[7], qy = g[8], qz = g[9];
            const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
            const float inv = 1.0f / sqrtf(n2);
            qw = qw * inv;
            qx = qx * inv;
            qy = qy * inv;
            qz = qz * inv;
            float Qr[3];
            if (lane == 0) {
                Qr[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
                Qr[1] = 2.0f * (qx * qy - qw * qz);
                Qr[2] = 2.0f * (qx * qz + qw * qy);
            } else if (lane == 1) {
                Qr[0] = 2.0f * (qx * qy + qw * qz);
                Qr[1] = 1.0f - 2.0f * (qx * qx + qz * qz);
                Qr[2] = 2.0f * (qy * qz - qw * qx);
            } else {
                Qr[0] = 2.0f * (qx * qz - qw * qy);
                Qr[1] = 2.0f * (qy * qz + qw * qx);
                Qr[2] = 1.0f - 2.0f * (qx * qx + qy * qy);
            }
            const float sg0 = exp_cw(g[3]), sg1 = exp_cw(g[4]), sg2 = exp_cw(g[5]);
            for (int j = 0; j < 2; ++j) {
                const int64_t o = p2 + j;
                if (o >= a.dn) continue;
                float val;
                if (lane < 3) {
                    float z[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        const u64 h = sm_at(sm_at(sm_at(a.seed, (u64)i), (u64)j), (u64)ax);
                        const u64 u = (h & 0xffffull) + ((h >> 16) & 0xffffull) + ((h >> 32) & 0xffffull) +
                                      ((h >> 48) & 0xffffull);
                        const double inv_sd = 1.0 / sqrt(4.0 * (65536.0 * 65536.0 - 1.0) / 12.0);
                        z[ax] = (float)(((double)u - 131070.0) * inv_sd);
                    }
                    const float v0 = sg0 * z[0], v1 = sg1 * z[1], v2 = sg2 * z[2];
                    val = g[lane] + ((Qr[0] * v0 + Qr[1] * v1) + Qr[2] * v2);
                } else {
                    val = g[lane] - a.log_split;
                }
                a.dgw[o * 10 + lane] = val;
            }
            cx = 0.0f;  // written above
        }
        for (int j = 0; j < 2; ++j) {
            const int64_t o = p2 + j;
            if (o >= a.dn || !act) continue;
            if (isG) {
                if (lane >= 6) a.dgw[o * 10 + lane] = cx;
                mom_store<GST>(a.dgm, o, lane, 0.0f, 0u, false);
                mom_store<GST>(a.dgv, o, lane, 0.0f, 0u, true);
            } else {
                a.daw[o * a.daw_ld + ca] = cx;
                mom_store<AST>(a.dam, o, ca, 0.0f, 0u, false);
                mom_store<AST>(a.dav, o, ca, 0.0f, 0u, true);
            }
            if (lane == 0) a.dlast[o] = a.step;
        }
    }
}

}  // namespace

namespace {

// autotuned variants of the batched cull: (block size, rows per thread) with
// block in 64..1024 and a tile of block x rows <= 1024 rows (scenes start at
// multiples of 1024 rows and a tile must lie in one scene)
constexpr int kMultiVariants = GS_MULTI_VARIANTS;

int64_t multi_ws_bytes(int64_t n)
{
    const int64_t tiles = (n + kMultiMinTile - 1) / kMultiMinTile;
    const int64_t groups = (tiles + 63) / 64;
    return gsdp::kWsHeader + 2 * tiles * kNCnt * 4 + groups * kNCnt * 4 + 4 * ((n + 1) / 2 * 2);
}

int multi_args(const gs_model *model, const gs_multi *d, int64_t step, void *ws, size_t ws_bytes, MultiArgs &a)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!d || !step_ok(model, step)) return GS_EINVAL;
    if (model->max_defer != 0 || model->geo_mode != 0 || model->optimizer != GS_OPT_ADAM) return GS_EUNSUPPORTED;
    if (d->n_scenes < 1 || d->cams_per_scene < 1 || d->cams_per_scene > kMaxCams || d->n_sets < 1) return GS_EINVAL;
    if (d->variant < 0 || d->variant >= kMultiVariants) return GS_EINVAL;
    if (!d->scene_row0 || !d->cams || !d->union_ids || !d->union_count || !d->cam_pos || !d->cam_count ||
        !d->scene_start)
        return GS_EINVAL;
    if (!ws || !aligned(ws, 256) || (int64_t)ws_bytes < multi_ws_bytes(model->n)) return GS_ESPACE;
    memset(&a, 0, sizeof a);
    a.gw = model->geo.w;
    a.gm = {model->geo.m, model->geo.m_scale, model->geo.m_ld};
    a.gv = {model->geo.v, model->geo.v_scale, model->geo.v_ld};
    a.gst = model->geo.state;
    a.rb = restore_bound(model->beta1, model->beta2);
    a.mode = (model->cull_mode == 1 && model->eps > 0.0 && std::isfinite(a.rb)) ? 1 : 0;
    a.eps = (float)model->eps;
    a.last = model->last_step;
    a.n = model->n;
    a.step = step_k(model, step);
    for (int c = 0; c < 10; ++c) a.lr[c] = model->geo.lr[c];
    a.S = d->n_scenes;
    a.C = d->cams_per_scene;
    a.n_sets = d->n_sets;
    a.scene_row0 = d->scene_row0;
    a.cams = static_cast<const CamPack *>(d->cams);
    a.union_ids = d->union_ids;
    a.union_count = d->union_count;
    a.cam_pos = d->cam_pos;
    a.cam_count = d->cam_count;
    a.cap_union = d->cap_union;
    a.cap_cam = d->cap_cam;
    a.scene_start = d->scene_start;
    a.chunk_start = d->chunk_start;
    char *wsb = static_cast<char *>(ws);
    const int64_t max_tiles = (model->n + kMultiMinTile - 1) / kMultiMinTile;
    a.cnt = reinterpret_cast<u32 *>(wsb + gsdp::kWsHeader);
    a.off = a.cnt + max_tiles * kNCnt;
    a.gstride = (max_tiles + 63) / 64;
    a.grp = a.off + max_tiles * kNCnt;
    a.mask = a.grp + a.gstride * kNCnt;
    a.tiles = max_tiles;  // replaced per variant in launch_multi
    return GS_OK;
}

// The state buffers are laid out for the smallest tile; a variant with
// larger tiles uses the first n/TR entries of each half.
template <int BLOCK, int IPT>
void launch_multi_t(MultiArgs a, int64_t n, int64_t max_tiles, hipStream_t st)
{
    constexpr int TR = BLOCK * IPT;
    a.tiles = (n + TR - 1) / TR;
    a.stride = max_tiles;
    a.tile_rows = TR;
    if (a.tiles > 0) hipLaunchKernelGGL((k_cull_multi<BLOCK, IPT>), dim3((unsigned)a.tiles), dim3(BLOCK), 0, st, a);
    const int64_t groups = (a.tiles + 63) / 64;
    const unsigned gblocks = (unsigned)((groups + 3) / 4);
    if (groups > 0) hipLaunchKernelGGL(k_multi_reduce, dim3(gblocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_multi_gscan, dim3((unsigned)(1 + a.C)), dim3(kScanThreads), 0, st, a);
    if (groups > 0) hipLaunchKernelGGL(k_multi_offsets, dim3(gblocks), dim3(256), 0, st, a);
    if (a.tiles > 0) hipLaunchKernelGGL((k_multi_ids<BLOCK, IPT>), dim3((unsigned)a.tiles), dim3(BLOCK), 0, st, a);
}

int launch_multi(int variant, const MultiArgs &a, int64_t n, hipStream_t st)
{
    const int64_t max_tiles = (n + kMultiMinTile - 1) / kMultiMinTile;
    switch (variant) {
    case 0: launch_multi_t<64, 1>(a, n, max_tiles, st); break;
    case 1: launch_multi_t<64, 2>(a, n, max_tiles, st); break;
    case 2: launch_multi_t<64, 4>(a, n, max_tiles, st); break;
    case 3: launch_multi_t<64, 8>(a, n, max_tiles, st); break;
    case 4: launch_multi_t<64, 16>(a, n, max_tiles, st); break;
    case 5: launch_multi_t<128, 1>(a, n, max_tiles, st); break;
    case 6: launch_multi_t<128, 2>(a, n, max_tiles, st); break;
    case 7: launch_multi_t<128, 4>(a, n, max_tiles, st); break;
    case 8: launch_multi_t<128, 8>(a, n, max_tiles, st); break;
    case 9: launch_multi_t<256, 1>(a, n, max_tiles, st); break;
    case 10: launch_multi_t<256, 2>(a, n, max_tiles, st); break;
    case 11: launch_multi_t<256, 4>(a, n, max_tiles, st); break;
    case 12: launch_multi_t<512, 1>(a, n, max_tiles, st); break;
    case 13: launch_multi_t<512, 2>(a, n, max_tiles, st); break;
    default: launch_multi_t<1024, 1>(a, n, max_tiles, st); break;
    }
    return launched("gs_cull_multi");
}

}  // namespace

namespace {

int cull_launch(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids, uint32_t *count_dev,
                uint32_t capacity, char *wsb, hipStream_t st, const void *cams = nullptr, int32_t n_cams = 0);

// Launch the move of the tables' restore rows from `step` to step + 1.
int lut_advance(const gs_model *m, int64_t step, hipStream_t st)
{
    const gsdp::LutLayout L = gsdp::lut_layout(m->lut_max_steps, m->max_defer);
    const int64_t blocks = std::min<int64_t>((L.nrow + 255) / 256, 1024);
    hipLaunchKernelGGL(k_lut_advance, dim3((unsigned)blocks), dim3(256), 0, st, step_k(m, step), lut_adv(m));
    return launched("table advance");
}

// Workspace of gs_cull_noalloc: one array per GPU, zero at load (static
// storage), held until the process ends.  Host code must not pass `scratch`
// itself to a kernel (on the host it names a host-side stand-in); its device
// address comes from hipGetSymbolAddress once per device, with that device
// current, and only that address is used.
__device__ __align__(256) unsigned char scratch[GS_CULL_NOALLOC_MAX_WS];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices];

int scratch_ptr(char **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        snprintf(g_err, sizeof g_err, "gs_cull_noalloc: no usable current device (%d)", dev);
        return GS_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            snprintf(g_err, sizeof g_err, "gs_cull_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return GS_EHIP;
        }
        g_scratch_dev[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_dev[dev];
    return GS_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *gs_status_string(int s)
{
    switch (s) {
    case GS_OK: return "GS_OK";
    case GS_EINVAL: return "GS_EINVAL: invalid argument";
    case GS_EHIP: return "GS_EHIP: HIP runtime error";
    case GS_EUNSUPPORTED: return "GS_EUNSUPPORTED: unsupported mode or dtype";
    case GS_ESPACE: return "GS_ESPACE: buffer too small";
    default: return "unknown gs_status";
    }
}

const char *gs_last_hip_error(void) { return g_err; }

int gs_device_cu_count(void) { return cu_count(); }

int gs_lut_bytes(int32_t max_steps, int32_t max_defer, size_t *bytes)
{
    if (!bytes || max_steps < 1 || max_defer < 0) return GS_EINVAL;
    *bytes = (size_t)gsdp::lut_total_bytes(max_steps, max_defer, 0);
    return GS_OK;
}

int gs_lut_build_schedule_host(double beta1, double beta2, int32_t max_steps, int32_t max_defer, const double *lr_scale,
                               void *lut_host, size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes(max_steps, max_defer, &need);
    if (rc) return rc;
    if (!lut_host || !aligned(lut_host, 8)) return GS_EINVAL;
    if (!(beta1 > 0.0 && beta1 < 1.0 && beta2 > 0.0 && beta2 < 1.0)) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    if (lr_scale)
        for (int64_t t = 0; t <= (int64_t)max_steps + 1; ++t)
            if (!(lr_scale[t] >= 0.0) || !std::isfinite(lr_scale[t])) return GS_EINVAL;
    return gsdp::build_lut_host(beta1, beta2, max_steps, max_defer, lr_scale, lut_host, (int64_t)bytes) == 0
               ? GS_OK
               : GS_ESPACE;
}

int gs_lut_build_host(double beta1, double beta2, int32_t max_steps, int32_t max_defer, void *lut_host,
                      size_t bytes)
{
    return gs_lut_build_schedule_host(beta1, beta2, max_steps, max_defer, nullptr, lut_host, bytes);
}

int gs_lut_build_schedule(double beta1, double beta2, int32_t max_steps, int32_t max_defer, const double *lr_scale,
                          void *lut_dev, size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes(max_steps, max_defer, &need);
    if (rc) return rc;
    if (!lut_dev) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    std::vector<double> host(need / sizeof(double));
    rc = gs_lut_build_schedule_host(beta1, beta2, max_steps, max_defer, lr_scale, host.data(), need);
    if (rc) return rc;
    hipError_t e = hipMemcpy(lut_dev, host.data(), need, hipMemcpyHostToDevice);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_lut_build: hipMemcpy");
}

int gs_lut_build(double beta1, double beta2, int32_t max_steps, int32_t max_defer, void *lut_dev, size_t bytes)
{
    return gs_lut_build_schedule(beta1, beta2, max_steps, max_defer, nullptr, lut_dev, bytes);
}

int gs_lut_build_sgd_momentum_host(double momentum, int32_t max_steps, int32_t max_defer, const double *lr_scale,
                                   void *lut_host, size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes(max_steps, max_defer, &need);
    if (rc) return rc;
    if (!lut_host || !aligned(lut_host, 8)) return GS_EINVAL;
    if (!(momentum > 0.0 && momentum < 1.0)) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    if (lr_scale)
        for (int64_t t = 0; t <= (int64_t)max_steps + 1; ++t)
            if (!(lr_scale[t] >= 0.0) || !std::isfinite(lr_scale[t])) return GS_EINVAL;
    return gsdp::build_lut_sgdm_host(momentum, max_steps, max_defer, lr_scale, lut_host, (int64_t)bytes) == 0
               ? GS_OK
               : GS_ESPACE;
}

int gs_lut_build_sgd_momentum(double momentum, int32_t max_steps, int32_t max_defer, const double *lr_scale,
                              void *lut_dev, size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes(max_steps, max_defer, &need);
    if (rc) return rc;
    if (!lut_dev) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    std::vector<double> host(need / sizeof(double));
    rc = gs_lut_build_sgd_momentum_host(momentum, max_steps, max_defer, lr_scale, host.data(), need);
    if (rc) return rc;
    hipError_t e = hipMemcpy(lut_dev, host.data(), need, hipMemcpyHostToDevice);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_lut_build_sgd_momentum: hipMemcpy");
}

int gs_lut_seek_host(void *lut_host, size_t bytes, int64_t step)
{
    if (!lut_host || !aligned(lut_host, 8)) return GS_EINVAL;
    return gsdp::seek_lut_host(lut_host, (int64_t)bytes, step) == 0 ? GS_OK : GS_EINVAL;
}

int gs_lut_seek(const gs_model *model, int64_t step, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (step < 1 || step > (int64_t)model->lut_max_steps + 1) return GS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    gsdp::LutHeader h;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(&h, model->lut, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "gs_lut_seek");
    if (h.T != model->lut_max_steps || h.K != model->max_defer) return GS_EINVAL;
    const int64_t cur = h.t_row[0] > h.t_row[1] ? h.t_row[0] : h.t_row[1];
    if (cur < 1 || step < cur) return GS_EINVAL;
    for (int64_t t = cur; t < step; ++t) {
        rc = lut_advance(model, t, st);
        if (rc) return rc;
    }
    e = hipStreamSynchronize(st);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_lut_seek");
}

int gs_lut_bytes_adamw(const gs_model *model, size_t *bytes)
{
    if (!model || !bytes) return GS_EINVAL;
    size_t base = 0;
    int rc = gs_lut_bytes(model->lut_max_steps, model->max_defer, &base);
    if (rc) return rc;
    float rates[gsdp::kMaxDecayClasses];
    const int nc = decay_classes(model, rates, nullptr);
    if (nc < 0) return GS_EUNSUPPORTED;
    *bytes = (size_t)gsdp::lut_total_bytes(model->lut_max_steps, model->max_defer, nc);
    return GS_OK;
}

int gs_lut_build_adamw_host(const gs_model *model, double weight_decay, const double *lr_scale, void *lut_host,
                            size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes_adamw(model, &need);
    if (rc) return rc;
    if (!lut_host || !aligned(lut_host, 8) || !(weight_decay >= 0.0) || !std::isfinite(weight_decay))
        return GS_EINVAL;
    if (!(model->beta1 > 0.0 && model->beta1 < 1.0 && model->beta2 > 0.0 && model->beta2 < 1.0)) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    const int32_t T = model->lut_max_steps;
    if (lr_scale)
        for (int64_t t = 0; t <= (int64_t)T + 1; ++t)
            if (!(lr_scale[t] >= 0.0) || !std::isfinite(lr_scale[t])) return GS_EINVAL;
    float rates[gsdp::kMaxDecayClasses];
    const int nc = decay_classes(model, rates, nullptr);
    return gsdp::build_lut_adamw_host(model->beta1, model->beta2, weight_decay, rates, nc, T, model->max_defer,
                                      lr_scale, lut_host, (int64_t)bytes) == 0
               ? GS_OK
               : GS_ESPACE;
}

int gs_lut_build_adamw(const gs_model *model, double weight_decay, const double *lr_scale, void *lut_dev,
                       size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes_adamw(model, &need);
    if (rc) return rc;
    if (!lut_dev) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    std::vector<double> host(need / sizeof(double));
    rc = gs_lut_build_adamw_host(model, weight_decay, lr_scale, host.data(), need);
    if (rc) return rc;
    hipError_t e = hipMemcpy(lut_dev, host.data(), need, hipMemcpyHostToDevice);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_lut_build_adamw: hipMemcpy");
}

int gs_workspace_bytes(const gs_model *model, size_t *bytes)
{
    if (!model || !bytes || model->n < 0 || model->max_defer < 0) return GS_EINVAL;
    *bytes = (size_t)gsdp::ws_bytes_for(model->n, model->max_defer, has_fp8(model));
    return GS_OK;
}

int gs_cull(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids, uint32_t *count_dev,
            uint32_t capacity, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!cam || !count_dev || !ws || (capacity > 0 && !ids)) return GS_EINVAL;
    if (!step_ok(model, step)) return GS_EINVAL;
    if (!(cam->fx > 0.0f && cam->fy > 0.0f) || cam->width <= 0 || cam->height <= 0) return GS_EINVAL;
    if (!aligned(ws, 256)) return GS_EINVAL;
    if ((int64_t)ws_bytes < gsdp::ws_bytes_for(model->n, model->max_defer, has_fp8(model))) return GS_ESPACE;
    return cull_launch(model, cam, step, ids, count_dev, capacity, static_cast<char *>(ws), (hipStream_t)stream);
}

int gs_cull_table(const gs_model *model, const void *cams, int32_t n_cams, int64_t step, uint32_t *ids,
                  uint32_t *count_dev, uint32_t capacity, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!cams || n_cams < 1 || !count_dev || !ws || (capacity > 0 && !ids)) return GS_EINVAL;
    if (!step_ok(model, step)) return GS_EINVAL;
    if (!aligned(ws, 256) || !aligned(cams, 16)) return GS_EINVAL;
    if ((int64_t)ws_bytes < gsdp::ws_bytes_for(model->n, model->max_defer, has_fp8(model))) return GS_ESPACE;
    // only the summary cull reads its camera from device memory
    const bool band = model->cull_mode == 1 && model->eps > 0.0 && std::isfinite(restore_bound(model->beta1, model->beta2));
    if (!band || !model->cull_sum || model->geo_mode != 0 || model->optimizer != GS_OPT_ADAM) return GS_EUNSUPPORTED;
    return cull_launch(model, nullptr, step, ids, count_dev, capacity, static_cast<char *>(ws), (hipStream_t)stream,
                       cams, n_cams);
}

int gs_cull_chunk_flags(const gs_model *model, const gs_camera *cam, int64_t step, uint8_t *flags, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!cam || (model->n > 0 && !flags)) return GS_EINVAL;
    if (!step_ok(model, step)) return GS_EINVAL;
    if (!(cam->fx > 0.0f && cam->fy > 0.0f) || cam->width <= 0 || cam->height <= 0) return GS_EINVAL;
    const bool band = model->cull_mode == 1 && model->eps > 0.0 && std::isfinite(restore_bound(model->beta1, model->beta2));
    if (!band || !model->cull_sum || !model->cull_chunk || model->geo_mode != 0 || model->optimizer != GS_OPT_ADAM ||
        model->max_defer != 0)
        return GS_EUNSUPPORTED;
    if (model->n == 0) return GS_OK;
    CamK ck;
    BandK bk;
    pack_camera(model, cam, ck, bk);
    const int64_t chunks = (model->n + kChunkRows - 1) / kChunkRows;
    hipLaunchKernelGGL(k_chunk_flags, dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float4 *>(model->cull_chunk), chunks, step_k(model, step).hdr, ck, bk,
                       flags);
    return launched("gs_cull_chunk_flags");
}

int gs_cull_noalloc(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids, uint32_t *count_dev,
                    uint32_t capacity, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!cam || !count_dev || (capacity > 0 && !ids)) return GS_EINVAL;
    if (!step_ok(model, step)) return GS_EINVAL;
    if (!(cam->fx > 0.0f && cam->fy > 0.0f) || cam->width <= 0 || cam->height <= 0) return GS_EINVAL;
    // the saturated-row list and the dense geometric update read this cull's
    // workspace in the following update call, which cannot reach the array
    if (model->max_defer != 0 || model->geo_mode != 0) return GS_EUNSUPPORTED;
    if (gsdp::ws_bytes_for(model->n, 0, 0) > (int64_t)GS_CULL_NOALLOC_MAX_WS) {
        snprintf(g_err, sizeof g_err, "gs_cull_noalloc: the model needs %lld workspace bytes, the library's "
                 "array holds %lld", (long long)gsdp::ws_bytes_for(model->n, 0, 0),
                 (long long)GS_CULL_NOALLOC_MAX_WS);
        return GS_ESPACE;
    }
    char *wsb = nullptr;
    rc = scratch_ptr(&wsb);
    if (rc) return rc;
    return cull_launch(model, cam, step, ids, count_dev, capacity, wsb, (hipStream_t)stream);
}

int gs_cull_summary_build(const gs_model *model, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!model->cull_sum) return GS_EINVAL;
    if (model->n == 0) return GS_OK;
    const int cu = cu_count();
    const int64_t blocks = std::min<int64_t>((model->n + 255) / 256, (int64_t)(cu > 0 ? cu : 256) * 16);
    hipLaunchKernelGGL(k_cull_summary_build, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, model->geo.w,
                       model->last_step, reinterpret_cast<float4 *>(model->cull_sum), model->n);
    rc = launched("gs_cull_summary_build");
    if (rc || !model->cull_chunk) return rc;
    const int64_t chunks = (model->n + kChunkRows - 1) / kChunkRows;
    hipLaunchKernelGGL(k_cull_chunk_build, dim3((unsigned)chunks), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float4 *>(model->cull_sum), model->n, model->cull_chunk);
    return launched("gs_cull_summary_build (chunks)");
}

}  // extern "C"

namespace {

template <bool NT, bool PACKED, int TPB>
void launch_cull_sum_c(bool camdev, hipStream_t st, const CullArgs &a)
{
    const dim3 grid((unsigned)((a.tiles + TPB - 1) / TPB));
    if (camdev) hipLaunchKernelGGL((k_cull_sum<NT, TPB, PACKED, true>), grid, dim3(kCullBlock), 0, st, a);
    else hipLaunchKernelGGL((k_cull_sum<NT, TPB, PACKED, false>), grid, dim3(kCullBlock), 0, st, a);
}

template <int TPB>
void launch_cull_sum_t(bool nt, bool packed, bool camdev, hipStream_t st, const CullArgs &a)
{
    if (nt && packed) launch_cull_sum_c<true, true, TPB>(camdev, st, a);
    else if (packed) launch_cull_sum_c<false, true, TPB>(camdev, st, a);
    else if (nt) launch_cull_sum_c<true, false, TPB>(camdev, st, a);
    else launch_cull_sum_c<false, false, TPB>(camdev, st, a);
}

// the summary cull: two tiles a block, four with chunk decisions
void launch_cull_sum(bool nt, bool packed, bool camdev, hipStream_t st, const CullArgs &a)
{
    if (a.chunk_flags) launch_cull_sum_t<kCullSumChunkTiles>(nt, packed, camdev, st, a);
    else launch_cull_sum_t<kCullSumTiles>(nt, packed, camdev, st, a);
}

// The cull and ordered compaction of gs_cull on the workspace `wsb` (checked
// by the caller).  With a camera table (`cams`, n_cams records; cam unused)
// only the summary cull runs (the caller checked that the model has it).
int cull_launch(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids, uint32_t *count_dev,
                uint32_t capacity, char *wsb, hipStream_t st, const void *cams, int32_t n_cams)
{
    CullArgs a;
    memset(&a, 0, sizeof a);
    a.gw = model->geo.w;
    a.gm = {model->geo.m, model->geo.m_scale, model->geo.m_ld};
    a.gv = {model->geo.v, model->geo.v_scale, model->geo.v_ld};
    a.gst = model->geo.state;
    a.rb = restore_bound(model->beta1, model->beta2);
    a.last = model->last_step;
    a.n = model->n;
    a.step = step_k(model, step);
    for (int c = 0; c < 10; ++c) a.lr[c] = model->geo.lr[c];
    a.eps = (float)model->eps;
    // the band cull needs eps > 0 (with eps = 0 a row with m = v = 0 restores
    // to NaN) and a finite restore bound; otherwise the exact cull runs
    a.mode = (model->cull_mode == 1 && model->eps > 0.0 && std::isfinite(a.rb)) ? 1 : 0;
    // the band bound rests on |m|/sqrt(v) <= rb, which a momentum buffer lacks
    a.sgd = model->optimizer == GS_OPT_SGD_MOMENTUM;
    // with weight decay a restore also moves w by (1 - P) |w|, outside the band bound
    a.adamw = model->optimizer == GS_OPT_ADAMW;
    if (a.sgd || a.adamw) a.mode = 0;
    if (a.adamw) {
        float rates[gsdp::kMaxDecayClasses];
        uint8_t cls[64];
        decay_classes(model, rates, cls);
        for (int j = 0; j < 10; ++j) a.cls[j] = cls[j];
        adamw_ptrs(model, &a.aw_base, &a.aw_per, &a.aw_nW);
    }
    if (cams) {
        a.cams = static_cast<const CamPack *>(cams);
        a.n_cams = n_cams;
    } else {
        pack_camera(model, cam, a.cam, a.band);
        pack_side(cam, a.band, a.side);
    }
    a.geo_dense = model->geo_mode == 1;
    a.K = model->max_defer;
    const int64_t n = model->n;
    a.tiles = gsdp::cull_tiles(n);
    a.tile_vs = reinterpret_cast<u64 *>(wsb + gsdp::ws_cnt_offset(n));
    a.tile_rest = reinterpret_cast<u32 *>(wsb + gsdp::ws_cnt_offset(n) + 8 * a.tiles);
    a.keep_bits = reinterpret_cast<u64 *>(wsb + gsdp::ws_keep_offset(n));
    a.sat_bits = model->max_defer > 0 ? reinterpret_cast<u64 *>(wsb + gsdp::ws_satbits_offset(n)) : nullptr;
    if (a.tiles > 0x7fffffff) return GS_EINVAL;
    a.sum = reinterpret_cast<const float4 *>(model->cull_sum);
    a.chunk = (model->cull_sum && model->max_defer == 0) ? reinterpret_cast<const float4 *>(model->cull_chunk)
                                                          : nullptr;
    if (a.cams && !(a.mode == 1 && a.sum && !a.geo_dense)) return GS_EUNSUPPORTED;
    if (a.tiles > 0) {
        if (a.mode == 1 && a.sum && !a.geo_dense) {
            // the summary (and the last step past 2^16 steps): 16 (20) bytes a row
            const bool packed = model->lut_max_steps <= 65536;
            const bool nt = (int64_t)n * (packed ? 16 : 20) > kLastLevelCacheBytes;
            if (a.chunk) {
                a.chunk_flags = reinterpret_cast<u32 *>(wsb + gsdp::ws_chunk_offset(n, model->max_defer));
                if (a.tiles > kDirectTiles) {
                    a.grp_vs = reinterpret_cast<u64 *>(wsb + gsdp::ws_grp_offset(n));
                    a.grp_rest = a.grp_vs + gsdp::cull_groups(n);
                }
                const unsigned cb = (unsigned)((gsdp::cull_chunks(n) + 255) / 256);
                if (a.cams) hipLaunchKernelGGL(k_chunk_scan<true>, dim3(cb), dim3(256), 0, st, a);
                else hipLaunchKernelGGL(k_chunk_scan<false>, dim3(cb), dim3(256), 0, st, a);
            }
            launch_cull_sum(nt, packed, a.cams != nullptr, st, a);
        } else if ((int64_t)n * 44 > kLastLevelCacheBytes) {
            // geometry and last step: 44 bytes a row
            hipLaunchKernelGGL(k_cull<true>, dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
        } else {
            hipLaunchKernelGGL(k_cull<false>, dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
        }
        int rc1 = launched("gs_cull (tiles)");
        if (rc1) return rc1;
    }
    IdsArgs ia;
    memset(&ia, 0, sizeof ia);
    ia.keep_bits = a.keep_bits;
    ia.sat_bits = a.sat_bits;
    ia.tile_vs = a.tile_vs;
    ia.tile_rest = a.tile_rest;
    ia.tile_off = reinterpret_cast<u64 *>(wsb + gsdp::ws_off_offset(n));
    ia.grp_vs = reinterpret_cast<u64 *>(wsb + gsdp::ws_grp_offset(n));
    ia.grp_rest = ia.grp_vs + gsdp::cull_groups(n);
    ia.tiles = a.tiles;
    ia.groups = gsdp::cull_groups(n);
    ia.n = n;
    ia.ids = ids;
    ia.cap = capacity;
    ia.sat_ids = model->max_defer > 0 ? reinterpret_cast<u32 *>(wsb + gsdp::ws_sat_offset(n, model->max_defer))
                                      : nullptr;
    ia.count = count_dev;
    ia.hdr = reinterpret_cast<gsdp::WsHeader *>(wsb);
    ia.direct = ia.tiles <= kDirectTiles;
    if (ia.groups > 0 && !ia.direct && !a.grp_vs) {
        hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)((ia.groups + 3) / 4)), dim3(256), 0, st, ia);
        int rc2 = launched("gs_cull (group sums)");
        if (rc2) return rc2;
    }
    const dim3 ig((unsigned)(ia.groups > 0 ? ia.groups : 1));
    if (ia.direct) hipLaunchKernelGGL(k_tile_ids<true>, ig, dim3(kIdsThreads), 0, st, ia);
    else hipLaunchKernelGGL(k_tile_ids<false>, ig, dim3(kIdsThreads), 0, st, ia);
    return launched("gs_cull");
}

}  // namespace

extern "C" {

int gs_gather(const gs_model *model, int64_t step, const uint32_t *ids, const uint32_t *count_dev,
              uint32_t capacity, float *out_geo, float *out_app, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!count_dev || (capacity > 0 && !ids)) return GS_EINVAL;
    if (!step_ok(model, step)) return GS_EINVAL;
    if (capacity == 0 || (!out_geo && !out_app)) return GS_OK;
    FastArgs f;
    if (out_geo && out_app && fill_fast(f, model)) {
        f.step = step_k(model, step);
        f.ids = ids;
        f.count = count_dev;
        f.cap = capacity;
        f.out_geo = out_geo;
        f.out_app = out_app;
        launch_fast<kGather, kFastGatherRows>(model->geo.state, row_grid(capacity, kRowBlocksGather),
                                              (hipStream_t)stream, f);
        return launched("gs_gather");
    }
    RowArgs a;
    fill_rows(a, model);
    a.step = step_k(model, step);
    a.ids = ids;
    a.count = count_dev;
    a.cap = capacity;
    a.out_geo = out_geo;
    a.out_app = out_app;
    launch_rows<kGather>(model, row_grid(capacity, kRowBlocksGather), (hipStream_t)stream, a);
    return launched("gs_gather");
}

int gs_scatter_grad(const uint32_t *ids, const uint32_t *count_dev, uint32_t capacity, int32_t dim,
                    const float *g_compact, float *g_dense, int32_t accumulate, void *stream)
{
    if (!count_dev || dim < 1 || (capacity > 0 && (!ids || !g_compact || !g_dense))) return GS_EINVAL;
    if (capacity == 0) return GS_OK;
    const int cu = cu_count();
    int64_t want = ((int64_t)capacity * dim + 255) / 256;
    int64_t cap = (int64_t)(cu > 0 ? cu : 256) * 8;
    int grid = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, (hipStream_t)stream, ids, count_dev, capacity, dim,
                       g_compact, g_dense, accumulate);
    return launched("gs_scatter_grad");
}

int gs_adam_step_deferred(const gs_model *model, int64_t step, const uint32_t *ids, const uint32_t *count_dev,
                          uint32_t capacity, const float *g_geo, const float *g_app, float *g_geo_dense,
                          float *g_app_dense, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!count_dev || (capacity > 0 && !ids)) return GS_EINVAL;
    if (!step_ok(model, step)) return GS_EINVAL;
    const bool compact = g_geo || g_app;
    if (compact && (!g_geo || !g_app)) return GS_EINVAL;
    if (!compact && capacity > 0 && (!g_geo_dense || !g_app_dense)) return GS_EINVAL;
    const bool geo_dense = model->geo_mode == 1;
    if (model->max_defer > 0 || (geo_dense && compact) || has_fp8(model)) {
        if (!ws || !aligned(ws, 256)) return GS_EINVAL;
        if ((int64_t)ws_bytes < gsdp::ws_bytes_for(model->n, model->max_defer, has_fp8(model))) return GS_ESPACE;
    }
    RowArgs a;
    fill_rows(a, model);
    a.step = step_k(model, step);
    const LutPtrs L = lut_ptrs(model);
    a.Mf = L.Mf;
    a.Vf = L.Vf;
    a.SS = L.SS;
    a.BC = L.BC;
    a.ids = ids;
    a.count = count_dev;
    a.cap = capacity;
    a.g_geo = g_geo;
    a.g_app = g_app;
    a.gd_geo = g_geo_dense;
    a.gd_app = g_app_dense;
    int64_t rows = capacity;
    if (model->max_defer > 0) {
        char *wsb = static_cast<char *>(ws);
        a.sat_count = &reinterpret_cast<gsdp::WsHeader *>(wsb)->sat_total;
        a.sat_ids = reinterpret_cast<const u32 *>(wsb + gsdp::ws_sat_offset(model->n, model->max_defer));
        rows += model->n;
    }
    if (geo_dense && model->n > 0) {
        DenseArgs da;
        memset(&da, 0, sizeof da);
        da.w = model->geo.w;
        da.m = {model->geo.m, model->geo.m_scale, model->geo.m_ld};
        da.v = {model->geo.v, model->geo.v_scale, model->geo.v_ld};
        da.n = model->n;
        da.rb = restore_bound(model->beta1, model->beta2);
        da.step = step_k(model, step);
        for (int c = 0; c < 10; ++c) da.lr[c] = model->geo.lr[c];
        da.eps = (float)model->eps;
        da.omb1 = (float)(1.0 - model->beta1);
        da.omb2 = (float)(1.0 - model->beta2);
        // b^(0+1) of the tables, i.e. the FP32 rounding of b (a d = 0 step)
        da.b1f = (float)model->beta1;
        da.b2f = (float)model->beta2;
        da.SS = L.SS;
        da.BC = L.BC;
        da.sr_seed = model->sr_seed;
        da.g_geo = g_geo;
        da.gd_geo = g_geo_dense;
        da.cap = capacity;
        da.tiles = gsdp::cull_tiles(model->n);
        if (compact) {
            char *wsb = static_cast<char *>(ws);
            da.tile_off = reinterpret_cast<const u64 *>(wsb + gsdp::ws_off_offset(model->n));
            da.keep_bits = reinterpret_cast<const u64 *>(wsb + gsdp::ws_keep_offset(model->n));
        }
        if (model->geo.state == GS_F32)
            hipLaunchKernelGGL(k_dense_geo<GS_F32>, dim3((unsigned)da.tiles), dim3(256), 0, (hipStream_t)stream, da);
        else
            hipLaunchKernelGGL(k_dense_geo<GS_BF16>, dim3((unsigned)da.tiles), dim3(256), 0, (hipStream_t)stream, da);
        int rc2 = launched("gs_adam_step_deferred (dense geometry)");
        if (rc2) return rc2;
    }
    if (has_fp8(model)) {
        // pass 1: per-block max of the new moments that outgrow their scale
        char *wsb = static_cast<char *>(ws);
        const int64_t nb = gsdp::fp8_blocks(model->n);
        u32 *mx = reinterpret_cast<u32 *>(wsb + gsdp::ws_fp8_offset(model->n, model->max_defer));
        for (int k = 0; k < 4; ++k) a.fp8max[k] = mx + k * nb;
        a.fp8list = mx + 4 * nb;
        a.fp8count = mx + 8 * nb;
        a.nb = nb;
        launch_rows<kAdamMax>(model, row_grid(rows, kRowBlocksUpdate), (hipStream_t)stream, a);
        int rc1 = launched("gs_adam_step_deferred (fp8 max pass)");
        if (rc1) return rc1;
        // pass 2: grow scales and re-encode those blocks
        RescaleArgs ra;
        memset(&ra, 0, sizeof ra);
        const gs_group *grp[2] = {&model->geo, &model->app};
        for (int k = 0; k < 4; ++k) {
            const gs_group &gg = *grp[k / 2];
            const bool isv = k & 1;
            ra.q[k] = static_cast<uint8_t *>(isv ? gg.v : gg.m);
            ra.s[k] = isv ? gg.v_scale : gg.m_scale;
            ra.ld[k] = isv ? gg.v_ld : gg.m_ld;
            ra.dim[k] = gg.dim;
            ra.col0[k] = k < 2 ? 0 : 10;
            ra.maxb[k] = a.fp8max[k];
            ra.fp8[k] = gg.state == GS_FP8E4M3;
        }
        ra.n = model->n;
        ra.nb = nb;
        ra.sr_seed = model->sr_seed;
        ra.step = step_k(model, step);
        ra.list = a.fp8list;
        ra.count = a.fp8count;
        const int cu = cu_count();
        hipLaunchKernelGGL(k_fp8_rescale, dim3((unsigned)((cu > 0 ? cu : 256) * 8)), dim3(256), 0,
                           (hipStream_t)stream, ra);
        rc1 = launched("gs_adam_step_deferred (fp8 rescale)");
        if (rc1) return rc1;
    }
    FastArgs f;
    if (compact && !geo_dense && fill_fast(f, model)) {
        f.step = a.step;
        f.ids = ids;
        f.count = count_dev;
        f.cap = capacity;
        f.sat_ids = a.sat_ids;
        f.sat_count = a.sat_count;
        f.g_geo = g_geo;
        f.g_app = g_app;
        f.Mf = a.Mf;
        f.Vf = a.Vf;
        f.SS = a.SS;
        f.BC = a.BC;
        f.adv = lut_adv(model);
        launch_fast<kAdam, kFastUpdateRows>(model->geo.state, row_grid(rows, kRowBlocksUpdate), (hipStream_t)stream,
                                            f);
    } else {
        a.adv = lut_adv(model);
        launch_rows<kAdam>(model, row_grid(rows, kRowBlocksUpdate), (hipStream_t)stream, a);
    }
    return launched("gs_adam_step_deferred");
}

int gs_adam_flush(const gs_model *model, int64_t step, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!step_ok(model, step)) return GS_EINVAL;
    if (model->n == 0) return GS_OK;
    RowArgs a;
    fill_rows(a, model);
    a.step = step_k(model, step);
    const LutPtrs L = lut_ptrs(model);
    a.Mf = L.Mf;
    a.Vf = L.Vf;
    launch_rows<kFlush>(model, row_grid(model->n, kRowBlocksUpdate), (hipStream_t)stream, a);
    return launched("gs_adam_flush");
}

// ------------------------------------------------------------ densification
namespace {

int64_t dens_ws_bytes(int64_t n)
{
    const int64_t tiles = gsdp::cull_tiles(n);
    return gsdp::kWsHeader + (n + 255) / 256 * 256 + 2 * 3 * 4 * tiles;
}

int dens_args(const gs_model *m, const gs_densify_params *p, void *ws, size_t ws_bytes, DensArgs &a)
{
    int rc = check_model(m);
    if (rc) return rc;
    if (!p || !ws || !aligned(ws, 256)) return GS_EINVAL;
    if (m->geo.state == GS_FP8E4M3 || m->app.state == GS_FP8E4M3) return GS_EUNSUPPORTED;
    if (!(p->scene_extent > 0.0f) || !(p->percent_dense > 0.0f) || !(p->min_opacity > 0.0f && p->min_opacity < 1.0f) ||
        !(p->max_screen_size >= 0.0f) || !(p->grad_threshold == p->grad_threshold))
        return GS_EINVAL;
    if ((int64_t)ws_bytes < dens_ws_bytes(m->n)) return GS_ESPACE;
    memset(&a, 0, sizeof a);
    a.gw = m->geo.w;
    a.aw = m->app.w;
    a.aw_ld = m->app.w_ld;
    a.adim = m->app.dim;
    a.big_on = p->prune_big != 0;
    a.thr = p->grad_threshold;
    // thresholds: FP64 logs rounded once
    a.log_dense = (float)std::log((double)p->percent_dense * (double)p->scene_extent);
    a.log_big = (float)std::log(0.1 * (double)p->scene_extent);
    a.logit_min = (float)std::log((double)p->min_opacity / (1.0 - (double)p->min_opacity));
    a.log_split = (float)std::log(1.6);
    a.max_screen = p->max_screen_size;
    a.seed = p->seed;
    a.n = m->n;
    a.tiles = gsdp::cull_tiles(m->n);
    char *wsb = static_cast<char *>(ws);
    a.totals = reinterpret_cast<u32 *>(wsb);
    a.code = reinterpret_cast<uint8_t *>(wsb + gsdp::kWsHeader);
    a.cnt = reinterpret_cast<u32 *>(wsb + gsdp::kWsHeader + (m->n + 255) / 256 * 256);
    a.off = a.cnt + 3 * a.tiles;
    return GS_OK;
}

}  // namespace

int gs_densify_workspace_bytes(const gs_model *model, size_t *bytes)
{
    if (!model || !bytes || model->n < 0) return GS_EINVAL;
    *bytes = (size_t)dens_ws_bytes(model->n);
    return GS_OK;
}

int gs_densify_plan(const gs_model *model, const float *grad_accum, const float *grad_denom,
                    const float *max_radii2d, const gs_densify_params *params, void *ws, size_t ws_bytes,
                    void *stream, int64_t *n_out, int64_t *counts)
{
    DensArgs a;
    int rc = dens_args(model, params, ws, ws_bytes, a);
    if (rc) return rc;
    if (!n_out || (model->n > 0 && (!grad_accum || !grad_denom))) return GS_EINVAL;
    if (params->max_screen_size > 0.0f && model->n > 0 && !max_radii2d) return GS_EINVAL;
    if (a.tiles > 0x7fffffff) return GS_EINVAL;
    a.accum = grad_accum;
    a.denom = grad_denom;
    a.radii = params->max_screen_size > 0.0f ? max_radii2d : nullptr;
    hipStream_t st = (hipStream_t)stream;
    if (a.tiles > 0) {
        hipLaunchKernelGGL(k_dens_plan, dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
        rc = launched("gs_densify_plan");
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_dens_scan, dim3(1), dim3(kScanThreads), 0, st, a);
    rc = launched("gs_densify_plan (scan)");
    if (rc) return rc;
    u32 tot[3] = {0, 0, 0};
    hipError_t e = hipMemcpyAsync(tot, a.totals, sizeof tot, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gs_densify_plan: totals");
    *n_out = (int64_t)tot[0] + tot[1] + tot[2];
    if (counts)
        for (int j = 0; j < 3; ++j) counts[j] = tot[j];
    return GS_OK;
}

int gs_densify_apply(const gs_model *src, const gs_densify_params *params, const gs_model *dst, int64_t step,
                     void *ws, size_t ws_bytes, void *stream)
{
    DensArgs a;
    int rc = dens_args(src, params, ws, ws_bytes, a);
    if (rc) return rc;
    rc = check_model(dst);
    if (rc) return rc;
    if (step < 0 || step > 0x7fffffff) return GS_EINVAL;
    if (dst->app.dim != src->app.dim || dst->geo.state != src->geo.state || dst->app.state != src->app.state)
        return GS_EINVAL;
    if (dst->n > 0 && !dst->last_step) return GS_EINVAL;
    a.sgm = {src->geo.m, src->geo.m_scale, src->geo.m_ld};
    a.sgv = {src->geo.v, src->geo.v_scale, src->geo.v_ld};
    a.sam = {src->app.m, src->app.m_scale, src->app.m_ld};
    a.sav = {src->app.v, src->app.v_scale, src->app.v_ld};
    a.dgw = dst->geo.w;
    a.daw = dst->app.w;
    a.daw_ld = dst->app.w_ld;
    a.dgm = {dst->geo.m, dst->geo.m_scale, dst->geo.m_ld};
    a.dgv = {dst->geo.v, dst->geo.v_scale, dst->geo.v_ld};
    a.dam = {dst->app.m, dst->app.m_scale, dst->app.m_ld};
    a.dav = {dst->app.v, dst->app.v_scale, dst->app.v_ld};
    a.dlast = dst->last_step;
    a.dn = dst->n;
    a.step = (int32_t)step;
    if (a.tiles == 0) return GS_OK;
    if (a.tiles > 0x7fffffff) return GS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const bool gb = src->geo.state == GS_BF16, ab = src->app.state == GS_BF16;
    if (!gb && !ab) hipLaunchKernelGGL((k_dens_apply<GS_F32, GS_F32>), dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
    else if (!gb && ab) hipLaunchKernelGGL((k_dens_apply<GS_F32, GS_BF16>), dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
    else if (gb && !ab) hipLaunchKernelGGL((k_dens_apply<GS_BF16, GS_F32>), dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
    else hipLaunchKernelGGL((k_dens_apply<GS_BF16, GS_BF16>), dim3((unsigned)a.tiles), dim3(kCullBlock), 0, st, a);
    rc = launched("gs_densify_apply");
    if (rc || !dst->cull_sum) return rc;
    return gs_cull_summary_build(dst, stream);
}

int gs_synth_grad(uint64_t seed, int64_t step, const uint32_t *ids, const uint32_t *count_dev, uint32_t capacity,
                  int32_t dim, int32_t col0, double sigma, float *out, void *stream)
{
    if (!count_dev || !out || dim < 1 || col0 < 0 || step < 0) return GS_EINVAL;
    if (capacity == 0) return GS_OK;
    const double var = 4.0 * (65536.0 * 65536.0 - 1.0) / 12.0;
    const double scale = sigma / sqrt(var) / 2.0;
    const int cu = cu_count();
    int64_t want = ((int64_t)capacity * dim + 255) / 256;
    int64_t cap = (int64_t)(cu > 0 ? cu : 256) * 8;
    int grid = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
    hipLaunchKernelGGL(k_synth, dim3(grid), dim3(256), 0, (hipStream_t)stream, (u64)seed, (u64)step, ids, count_dev,
                       capacity, dim, col0, scale, out);
    return launched("gs_synth_grad");
}

int gs_camera_pack_bytes(size_t *bytes)
{
    if (!bytes) return GS_EINVAL;
    *bytes = sizeof(CamPack);
    return GS_OK;
}

int gs_camera_pack(const gs_model *model, const gs_camera *cams, int32_t count, void *out_host)
{
    if (!model || !cams || !out_host || count < 0) return GS_EINVAL;
    CamPack *out = static_cast<CamPack *>(out_host);
    for (int i = 0; i < count; ++i) {
        if (!(cams[i].fx > 0.0f && cams[i].fy > 0.0f) || cams[i].width <= 0 || cams[i].height <= 0) return GS_EINVAL;
        memset(&out[i], 0, sizeof(CamPack));
        pack_camera(model, &cams[i], out[i].cam, out[i].band);
        pack_side(&cams[i], out[i].band, out[i].side);
    }
    return GS_OK;
}

int gs_multi_workspace_bytes(const gs_model *model, size_t *bytes)
{
    if (!model || !bytes || model->n < 0) return GS_EINVAL;
    *bytes = (size_t)multi_ws_bytes(model->n);
    return GS_OK;
}

int gs_cull_multi(const gs_model *model, const gs_multi *desc, int64_t step, void *ws, size_t ws_bytes, void *stream)
{
    MultiArgs a;
    int rc = multi_args(model, desc, step, ws, ws_bytes, a);
    if (rc) return rc;
    return launch_multi(desc->variant, a, model->n, (hipStream_t)stream);
}

int gs_cull_multi_autotune(const gs_model *model, gs_multi *desc, int64_t step, void *ws, size_t ws_bytes,
                           void *stream, float *times_ms, int32_t *n_variants)
{
    MultiArgs a;
    int rc = multi_args(model, desc, step, ws, ws_bytes, a);
    if (rc) return rc;
    if (n_variants) *n_variants = kMultiVariants;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return hip_fail(hipGetLastError(), "autotune events");
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < kMultiVariants; ++v) {
        rc = launch_multi(v, a, model->n, st);  // warm-up
        if (rc) break;
        hipError_t he = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && !rc; ++r) rc = launch_multi(v, a, model->n, st);
        if (rc) break;
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = hip_fail(he, "autotune");
            break;
        }
        ms /= 3.0f;
        if (times_ms) times_ms[v] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    desc->variant = best;
    return GS_OK;
}

int gs_grad_sum_multi(const gs_multi *desc, int32_t adim, const float *g_cam, float *out_geo, float *out_app,
                      void *stream)
{
    if (!desc || !g_cam || !out_geo || !out_app || adim < 1 || adim > 54) return GS_EINVAL;
    if (desc->cams_per_scene < 1 || desc->cams_per_scene > kMaxCams) return GS_EINVAL;
    if (!desc->cam_pos || !desc->cam_count || !desc->union_count) return GS_EINVAL;
    GradSumArgs a;
    a.cam_pos = desc->cam_pos;
    a.cam_count = desc->cam_count;
    a.union_count = desc->union_count;
    a.chunk_start = desc->chunk_start;
    a.cap_cam = desc->cap_cam;
    a.cap_union = desc->cap_union;
    a.C = desc->cams_per_scene;
    a.adim = adim;
    a.g_cam = g_cam;
    a.out_geo = out_geo;
    a.out_app = out_app;
    const int cu = cu_count();
    int64_t want = ((int64_t)desc->cap_union + kSumRows - 1) / kSumRows;
    int64_t cap = (int64_t)(cu > 0 ? cu : 256) * 8;
    int grid = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
    hipLaunchKernelGGL(k_grad_sum, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
    return launched("gs_grad_sum_multi");
}

int gs_plan_image_split(const gs_model *model, const gs_camera *cam, int64_t step, double mem_limit, gs_multi *desc,
                        void *ws, size_t ws_bytes, void *stream, int32_t *split_x, uint32_t *counts)
{
    if (!model || !cam || !desc || !split_x || !(mem_limit > 0.0)) return GS_EINVAL;
    if (desc->n_scenes != 1 || desc->cams_per_scene != 2 || desc->n_sets != 1 || !desc->cams) return GS_EINVAL;
    if (step == 0) return GS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t cap_u = desc->cap_union, cap_c = desc->cap_cam;
    desc->cap_union = 0;  // counts only
    desc->cap_cam = 0;
    CamPack rec[2];
    int rc = GS_OK;
    auto count_split = [&](int x, uint32_t out[3]) -> int {
        gs_camera h[2] = {*cam, *cam};
        h[0].width = x;                       // left crop [0, x)
        h[1].width = cam->width - x;          // right crop [x, W): principal point shifts
        h[1].cx = cam->cx - (float)x;
        memset(rec, 0, sizeof rec);
        for (int i = 0; i < 2; ++i) pack_camera(model, &h[i], rec[i].cam, rec[i].band);
        hipError_t e = hipMemcpyAsync(const_cast<void *>(desc->cams), rec, sizeof rec, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "gs_plan_image_split: camera upload");
        int r = gs_cull_multi(model, desc, step, ws, ws_bytes, stream);
        if (r) return r;
        uint32_t cc[2], uc = 0;
        e = hipMemcpyAsync(cc, desc->cam_count, sizeof cc, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&uc, desc->union_count, sizeof uc, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "gs_plan_image_split: count readback");
        out[0] = uc;
        out[1] = cc[0];
        out[2] = cc[1];
        return GS_OK;
    };
    // active count of the whole image: both halves empty except the full frame
    uint32_t full[3];
    {
        gs_camera h[2] = {*cam, *cam};
        memset(rec, 0, sizeof rec);
        for (int i = 0; i < 2; ++i) pack_camera(model, &h[i], rec[i].cam, rec[i].band);
        hipError_t e = hipMemcpyAsync(const_cast<void *>(desc->cams), rec, sizeof rec, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) rc = hip_fail(e, "gs_plan_image_split: camera upload");
        if (!rc) rc = gs_cull_multi(model, desc, step, ws, ws_bytes, stream);
        if (!rc) {
            e = hipMemcpyAsync(&full[0], desc->union_count, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = hip_fail(e, "gs_plan_image_split: count readback");
        }
    }
    if (!rc) {
        if (counts) counts[0] = full[0];
        if ((double)full[0] <= mem_limit * (double)model->n || cam->width < 2) {
            *split_x = 0;  // no split needed
        } else {
            // start at the midpoint and move the split toward the less populated
            // side, halving the step, five times (Sec. 4.4)
            int lo = 1, hi = cam->width - 1, x = cam->width / 2;
            uint32_t c3[3] = {0, 0, 0};
            for (int it = 0; it < 5 && !rc; ++it) {
                rc = count_split(x, c3);
                if (rc) break;
                if (c3[1] > c3[2]) hi = x;
                else lo = x;
                x = (lo + hi) / 2;
            }
            if (!rc) rc = count_split(x, c3);
            if (!rc) {
                *split_x = x;
                if (counts) {
                    counts[1] = c3[1];
                    counts[2] = c3[2];
                }
            }
        }
    }
    desc->cap_union = cap_u;
    desc->cap_cam = cap_c;
    return rc;
}

int gs_stream_read_probe(const void *buf, size_t bytes, float *sink, void *stream)
{
    if (!buf || !sink || (bytes % 16) != 0 || !aligned(buf, 16)) return GS_EINVAL;
    if (bytes == 0) return GS_OK;
    const int64_t n4 = (int64_t)(bytes / 16), per = (int64_t)kProbeP * 256;
    const int64_t grid = (n4 + per - 1) / per;
    if (grid > 0x7fffffff) return GS_EINVAL;
    hipLaunchKernelGGL(k_stream_read, dim3((u32)grid), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const float4 *>(buf), n4, sink);
    return launched("gs_stream_read_probe");
}

int gs_row_probe(const uint32_t *ids, uint32_t count, void *base, uint64_t n_rows, uint32_t row_bytes, int32_t write,
                 float *sink, void *stream)
{
    if (!ids || !base || !sink || row_bytes == 0 || row_bytes > 1024 || (row_bytes % 16) != 0 || !aligned(base, 16))
        return GS_EINVAL;
    if (count == 0 || n_rows == 0) return GS_OK;
    const int cu = cu_count();
    const u32 grid = (u32)std::min<int64_t>(((int64_t)count + 15) / 16, (int64_t)(cu > 0 ? cu : 256) * 8);
    if (write)
        hipLaunchKernelGGL(k_row_probe<true>, dim3(grid), dim3(256), 0, (hipStream_t)stream, ids, count, (u64)n_rows,
                           static_cast<float4 *>(base), row_bytes / 16, sink);
    else
        hipLaunchKernelGGL(k_row_probe<false>, dim3(grid), dim3(256), 0, (hipStream_t)stream, ids, count,
                           (u64)n_rows, static_cast<float4 *>(base), row_bytes / 16, sink);
    return launched("gs_row_probe");
}

int gs_step_advance(int32_t *step_dev, void *stream)
{
    if (!step_dev) return GS_EINVAL;
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, (hipStream_t)stream, step_dev);
    return launched("gs_step_advance");
}

}  // extern "C"
