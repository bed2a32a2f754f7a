// libgsdp: HIP kernels and C ABI of the Gaussian-parameter hot path of
// GS-Scale-style 3DGS training (arXiv 2509.15645) for MI355X (gfx950).
//
// Build flags matter for exactness: -ffp-contract=off (no FMA contraction),
// correctly rounded FP32 division and square root, denormals preserved, and
// packed-FP32 instructions disabled.  Every floating-point expression below is
// written as the exact sequence of IEEE operations that defines the result.
//
// Kernels
//   k_cull      persistent; each block claims 1024-row tiles with a ticket,
//               stages the tile's geometry through LDS with 128-bit loads,
//               restores deferred rows, culls, and compacts the kept rows in
//               id order: wave ballot + mbcnt, block scan in LDS, decoupled
//               look-back across tiles (single pass, deterministic).
//   k_rows      one wavefront per Gaussian row, lanes 0..9 = G columns,
//               lanes 10..10+dim = A columns; three modes:
//                 gather  restore current values into compact buffers
//                 adam    restore + Adam with fused gradient scatter
//                 flush   catch up every deferred row
//   k_scatter   compact -> dense gradient rows
//   k_synth     synthetic gradients (harness only)
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gsdp.h"
#include "gsdp_internal.h"

using u32 = uint32_t;
using u64 = unsigned long long;
using gsdp::kCullBlock;
using gsdp::kCullIpt;
using gsdp::kCullTile;

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
// (Sec. 2.3 step 1).  All comparisons are positive, so a NaN anywhere culls.
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
// w - ((W[d] lr) m) / (sqrt(v) + eps), with the stored (old) moments.
__device__ __forceinline__ float restore1(float w, float m, float v, float wd, float lr, float eps)
{
    const float wsc = wd * lr;
    const float num = wsc * m;
    const float den = sqrtf(v) + eps;
    return w - num / den;
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

// ---------------------------------------------------------------------------
// cull + ordered compaction
// ---------------------------------------------------------------------------
constexpr u64 kFlagAgg = 1ull << 62;
constexpr u64 kFlagInc = 2ull << 62;
constexpr u64 kValMask = (1ull << 62) - 1;
constexpr u32 kSpinLimit = 1u << 24;

__device__ __forceinline__ u64 pack_vs(u32 vis, u32 sat) { return ((u64)vis << 31) | (u64)sat; }

struct CullArgs {
    const float *gw;                 // [n][10]
    const float *gm, *gv;            // G moments (restore)
    int64_t m_ld, v_ld;
    const int32_t *last;
    int64_t n;
    int32_t t, K, dmax, pad0;
    const float *Wrow;               // LUT row of step t
    float lr[10];
    float eps;
    CamK cam;
    u32 *ids, *count;
    u32 cap, pad1;
    u32 *sat_ids;
    gsdp::WsHeader *hdr;
    u64 *st;                         // tile states [2][tiles]
    int64_t tiles;
};

__global__ __launch_bounds__(kCullBlock) void k_cull(CullArgs a)
{
    __shared__ float4 sG4[kCullTile * 10 / 4];
    __shared__ u32 sCntV[kCullIpt * 4], sCntS[kCullIpt * 4];
    __shared__ u32 sOffV[kCullIpt * 4], sOffS[kCullIpt * 4];
    __shared__ u32 sTile, sParity, sRestored;
    __shared__ u64 sAgg, sExcl;
    float *sG = reinterpret_cast<float *>(sG4);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        sParity = __hip_atomic_load(&a.hdr->parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sRestored = 0;
    }
    __syncthreads();
    const u32 parity = sParity & 1u;
    u64 *st = a.st + (size_t)parity * a.tiles;
    u64 *st_other = a.st + (size_t)(parity ^ 1u) * a.tiles;

    for (;;) {
        if (tid == 0) sTile = atomicAdd(&a.hdr->ticket, 1u);
        __syncthreads();
        const u32 tile = sTile;
        if ((int64_t)tile >= a.tiles) break;
        const int64_t row0 = (int64_t)tile * kCullTile;
        const int rows = (int)min((int64_t)kCullTile, a.n - row0);

        // stage the tile's geometry (rows x 40 B, contiguous) through LDS
        const int nf = rows * 10, nf4 = nf >> 2;
        const float *src = a.gw + row0 * 10;
        const float4 *src4 = reinterpret_cast<const float4 *>(src);
        for (int j = tid; j < nf4; j += kCullBlock) sG4[j] = src4[j];
        for (int j = nf4 * 4 + tid; j < nf; j += kCullBlock) sG[j] = src[j];
        int lastv[kCullIpt];
#pragma unroll
        for (int k = 0; k < kCullIpt; ++k) {
            const int r = k * kCullBlock + tid;
            lastv[k] = r < rows ? a.last[row0 + r] : 0;
        }
        __syncthreads();

        u64 bv[kCullIpt], bs[kCullIpt];
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
                int d = a.t - 1 - lastv[k];
                d = d < 0 ? 0 : (d > a.dmax ? a.dmax : d);
                if (d > 0) {
                    const int64_t row = row0 + r;
                    const float *mr = a.gm + row * a.m_ld;
                    const float *vr = a.gv + row * a.v_ld;
                    const float wd = a.Wrow[d];
#pragma unroll
                    for (int j = 0; j < 10; ++j) g[j] = restore1(g[j], mr[j], vr[j], wd, a.lr[j], a.eps);
                    ++nrest;
                }
                keep = cull_v1(g, a.cam);
                sat = (a.K > 0) && !keep && d == a.K;
            }
            bv[k] = __ballot(keep);
            bs[k] = __ballot(sat);
            if (lane == 0) {
                sCntV[k * 4 + wave] = (u32)__popcll(bv[k]);
                sCntS[k * 4 + wave] = (u32)__popcll(bs[k]);
            }
        }
        if (nrest) atomicAdd(&sRestored, nrest);
        __syncthreads();

        if (tid == 0) {
            u32 sv = 0, ss = 0;
            for (int e = 0; e < kCullIpt * 4; ++e) {
                sOffV[e] = sv;
                sv += sCntV[e];
                sOffS[e] = ss;
                ss += sCntS[e];
            }
            sAgg = pack_vs(sv, ss);
        }
        __syncthreads();

        // decoupled look-back by wave 0
        if (wave == 0) {
            const u64 agg = sAgg;
            u64 excl = 0;
            if (tile == 0) {
                if (lane == 0) __hip_atomic_store(&st[0], kFlagInc | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                if (lane == 0)
                    __hip_atomic_store(&st[tile], kFlagAgg | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                int64_t base = (int64_t)tile - 1;
                for (;;) {
                    const int64_t idx = base - lane;
                    u64 s = kFlagInc;
                    if (idx >= 0) {
                        u32 spins = 0;
                        s = __hip_atomic_load(&st[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        while ((s >> 62) == 0 && spins < kSpinLimit) {
                            __builtin_amdgcn_s_sleep(1);
                            s = __hip_atomic_load(&st[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                            ++spins;
                        }
                        if ((s >> 62) == 0) {
                            atomicOr(&a.hdr->error, 1u);
                            s = kFlagInc;
                        }
                    }
                    const u64 incm = __ballot((s >> 62) == 2);
                    const u64 val = s & kValMask;
                    if (incm) {
                        const int stop = __builtin_ctzll(incm);
                        excl += wave_sum_u64(lane <= stop ? val : 0ull);
                        break;
                    }
                    excl += wave_sum_u64(val);
                    base -= 64;
                }
                if (lane == 0)
                    __hip_atomic_store(&st[tile], kFlagInc | (excl + agg), __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            if (lane == 0) {
                sExcl = excl;
                if ((int64_t)tile == a.tiles - 1) {
                    const u64 inc = excl + agg;
                    *a.count = (u32)(inc >> 31);
                    a.hdr->sat_total = (u32)(inc & 0x7fffffffu);
                    a.hdr->vis_accum += inc >> 31;
                }
                st_other[tile] = 0;  // the next call uses the other buffer
            }
        }
        __syncthreads();

        const u64 ex = sExcl;
        const u32 pv = (u32)(ex >> 31), ps = (u32)(ex & 0x7fffffffu);
#pragma unroll
        for (int k = 0; k < kCullIpt; ++k) {
            const u32 row = (u32)(row0 + k * kCullBlock + tid);
            if ((bv[k] >> lane) & 1ull) {
                const u32 pos = pv + sOffV[k * 4 + wave] + lane_rank(bv[k]);
                if (pos < a.cap) a.ids[pos] = row;
            }
            if ((bs[k] >> lane) & 1ull) a.sat_ids[ps + sOffS[k * 4 + wave] + lane_rank(bs[k])] = row;
        }
    }

    __syncthreads();
    if (tid == 0) {
        if (sRestored) atomicAdd(&a.hdr->restored, sRestored);
        __threadfence();
        const u32 prev = atomicAdd(&a.hdr->done, 1u);
        if (prev == gridDim.x - 1) {
            __threadfence();
            if (a.tiles == 0) {
                *a.count = 0;
                a.hdr->sat_total = 0;
            }
            const u32 rest = __hip_atomic_load(&a.hdr->restored, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a.hdr->restored_last = rest;
            a.hdr->restored_accum += rest;
            a.hdr->restored = 0;
            a.hdr->ticket = 0;
            a.hdr->done = 0;
            a.hdr->parity = parity ^ 1u;
        }
    }
}

// ---------------------------------------------------------------------------
// row kernels: gather / adam / flush
// ---------------------------------------------------------------------------
enum RowMode { kGather = 0, kAdam = 1, kFlush = 2 };
constexpr int kRowUnroll = 4;

struct RowArgs {
    float *gw, *gm, *gv;
    int64_t gw_ld, gm_ld, gv_ld;
    float *aw, *am, *av;
    int64_t aw_ld, am_ld, av_ld;
    int32_t adim, t, K, dmax;
    float lr[64];                    // lane-indexed: 0..9 G, 10.. A
    float eps, omb1, omb2, pad0;
    int32_t *last;
    int64_t n;
    const float *Wrow, *Mf, *Vf, *SS, *BC;
    const u32 *ids, *count;
    u32 cap, pad1;
    const u32 *sat_ids, *sat_count;
    const float *g_geo, *g_app;      // compact gradients
    float *gd_geo, *gd_app;          // dense gradients (read and cleared)
    float *out_geo, *out_app;        // gather outputs
};

template <int MODE>
__global__ __launch_bounds__(256) void k_rows(RowArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * 4;
    const bool isG = lane < 10;
    const bool act = lane < 10 + a.adim;
    const int ca = lane - 10;
    const float lr = a.lr[lane];

    int64_t nvis, total;
    if (MODE == kFlush) {
        nvis = a.n;
        total = a.n;
    } else {
        const u32 c = *a.count;
        nvis = c < a.cap ? c : a.cap;
        total = nvis + ((MODE == kAdam && a.sat_count) ? (int64_t)*a.sat_count : 0);
    }
    float ss = 0.0f, bc = 1.0f;
    if (MODE == kAdam) {
        ss = a.SS[a.t];
        bc = a.BC[a.t];
    }
    const float step = lr * ss;

    for (int64_t base = wid * kRowUnroll; base < total; base += nw * kRowUnroll) {
        int64_t id[kRowUnroll];
        int d[kRowUnroll];
        bool ok[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t i = base + u;
            int64_t r = -1;
            if (i < total) {
                if (MODE == kFlush) r = i;
                else r = i < nvis ? (int64_t)a.ids[i] : (int64_t)a.sat_ids[i - nvis];
            }
            ok[u] = r >= 0 && r < a.n;
            id[u] = ok[u] ? r : 0;
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            int dd = 0;
            if (ok[u]) {
                const int last = a.last[id[u]];
                dd = (MODE == kFlush) ? a.t - last : a.t - 1 - last;
                dd = dd < 0 ? 0 : (dd > a.dmax ? a.dmax : dd);
            }
            d[u] = dd;
        }
        float w[kRowUnroll], m[kRowUnroll], v[kRowUnroll], g[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            w[u] = m[u] = v[u] = g[u] = 0.0f;
            const bool need = ok[u] && act && (MODE == kAdam || d[u] > 0 || MODE == kGather);
            if (!need) continue;
            const int64_t r = id[u];
            float *wp = isG ? a.gw + r * a.gw_ld + lane : a.aw + r * a.aw_ld + ca;
            w[u] = *wp;
            if (MODE == kAdam || d[u] > 0) {
                m[u] = isG ? a.gm[r * a.gm_ld + lane] : a.am[r * a.am_ld + ca];
                v[u] = isG ? a.gv[r * a.gv_ld + lane] : a.av[r * a.av_ld + ca];
            }
            if (MODE == kAdam && base + u < nvis) {
                if (a.g_geo) g[u] = isG ? a.g_geo[(base + u) * 10 + lane] : a.g_app[(base + u) * a.adim + ca];
                else g[u] = isG ? a.gd_geo[r * 10 + lane] : a.gd_app[r * a.adim + ca];
            }
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            if (!ok[u]) continue;
            const int64_t r = id[u];
            if (MODE == kGather) {
                float x = w[u];
                if (d[u] > 0) x = restore1(x, m[u], v[u], a.Wrow[d[u]], lr, a.eps);
                if (act) {
                    if (isG) {
                        if (a.out_geo) a.out_geo[(base + u) * 10 + lane] = x;
                    } else if (a.out_app) {
                        a.out_app[(base + u) * a.adim + ca] = x;
                    }
                }
            } else if (MODE == kAdam) {
                if (act) {
                    float x = w[u];
                    const int dd = d[u];
                    if (dd > 0) x = restore1(x, m[u], v[u], a.Wrow[dd], lr, a.eps);
                    const float m1 = a.Mf[dd] * m[u] + a.omb1 * g[u];
                    const float v1 = a.Vf[dd] * v[u] + (a.omb2 * g[u]) * g[u];
                    const float den = sqrtf(v1) / bc + a.eps;
                    x = x - (step * m1) / den;
                    if (isG) {
                        a.gw[r * a.gw_ld + lane] = x;
                        a.gm[r * a.gm_ld + lane] = m1;
                        a.gv[r * a.gv_ld + lane] = v1;
                    } else {
                        a.aw[r * a.aw_ld + ca] = x;
                        a.am[r * a.am_ld + ca] = m1;
                        a.av[r * a.av_ld + ca] = v1;
                    }
                    if (!a.g_geo && base + u < nvis) {
                        if (isG) a.gd_geo[r * 10 + lane] = 0.0f;
                        else a.gd_app[r * a.adim + ca] = 0.0f;
                    }
                }
                if (lane == 0) a.last[r] = a.t;
            } else {  // flush
                const int dl = d[u];
                if (dl > 0) {
                    if (act) {
                        const float x = restore1(w[u], m[u], v[u], a.Wrow[dl], lr, a.eps);
                        const float m1 = a.Mf[dl - 1] * m[u];
                        const float v1 = a.Vf[dl - 1] * v[u];
                        if (isG) {
                            a.gw[r * a.gw_ld + lane] = x;
                            a.gm[r * a.gm_ld + lane] = m1;
                            a.gv[r * a.gv_ld + lane] = v1;
                        } else {
                            a.aw[r * a.aw_ld + ca] = x;
                            a.am[r * a.am_ld + ca] = m1;
                            a.av[r * a.av_ld + ca] = v1;
                        }
                    }
                    if (lane == 0) a.last[r] = a.t;
                }
            }
        }
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

__device__ __forceinline__ u64 mix64(u64 z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ u64 sm_at(u64 s, u64 i) { return mix64(s + (i + 1ull) * 0x9E3779B97F4A7C15ull); }

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

int check_group(const gs_group &g, int64_t n, bool geo)
{
    if (geo && g.dim != 10) return GS_EINVAL;
    if (!geo && (g.dim < 1 || g.dim > 54)) return GS_EINVAL;
    if (g.w_ld < g.dim || g.m_ld < g.dim || g.v_ld < g.dim) return GS_EINVAL;
    if (g.state != GS_F32) return GS_EUNSUPPORTED;
    if (n > 0 && (!g.w || !g.m || !g.v)) return GS_EINVAL;
    if (!aligned(g.w, 4) || !aligned(g.m, 4) || !aligned(g.v, 4)) return GS_EINVAL;
    return GS_OK;
}

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
    return GS_OK;
}

struct LutPtrs {
    const float *W, *Mf, *Vf, *SS, *BC;
};

LutPtrs lut_ptrs(const gs_model *m, int64_t t)
{
    const gsdp::LutLayout L = gsdp::lut_layout(m->lut_max_steps, m->max_defer);
    const float *base = static_cast<const float *>(m->lut);
    return {base + gsdp::lut_w_row(t, m->max_defer), base + L.offM, base + L.offV, base + L.offSS, base + L.offBC};
}

int dmax_for(const gs_model *m, int64_t t_row)
{
    int64_t dm = t_row - 1;
    if (m->max_defer > 0 && dm > m->max_defer) dm = m->max_defer;
    return (int)dm;
}

void fill_rows(RowArgs &a, const gs_model *m)
{
    memset(&a, 0, sizeof a);
    a.gw = m->geo.w;
    a.gm = static_cast<float *>(m->geo.m);
    a.gv = static_cast<float *>(m->geo.v);
    a.gw_ld = m->geo.w_ld;
    a.gm_ld = m->geo.m_ld;
    a.gv_ld = m->geo.v_ld;
    a.aw = m->app.w;
    a.am = static_cast<float *>(m->app.m);
    a.av = static_cast<float *>(m->app.v);
    a.aw_ld = m->app.w_ld;
    a.am_ld = m->app.m_ld;
    a.av_ld = m->app.v_ld;
    a.adim = m->app.dim;
    a.K = m->max_defer;
    for (int c = 0; c < 10; ++c) a.lr[c] = m->geo.lr[c];
    for (int c = 0; c < m->app.dim; ++c) a.lr[10 + c] = m->app.lr[c];
    a.eps = (float)m->eps;
    a.omb1 = (float)(1.0 - m->beta1);
    a.omb2 = (float)(1.0 - m->beta2);
    a.last = m->last_step;
    a.n = m->n;
}

int row_grid(int64_t rows)
{
    const int cu = cu_count();
    int64_t want = (rows + 4 * kRowUnroll - 1) / (4 * kRowUnroll);
    int64_t cap = (int64_t)(cu > 0 ? cu : 256) * 8;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)want;
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
    *bytes = (size_t)gsdp::lut_layout(max_steps, max_defer).total * sizeof(float);
    return GS_OK;
}

int gs_lut_build_host(double beta1, double beta2, int32_t max_steps, int32_t max_defer, void *lut_host,
                      size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes(max_steps, max_defer, &need);
    if (rc) return rc;
    if (!lut_host) return GS_EINVAL;
    if (!(beta1 > 0.0 && beta1 < 1.0 && beta2 > 0.0 && beta2 < 1.0)) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    return gsdp::build_lut_host(beta1, beta2, max_steps, max_defer, static_cast<float *>(lut_host),
                                (int64_t)(bytes / sizeof(float))) == 0
               ? GS_OK
               : GS_ESPACE;
}

int gs_lut_build(double beta1, double beta2, int32_t max_steps, int32_t max_defer, void *lut_dev, size_t bytes)
{
    size_t need = 0;
    int rc = gs_lut_bytes(max_steps, max_defer, &need);
    if (rc) return rc;
    if (!lut_dev) return GS_EINVAL;
    if (bytes < need) return GS_ESPACE;
    std::vector<float> host(need / sizeof(float));
    rc = gs_lut_build_host(beta1, beta2, max_steps, max_defer, host.data(), need);
    if (rc) return rc;
    hipError_t e = hipMemcpy(lut_dev, host.data(), need, hipMemcpyHostToDevice);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_lut_build: hipMemcpy");
}

int gs_workspace_bytes(const gs_model *model, size_t *bytes)
{
    if (!model || !bytes || model->n < 0 || model->max_defer < 0) return GS_EINVAL;
    *bytes = (size_t)gsdp::ws_bytes_for(model->n, model->max_defer);
    return GS_OK;
}

int gs_cull(const gs_model *model, const gs_camera *cam, int64_t step, uint32_t *ids, uint32_t *count_dev,
            uint32_t capacity, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!cam || !count_dev || !ws || (capacity > 0 && !ids)) return GS_EINVAL;
    if (step < 1 || step > model->lut_max_steps) return GS_EINVAL;
    if (!(cam->fx > 0.0f && cam->fy > 0.0f) || cam->width <= 0 || cam->height <= 0) return GS_EINVAL;
    if (!aligned(ws, 256)) return GS_EINVAL;
    if ((int64_t)ws_bytes < gsdp::ws_bytes_for(model->n, model->max_defer)) return GS_ESPACE;

    CullArgs a;
    memset(&a, 0, sizeof a);
    a.gw = model->geo.w;
    a.gm = static_cast<const float *>(model->geo.m);
    a.gv = static_cast<const float *>(model->geo.v);
    a.m_ld = model->geo.m_ld;
    a.v_ld = model->geo.v_ld;
    a.last = model->last_step;
    a.n = model->n;
    a.t = (int32_t)step;
    a.K = model->max_defer;
    a.dmax = dmax_for(model, step);
    a.Wrow = lut_ptrs(model, step).W;
    for (int c = 0; c < 10; ++c) a.lr[c] = model->geo.lr[c];
    a.eps = (float)model->eps;
    for (int i = 0; i < 9; ++i) a.cam.R[i] = cam->R[i];
    for (int i = 0; i < 3; ++i) a.cam.T[i] = cam->t[i];
    a.cam.fx = cam->fx;
    a.cam.fy = cam->fy;
    a.cam.cx = cam->cx;
    a.cam.cy = cam->cy;
    a.cam.W = (float)cam->width;
    a.cam.H = (float)cam->height;
    a.cam.zn = cam->near_plane;
    a.cam.zf = cam->far_plane;
    a.ids = ids;
    a.count = count_dev;
    a.cap = capacity;
    char *wsb = static_cast<char *>(ws);
    a.hdr = reinterpret_cast<gsdp::WsHeader *>(wsb);
    a.tiles = gsdp::cull_tiles(model->n);
    a.st = reinterpret_cast<u64 *>(wsb + gsdp::kWsHeader);
    a.sat_ids = model->max_defer > 0 ? reinterpret_cast<u32 *>(wsb + gsdp::kWsHeader + 16 * a.tiles) : nullptr;

    // persistent grid: as many blocks as can be resident at once
    static std::atomic<int> s_cull_occ{0};
    int occ = s_cull_occ.load(std::memory_order_relaxed);
    if (occ == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_cull, kCullBlock, 0) != hipSuccess || occ < 1)
            occ = 1;
        s_cull_occ.store(occ, std::memory_order_relaxed);
    }
    const int cu = cu_count();
    int64_t grid = (int64_t)(cu > 0 ? cu : 256) * occ;
    if (grid > a.tiles) grid = a.tiles;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_cull, dim3((unsigned)grid), dim3(kCullBlock), 0, (hipStream_t)stream, a);
    return launched("gs_cull");
}

int gs_gather(const gs_model *model, int64_t step, const uint32_t *ids, const uint32_t *count_dev,
              uint32_t capacity, float *out_geo, float *out_app, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (!count_dev || (capacity > 0 && !ids)) return GS_EINVAL;
    if (step < 1 || step > model->lut_max_steps) return GS_EINVAL;
    if (capacity == 0 || (!out_geo && !out_app)) return GS_OK;
    RowArgs a;
    fill_rows(a, model);
    a.t = (int32_t)step;
    a.dmax = dmax_for(model, step);
    a.Wrow = lut_ptrs(model, step).W;
    a.ids = ids;
    a.count = count_dev;
    a.cap = capacity;
    a.out_geo = out_geo;
    a.out_app = out_app;
    hipLaunchKernelGGL(k_rows<kGather>, dim3(row_grid(capacity)), dim3(256), 0, (hipStream_t)stream, a);
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
    if (step < 1 || step > model->lut_max_steps) return GS_EINVAL;
    const bool compact = g_geo || g_app;
    if (compact && (!g_geo || !g_app)) return GS_EINVAL;
    if (!compact && capacity > 0 && (!g_geo_dense || !g_app_dense)) return GS_EINVAL;
    if (model->max_defer > 0) {
        if (!ws || !aligned(ws, 256)) return GS_EINVAL;
        if ((int64_t)ws_bytes < gsdp::ws_bytes_for(model->n, model->max_defer)) return GS_ESPACE;
    }
    RowArgs a;
    fill_rows(a, model);
    a.t = (int32_t)step;
    a.dmax = dmax_for(model, step);
    const LutPtrs L = lut_ptrs(model, step);
    a.Wrow = L.W;
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
        a.sat_ids = reinterpret_cast<const u32 *>(wsb + gsdp::kWsHeader + 16 * gsdp::cull_tiles(model->n));
        rows += model->n;
    }
    hipLaunchKernelGGL(k_rows<kAdam>, dim3(row_grid(rows)), dim3(256), 0, (hipStream_t)stream, a);
    return launched("gs_adam_step_deferred");
}

int gs_adam_flush(const gs_model *model, int64_t step, void *stream)
{
    int rc = check_model(model);
    if (rc) return rc;
    if (step < 1 || step > model->lut_max_steps) return GS_EINVAL;
    if (model->n == 0) return GS_OK;
    RowArgs a;
    fill_rows(a, model);
    a.t = (int32_t)step;
    a.dmax = dmax_for(model, step + 1);
    const LutPtrs L = lut_ptrs(model, step + 1);
    a.Wrow = L.W;
    a.Mf = L.Mf;
    a.Vf = L.Vf;
    hipLaunchKernelGGL(k_rows<kFlush>, dim3(row_grid(model->n)), dim3(256), 0, (hipStream_t)stream, a);
    return launched("gs_adam_flush");
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

}  // extern "C"
