// Internal definitions shared by the host and device parts of libgsdp.
#pragma once
#include <stdint.h>

namespace gsdp {

// Device tables for the deferred update (all FP32, offsets in floats):
//   W  : rows t = 1..T+1; row t holds w_scale for d = 0..min(t-1, K) (K = 0: unbounded)
//   Mf : b1^(d+1),  Vf : b2^(d+1)   for d = 0..Dm
//   SS : 1/(1-b1^t),  BC : sqrt(1-b2^t)   indexed by t = 0..T+1
struct LutLayout {
    int64_t T, K;
    int64_t nW, nMV;
    int64_t offM, offV, offSS, offBC, total;
};

inline LutLayout lut_layout(int64_t T, int64_t K)
{
    LutLayout L;
    L.T = T;
    L.K = K;
    const int64_t rows = T + 1;
    L.nW = K > 0 ? rows * (K + 1) : rows * (rows + 1) / 2;
    L.nMV = (K > 0 ? K : T) + 1;
    L.offM = L.nW;
    L.offV = L.offM + L.nMV;
    L.offSS = L.offV + L.nMV;
    L.offBC = L.offSS + (T + 2);
    L.total = L.offBC + (T + 2);
    return L;
}

// AdamW tables follow the Adam tables (whose Mf, Vf, SS, BC they share): for
// every decay class c (a distinct column rate) the decayed restore rows Wl and
// the decay products P (both in the W row layout) and the step decays q[t].
constexpr int kMaxDecayClasses = 8;
inline int64_t adamw_class_floats(int64_t T, int64_t K) { return 2 * lut_layout(T, K).nW + (T + 2); }
inline int64_t adamw_total_floats(int64_t T, int64_t K, int nclass)
{
    return lut_layout(T, K).total + nclass * adamw_class_floats(T, K);
}

// Offset of W row t (t >= 1).
inline int64_t lut_w_row(int64_t t, int64_t K) { return K > 0 ? (t - 1) * (K + 1) : t * (t - 1) / 2; }

// Cull tiles: 256 threads x 2 rows (512 rows, 20 KB of geometry in LDS).
constexpr int kCullBlock = 256;
constexpr int kCullIpt = 2;
constexpr int kCullTile = kCullBlock * kCullIpt;

// Workspace layout (bytes): header | tile counts (u64 visible<<32|saturated, then
// u32 restored) | tile prefixes (u64) | group sums [groups][2] (u64) | keep ballots
// [tiles][8] (u64) | saturated ballots [tiles][8] (u64, max_defer > 0) |
// saturated ids [n] (u32, max_defer > 0) | FP8 block maxima and task list
constexpr int64_t kWsHeader = 256;
struct WsHeader {
    uint32_t vis_total;      // visible rows of the last cull
    uint32_t sat_total;      // saturated rows listed by the last cull
    uint32_t restored_last;  // rows restored by the last cull
    uint32_t error;          // reserved, 0
    unsigned long long vis_accum;       // visible rows summed over all culls
    unsigned long long restored_accum;  // restored rows summed over all culls
};
static_assert(sizeof(WsHeader) == 32, "workspace header layout");

inline int64_t cull_tiles(int64_t n) { return (n + kCullTile - 1) / kCullTile; }
constexpr int kWordsPerTile = kCullTile / 64;
inline int64_t ws_cnt_offset(int64_t) { return kWsHeader; }
inline int64_t ws_off_offset(int64_t n) { return kWsHeader + 16 * cull_tiles(n); }
// groups of kGroupTiles tiles: per-group sums of (visible, saturated) and restored
constexpr int kGroupTiles = 64;
inline int64_t cull_groups(int64_t n) { return (cull_tiles(n) + kGroupTiles - 1) / kGroupTiles; }
inline int64_t ws_grp_offset(int64_t n) { return ws_off_offset(n) + 8 * cull_tiles(n); }
inline int64_t ws_keep_offset(int64_t n) { return ws_grp_offset(n) + 16 * cull_groups(n); }
inline int64_t ws_satbits_offset(int64_t n) { return ws_keep_offset(n) + 8 * kWordsPerTile * cull_tiles(n); }
inline int64_t ws_sat_offset(int64_t n, int32_t K)
{
    return ws_satbits_offset(n) + (K > 0 ? 8 * kWordsPerTile * cull_tiles(n) : 0);
}
inline int64_t fp8_blocks(int64_t n) { return (n + 127) / 128; }
inline int64_t ws_fp8_offset(int64_t n, int32_t K)
{
    const int64_t b = ws_sat_offset(n, K) + (K > 0 ? 4 * n : 0);
    return (b + 7) / 8 * 8;
}
// fp8: per-block max arrays for G m, G v, A m, A v (u32 each), the list of
// (moment, block) tasks that outgrew their scale this step (u32 each) and its
// length (u32, reset by the update pass)
inline int64_t ws_fp8_bytes(int64_t n) { return 32 * fp8_blocks(n) + 64; }
inline int64_t ws_bytes_for(int64_t n, int32_t K, int32_t fp8)
{
    const int64_t b = ws_fp8_offset(n, K) + (fp8 ? ws_fp8_bytes(n) : 0);
    return (b + 255) / 256 * 256;
}

int build_lut_host(double b1, double b2, int32_t T, int32_t K, const double *sched, float *out, int64_t nfloats);
int build_lut_sgdm_host(double mu, int32_t T, int32_t K, const double *sched, float *out, int64_t nfloats);
int build_lut_adamw_host(double b1, double b2, double lam, const float *rates, int nclass, int32_t T, int32_t K,
                         const double *sched, float *out, int64_t nfloats);

}  // namespace gsdp
