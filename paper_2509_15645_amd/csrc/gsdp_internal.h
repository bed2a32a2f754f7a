// Internal definitions shared by the host and device parts of libgsdp.
#pragma once
#include <stdint.h>

namespace gsdp {

// Device tables of the deferred update, O(T + K) bytes for T = max_steps and
// K = max_defer (Dn = K > 0 ? K : T is the largest defer count a row can hold,
// nrow = Dn + 1 entries per row).  Only the restore rows of two steps are
// held, in two slots (slot = step & 1): the update of step t reads the row
// of t and writes the row of t + 1 into the other slot.  Byte layout:
//   LutHeader                      64 bytes
//   Wf   [2][nrow] FP32            restore coefficient rows (unit rate)
//   Mf   [nrow]    FP32            b1^(d+1)
//   Vf   [nrow]    FP32            b2^(d+1)
//   SS   [T+2]     FP32            step size 1/(1-b1^t) (times the rate multiplier s[t])
//   BC   [T+2]     FP32            sqrt(1-b2^t)
//   Wd   [2][nrow] FP64            the rows before rounding (what the step advance accumulates)
//   R    [nrow]    FP64            weight of a newly skipped step at entry d+1
//   Cn   [T+2]     FP64            unit-rate contribution of skipped step k
//   per AdamW decay class: Wlf [2][nrow] FP32, Pf [2][nrow] FP32, qf [T+2] FP32,
//                          Wld [2][nrow] FP64, Pd [2][nrow] FP64, qd [T+2] FP64
// Advancing the rows from step t to t + 1 (d = 0 .. min(t, Dn) - 1):
//   W'[0] = 0,  W'[d+1] = W[d] + R[d] Cn[t]                  (Adam, SGD with momentum)
//   Wl'[0] = 0, Wl'[d+1] = q[t] Wl[d] + R[d] Cn[t],  P'[0] = 1, P'[d+1] = q[t] P[d]   (AdamW)
// every entry one IEEE binary64 multiply and add, rounded once to FP32.
struct LutHeader {
    int32_t t_row[2];        // step whose rows slot s holds (0: none)
    int32_t T, K;            // max_steps, max_defer
    int32_t nclass;          // AdamW decay classes (0 for Adam and SGD with momentum)
    int32_t error;           // bit 0: a call's step was not the one its row slot held;
                             // bit 1: a step outside [1, T] (graph replay past the tables)
    int32_t kind;            // 0 Adam, 1 SGD with momentum, 2 AdamW
    float wbound;            // >= every restore coefficient W_t[d] the tables hold, any t <= T + 1
    int32_t reserved[8];
};
static_assert(sizeof(LutHeader) == 64, "table header layout");
enum { kLutAdam = 0, kLutSgdm = 1, kLutAdamw = 2 };

inline int64_t align8(int64_t b) { return (b + 7) / 8 * 8; }

struct LutLayout {
    int64_t T, K, nrow;
    // byte offsets from the table base
    int64_t oWf, oMf, oVf, oSS, oBC, oWd, oR, oC, oCls;
    // byte offsets inside an AdamW class block, and its size
    int64_t cWlf, cPf, cqf, cWld, cPd, cqd, cls_bytes;
};

inline LutLayout lut_layout(int64_t T, int64_t K)
{
    LutLayout L;
    L.T = T;
    L.K = K;
    L.nrow = (K > 0 ? K : T) + 1;
    int64_t o = (int64_t)sizeof(LutHeader);
    L.oWf = o; o += 4 * 2 * L.nrow;
    L.oMf = o; o += 4 * L.nrow;
    L.oVf = o; o += 4 * L.nrow;
    L.oSS = o; o += 4 * (T + 2);
    L.oBC = o; o += 4 * (T + 2);
    o = align8(o);
    L.oWd = o; o += 8 * 2 * L.nrow;
    L.oR = o; o += 8 * L.nrow;
    L.oC = o; o += 8 * (T + 2);
    L.oCls = o;
    int64_t c = 0;
    L.cWlf = c; c += 4 * 2 * L.nrow;
    L.cPf = c; c += 4 * 2 * L.nrow;
    L.cqf = c; c += 4 * (T + 2);
    c = align8(c);
    L.cWld = c; c += 8 * 2 * L.nrow;
    L.cPd = c; c += 8 * 2 * L.nrow;
    L.cqd = c; c += 8 * (T + 2);
    L.cls_bytes = c;
    return L;
}

inline int64_t lut_total_bytes(int64_t T, int64_t K, int nclass)
{
    const LutLayout L = lut_layout(T, K);
    return L.oCls + nclass * L.cls_bytes;
}

constexpr int kMaxDecayClasses = 8;

// Cull tiles: 256 threads x 2 rows (512 rows, 20 KB of geometry in LDS).
constexpr int kCullBlock = 256;
constexpr int kCullIpt = 2;
constexpr int kCullTile = kCullBlock * kCullIpt;

// Workspace layout (bytes): header | tile counts (u64 visible<<32|saturated, then
// u32 restored) | tile prefixes (u64) | group sums [groups][2] (u64) | keep ballots
// [tiles][8] (u64) | saturated ballots [tiles][8] (u64, max_defer > 0) |
// saturated ids [n] (u32, max_defer > 0) | chunk decisions [chunks] (u32) |
// FP8 block maxima and task list
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
// rows of a chunk of the cull summaries' chunk records (GS_CHUNK_ROWS)
constexpr int kChunkRows = 1024;
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
// the summary cull's chunk decisions (u32 per chunk of kChunkRows rows)
inline int64_t cull_chunks(int64_t n) { return (n + kChunkRows - 1) / kChunkRows; }
inline int64_t ws_chunk_offset(int64_t n, int32_t K)
{
    const int64_t b = ws_sat_offset(n, K) + (K > 0 ? 4 * n : 0);
    return (b + 15) / 16 * 16;
}
inline int64_t fp8_blocks(int64_t n) { return (n + 127) / 128; }
inline int64_t ws_fp8_offset(int64_t n, int32_t K)
{
    const int64_t b = ws_chunk_offset(n, K) + 4 * cull_chunks(n);
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

// Host images of the tables at step 1 (`out`, lut_total_bytes bytes).
int build_lut_host(double b1, double b2, int32_t T, int32_t K, const double *sched, void *out, int64_t nbytes);
int build_lut_sgdm_host(double mu, int32_t T, int32_t K, const double *sched, void *out, int64_t nbytes);
int build_lut_adamw_host(double b1, double b2, double lam, const float *rates, int nclass, int32_t T, int32_t K,
                         const double *sched, void *out, int64_t nbytes);
// Advance a host image from the step it holds to `step` (each step as the
// device advance does it); -1 when step is below the held step or above T + 1.
int seek_lut_host(void *img, int64_t nbytes, int64_t step);

}  // namespace gsdp
