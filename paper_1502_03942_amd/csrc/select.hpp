// Host/device declarations of the single-instance selection path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace topk {

constexpr int PV_THREADS = 1024;               // sample/pivot, finisher, tail workgroup
constexpr int SEG_CAP = 16;                    // samples kept per sampler segment
constexpr int NSEG = PV_THREADS;               // sampler segments (one per thread)
constexpr int FIN_ITEMS = 16;                  // finisher keys per thread
constexpr int T_FIN_MAX = PV_THREADS * FIN_ITEMS;
constexpr int SW_THREADS = 1024;               // multi-workgroup sweep: 1 control + 15 data waves
constexpr int SW_DW = SW_THREADS / 64 - 1;     // data waves
constexpr int SW_COLS_IN = 64;                 // input keys per data-wave lane per tile
constexpr int SW_COLS_BAND = 16;               // band pairs per data-wave lane per tile
constexpr int SW_TILE_IN = SW_DW * 64 * SW_COLS_IN;     // 61440 keys
constexpr int SW_TILE_BAND = SW_DW * 64 * SW_COLS_BAND; // 15360 pairs
constexpr int SW_STASH = 320;                  // b pairs kept in LDS per wave-tile
constexpr int SW_SLOTS = 3;                    // wave-tile slots per data wave (pass 2 trails by 2)
constexpr int S_MAX = PV_THREADS * SEG_CAP;    // largest usable sample (16384)
constexpr int R_TRACE = 34;                    // attempt records kept (r_max <= 32, then the exact round)
constexpr int TRACE_STRIDE = NSEG * SEG_CAP;   // sampled objects per record
constexpr int64_t ROUND_EXACT = -2;            // lo = hi of the exact fallback round's record

enum : uint32_t { PH_PIVOT = 0, PH_SWEEP = 1, PH_DONE = 2 };

struct RoundRec {                 // same layout as topk_round_record
    uint32_t n_cur, k_cur, s, c_num;
    int64_t lo, hi;
    uint32_t l_idx, r_idx, has_l, has_r;
    uint32_t na, nb, ok, tag;
};

struct State {
    uint32_t phase, n_cur, k_cur, cursor;
    uint32_t src, tag, c_num, hs_ok;   // hs_ok: the sample collected by the last sweep is usable
    uint32_t na, nb, nrec, pad0;
    uint32_t l_ord, l_idx, r_ord, r_idx;
    uint32_t has_l, has_r, pad1, pad2;
    uint64_t hs_T;              // rate of the sample drawn from b (T = rho 2^32)
    uint32_t hs_count, pad4, pad5, pad6;   // elements taken into that sample
    // counters hit by every sweep workgroup, each on a 4 KiB page of its own
    // (atomics on words close together serialise with each other)
    alignas(4096) uint64_t resv; // sweep output reservations: |a| << 32 | |b|
    alignas(4096) uint32_t gen;  // sweep generations handed out beyond the first
    alignas(128) RoundRec rec[R_TRACE];
};

struct SelArgs {
    const uint32_t *keys;       // input key bits
    uint32_t n, k, flags;
    uint32_t *out_idx, *out_keys, *kth_key, *kth_idx, *status;
    State *st;
    uint32_t band_cap;
    uint32_t *band_ord[2], *band_idx[2];
    uint32_t *trace_pos;        // [R_TRACE][TRACE_STRIDE] sampled objects, or nullptr
    uint64_t *hs_buf;           // [S_MAX] sample drawn while b is formed: ord << 32 | position
    uint32_t *seg_cnt;          // [NSEG] round 1's sample size per segment (k_sample)
    uint32_t s_target, c_num0, t_fin, r_max;
    uint64_t seed;
    uint32_t first;             // first kernel of the call: initialise the state
    uint32_t presampled;        // round 1's sample is in hs_buf / seg_cnt
};

struct SelLaunch {
    int is_f32, largest;
    int r_fast;                 // multi-workgroup rounds before the tail kernel
    int sweep_grid[8];          // workgroups per enqueued sweep
};

// Optional HIP-event timing of the enqueued kernels (start/stop event pairs).
enum : int { KT_PIVOT_FIRST = 0, KT_PIVOT = 1, KT_SWEEP_FIRST = 2, KT_SWEEP = 3, KT_TAIL = 4 };
struct KernelTimer {
    int level;          // 0: off, 1: first sweep only, 2: every kernel
    hipEvent_t *ev;     // [2 * cap]
    int *kind;          // [cap]
    int cap, used;
};

hipError_t launch_select(const SelArgs &a, const SelLaunch &L, hipStream_t stream,
                         KernelTimer *tm);
int sweep_max_grid(bool is_f32, bool largest, int num_cu);

}  // namespace topk
