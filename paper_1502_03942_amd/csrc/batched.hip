// Batched selection: many rows of uneven length, each with its own k, in one
// persistent launch (§1: many similar selections solved together).
//
// Rows are ordered longest first (a counting sort by floor(log2 len)) and
// handed out from eight queues (one per XCD, each serving every eighth
// position of the order) to a persistent grid of 256-thread workgroups: one
// row per grab for the long rows, BT_QCHUNK per grab afterwards; rows under
// BT_WAVE_MAXLEN keys go one per wave, from a second set of queues.  One workgroup
// solves a row by the sampling method of §2 with the workgroup as the
// machine:
//   - a row of at most BT_REG_KEYS keys is the base case: its key order words
//     stay in registers, an exact radix select finds the pair of rank k and
//     the columns up to it are written in column order;
//   - a longer row draws a stratified sample of bt_s_target keys (one
//     uniform position in each of s equal strata) and takes the pivots L, R
//     at sample ranks k s / len -/+ Delta.  Then one sweep of the row:
//       fast form (the keys up to R are expected to fill at most 0.7 of the
//       LDS): every wave appends the keys <= R of its columns, with the
//       column, to a region of its own, counting those < L; no barrier until
//       the end.  The band [L, R] then holds rank k, found by one histogram
//       over the band's order words, and every candidate up to it is output;
//       general form: the part below L goes straight to the output, the band
//       to LDS, and the band is finished like a short row.
//     A miss (rank k outside the band) repeats the round with a new sample
//     and the spread doubled, an overflow of the LDS with the spread halved
//     (fast form: the general sweep of the same pivots); after bt_attempts
//     rounds an exact radix select over the row finishes it.
// Every decision is taken in the composite order (ord, column) of §2, or in
// the float order against a pivot value that is not NaN, which agrees with
// it, so the selected set is exactly the oracle's.
//
// Output per row: out_idx[out_off[r] .. + k) holds the selected columns in an
// order fixed by the inputs and the seed (short row or exact fallback: column
// order; general form: the part below L, then the rest, each in column order;
// fast form: wave by wave, each wave's columns ascending);
// kth_key[r] / kth_idx[r] the pair of rank k (key bits as stored).
//
// The waves of a workgroup exchange data only through LDS, so every barrier
// of k_batched orders LDS alone (lds_sync): output stores and key loads stay
// in flight across it.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"
#include "../../include/topk.h"

namespace topk {

constexpr int BT_THREADS = 256;                 // 4 waves
constexpr int BT_WAVES = BT_THREADS / WAVE;
constexpr u32 BT_CAP = 4096;                    // pairs in LDS: a band or the candidates
constexpr u32 BT_REG_KEYS = 8192;              // a short row: held in registers (32 per thread)
constexpr int BT_BITS = 10;                     // radix digit
constexpr u32 BT_BINS = 1u << BT_BITS;
constexpr int BT_BPT = (int)BT_BINS / BT_THREADS;   // histogram bins per thread in the scan
constexpr int BT_SEG = 8;                       // sample strata per thread (bt_s_target <= 2048)
static_assert(BT_SEG * BT_THREADS >= 2048 && BT_SEG * BT_THREADS <= BT_CAP,
              "the largest sample fits the strata slots and the LDS buffer");
constexpr int BT_IPT = 16;                      // keys per thread per step of the general sweep
constexpr u32 BT_STEP = BT_THREADS * BT_IPT;
constexpr int BT_NCLS = 34;                     // length classes 0 (empty) .. 33
constexpr int BT_HIST_THREADS = 1024;
constexpr u32 BT_REG = BT_CAP / BT_WAVES;       // fast sweep: candidate slots per wave
constexpr u32 BT_FAST_NUM = 7, BT_FAST_DEN = 10; // fast sweep when expected candidates <= 0.7 BT_CAP
constexpr u32 BT_NQ = 8;                        // row queues of each mode: one per XCD
constexpr u32 BT_QSTRIDE = 1088;                // words between two queue counters (4 KiB + 256 bytes)
constexpr u32 BT_Q1 = 64;                       // per queue: positions taken one at a time first
constexpr u32 BT_QCHUNK = 4;                    // then this many per grab
constexpr u32 BT_WAVE_M = 48;                   // wave mode: keys per lane at most
constexpr u32 BT_WAVE_MAXLEN = BT_WAVE_M * 64;  // rows shorter than this (3072 keys): one wave each
constexpr u32 BT_WAVE_CLS = 12;                 // the class of BT_WAVE_MAXLEN: rows of classes above
                                                // it are all longer, of classes below all shorter
constexpr u32 BT_WQCHUNK = 2;                   // rows per grab of a wave
constexpr size_t BT_GRAPHS_MAX = 32;            // instantiated graphs kept per context

struct BtShared {
    u64 buf[BT_CAP];
    u32 hist[BT_BINS];          // two targets' counts packed (low / high 16 bits)
    u64 cand[2][WAVE];
    alignas(16) u32 ecnt[BT_REG_KEYS / BT_THREADS][BT_WAVES];   // short row emit: counts per column block, wave
    u64 rmin[2], rmax[2], found[2];
    u32 ccount[2], sel_bin[2], sel_before[2], sel_count[2];
    u32 scan[BT_WAVES];
    u32 wt[2][BT_WAVES];        // sweep: per-wave (|a| | |b| << 16) of a step, by step parity
    u32 next;                   // the workgroup's last grab from a queue
    u32 n_wg;                   // order positions [0, n_wg): rows solved by the workgroup
};

// LDS of one wave in the wave-per-row mode (inside BtShared::buf).
struct BtWaveLds {
    u32 hist[BT_BINS];
    u64 cand[WAVE];
};
static_assert(sizeof(BtWaveLds) * BT_WAVES <= sizeof(u64) * BT_CAP, "wave LDS fits the band buffer");

struct BtArgs {
    const u32 *keys;
    const u64 *row_off;
    const u32 *k;
    const u64 *out_off;
    u32 rows, flags;
    u32 *out_idx, *kth_key, *kth_idx, *status;
    u32 *cls_cnt, *cls_fill, *order, *queue;
    u64 seed;
    u32 attempts, fast;
    u32 cls_lo, cls_hi;                 // only rows of these length classes
    u32 s_cls[BT_NCLS], c_cls[BT_NCLS]; // sample size and spread by length class
    u32 t_cls[BT_NCLS];                 // fast-sweep tile (keys per thread per step: 8 or 16)
};

__device__ __forceinline__ u32 len_class(u64 len)
{
    const u32 c = len == 0 ? 0u : 64u - (u32)__clzll((long long)len);
    return c < (u32)BT_NCLS ? c : (u32)BT_NCLS - 1;
}

// The thread index as a value the compiler cannot see through: what is
// derived from it is computed where it is used, not hoisted out of the
// persistent row loop into registers that then spill.
__device__ __forceinline__ u32 bt_tid()
{
    u32 t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

__device__ __forceinline__ u64 uniform64(u64 x)
{
    return ((u64)(u32)__builtin_amdgcn_readfirstlane((u32)(x >> 32)) << 32) |
           (u32)__builtin_amdgcn_readfirstlane((u32)x);
}

__device__ __forceinline__ bool bt_match(u64 x, u64 pref, int lowb)
{
    return lowb >= 64 || (x >> lowb) == (pref >> lowb);
}

// Pairs of 0-based ranks rank[0], rank[1] (each if act[t]) among src(0 .. n-1)
// (distinct pairs): radix select over windows of BT_BITS bits, from bit `top`
// down (every pair agrees above `top`), keeping the bucket that holds each
// rank; a bucket of at most 64 pairs is ranked by one wave.  Both targets
// share every scan of the source; their counts share one histogram (16 bits
// each) when n < 2^16, else only target 0 may be active.  All threads call it
// and get res[].
template <class SRC>
__device__ void bt_select(SRC src, u32 n, int top, const u64 rank_in[2], const bool act[2],
                          u64 res[2], BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const bool packed = n < 65536u;
    u64 pref[2] = {0ull, 0ull};
    int lowb[2] = {top, top};           // bits [lowb, 64) of the candidates equal pref's
    u64 rank[2] = {rank_in[0], rank_in[1]};
    bool done[2] = {!act[0], !act[1]};
    res[0] = res[1] = 0ull;
    // every histogram bin is zero on entry (all users leave it so); the
    // candidate counters are first used after the first pass's barriers
    if (tid < 2) sh.ccount[tid] = 0u;
    if (top >= 64) {
        // pref's bits at or above `top` are those of any pair
        const u64 x0 = n ? src(0) : 0ull;
        pref[0] = pref[1] = x0;
    } else {
        const u64 x0 = n ? src(0) : 0ull;
        pref[0] = pref[1] = top <= 0 ? x0 : (x0 >> top) << top;
    }
    for (int pass = 0; pass < 16 && !(done[0] && done[1]); ++pass) {
        int sh_[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (!done[t] && lowb[t] <= 0) {
                res[t] = pref[t];                   // every bit fixed: one pair
                done[t] = true;
            }
            sh_[t] = lowb[t] > BT_BITS ? lowb[t] - BT_BITS : 0;
        }
        if (done[0] && done[1]) break;
        // (1) histogram of each target's window
        for (u32 i = tid; i < n; i += BT_THREADS) {
            const u64 x = src(i);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                if (!done[t] && bt_match(x, pref[t], lowb[t]))
                    atomicAdd(&sh.hist[(u32)(x >> sh_[t]) & (BT_BINS - 1)], t == 0 ? 1u : 65536u);
        }
        lds_sync();
        // (2) scan: thread t covers bins [BT_BPT t, BT_BPT t + BT_BPT)
        u32 c[BT_BPT], csum = 0;
#pragma unroll
        for (int q = 0; q < BT_BPT; ++q) {
            c[q] = sh.hist[tid * BT_BPT + q];
            sh.hist[tid * BT_BPT + q] = 0u;      // clean for the next pass
            csum += c[q];
        }
        u32 tot;
        u32 before = block_excl_scan<BT_THREADS, true>(csum, sh.scan, &tot);
#pragma unroll
        for (int q = 0; q < BT_BPT; ++q) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (done[t]) continue;
                const u32 bt = !packed ? before : t == 0 ? (before & 0xFFFFu) : (before >> 16);
                const u32 ct = !packed ? c[q] : t == 0 ? (c[q] & 0xFFFFu) : (c[q] >> 16);
                if ((u64)bt <= rank[t] && rank[t] < (u64)bt + ct) {
                    sh.sel_bin[t] = tid * BT_BPT + q;
                    sh.sel_before[t] = bt;
                    sh.sel_count[t] = ct;
                }
            }
            before += c[q];
        }
        lds_sync();
        bool gather[2] = {false, false};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (done[t]) continue;
            const u32 wb = lowb[t] - sh_[t];                    // window width
            const u64 wmask = wb >= 64 ? ~0ull : ((1ull << wb) - 1) << sh_[t];
            pref[t] = (pref[t] & ~wmask) | (((u64)sh.sel_bin[t] << sh_[t]) & wmask);
            lowb[t] = sh_[t];
            rank[t] -= sh.sel_before[t];
            if (sh.sel_count[t] == 1u || lowb[t] == 0) {
                if (lowb[t] == 0) {
                    res[t] = pref[t];                           // every bit fixed
                    done[t] = true;
                } else {
                    gather[t] = true;
                }
            } else {
                gather[t] = sh.sel_count[t] <= (u32)WAVE;
            }
        }
        if (gather[0] || gather[1]) {
            for (u32 i = tid; i < n; i += BT_THREADS) {
                const u64 x = src(i);
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    if (gather[t] && bt_match(x, pref[t], lowb[t]))
                        sh.cand[t][atomicAdd(&sh.ccount[t], 1u)] = x;
            }
            lds_sync();
            if (w < 2 && gather[w]) {
                const u32 m = sh.ccount[w];
                const u64 mine = lane < m ? sh.cand[w][lane] : ~0ull;
                const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
                u32 below = 0;
                for (u32 i = 0; i < m; ++i) {
                    const u64 o = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                                  (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
                    below += o < mine ? 1u : 0u;
                }
                if (lane < m && (u64)below == rank[w]) sh.found[w] = mine;
            }
            lds_sync();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (!gather[t]) continue;
                res[t] = sh.found[t];
                done[t] = true;
            }
            if (tid < 2) sh.ccount[tid] = 0u;
            lds_sync();
        }
    }
}

// Write the columns of the pairs <= tau among src(0 .. n-1), in source order,
// to out[0 ..) (at most `limit`).  A step of BT_STEP pairs gives wave w the
// pairs [s0 + 1024 w, s0 + 1024 w + 1024) as 16 columns of 64 lanes (LDS
// reads without bank conflicts); the waves' counts are exchanged once per
// step, then every wave writes its pairs in order.
template <class SRC>
__device__ void bt_emit(SRC src, u32 n, u64 tau, u32 *out, u32 limit, BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    u32 cur = 0;
    for (u32 s0 = 0; s0 < n; s0 += BT_STEP) {
        const u32 b0 = s0 + w * (BT_STEP / BT_WAVES);
        u32 bits = 0, c = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const u32 i = b0 + (u32)j * WAVE + lane;
            const bool t = i < n && src(i) <= tau;
            bits |= (u32)t << j;
            c += (u32)__popcll(ballot(t));
        }
        if (lane == 0) sh.scan[w] = c;
        lds_sync();
        u32 pos = cur, tot = 0;
#pragma unroll
        for (int v = 0; v < BT_WAVES; ++v) {
            const u32 sv = __builtin_amdgcn_readfirstlane(sh.scan[v]);
            pos += (u32)v < w ? sv : 0u;
            tot += sv;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const bool t = (bits >> j) & 1u;
            const u64 m = ballot(t);
            if (t) {
                const u32 q = pos + mbcnt(m);
                if (q < limit) out[q] = (u32)src(b0 + (u32)j * WAVE + lane);
            }
            pos += (u32)__popcll(m);
        }
        cur += tot;
        lds_sync();            // sh.scan is rewritten by the next step
    }
}

// Stratified sample of a row for the pivots: the row is cut into s equal
// strata (boundaries floor(q len / s), q = 0 .. s) and one position is drawn
// uniformly from each, with 32-bit draws of Philox4x32-10 at counter (j / 4,
// t, tag, row), key = seed.  Thread t takes the strata q = j BT_THREADS + t
// below s and returns how many.  Against a Bernoulli sample at rate s / len
// the size is exact and, for any threshold, the number of sampled keys below
// it has the same mean and no larger variance (a sum of independent draws,
// one per stratum), so the pivot ranks of §2 keep their guarantee.
__device__ __forceinline__ int bt_sample(u32 t, u32 len, u32 s, u64 seed, u32 tag, u32 row,
                                         u32 (&pos)[BT_SEG])
{
    const u64 step = ((u64)len << 32) / s;      // stratum width, 32.32 fixed point
    const u32 nj = (s + BT_THREADS - 1) / BT_THREADS;
    int cnt = 0;
#pragma unroll
    for (int j0 = 0; j0 < BT_SEG; j0 += 4) {
        if ((u32)j0 >= nj) break;
        const uint4 r4 = philox4x32_10(make_uint4((u32)(j0 >> 2), t, tag, row), (u32)seed, (u32)(seed >> 32));
        const u32 w[4] = {r4.x, r4.y, r4.z, r4.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const u32 q = (u32)(j0 + i) * BT_THREADS + t;
            if (q < s) {
                const u32 b = (u32)(((u64)q * step) >> 32);
                const u32 e = (u32)(((u64)(q + 1) * step) >> 32);
                pos[j0 + i] = b + (u32)(((u64)w[i] * (e - b)) >> 32);
                cnt = j0 + i + 1;
            }
        }
    }
    return cnt;
}

// Float value whose key order word is o (o not the NaN image).
template <bool LARGEST>
__device__ __forceinline__ float ord_value(u32 o)
{
    const u32 v = LARGEST ? ~o : o;
    return __uint_as_float((v & 0x80000000u) ? (v & 0x7FFFFFFFu) : ~v);
}

template <bool LARGEST>
__device__ __forceinline__ bool ord_is_nan(u32 o) { return (LARGEST ? ~o : o) == 0xFFFFFFFFu; }

// min / max of a u32 over the wave (wave-uniform result)
template <bool MAX>
__device__ __forceinline__ u32 bt_wave_ext_u32(u32 v)
{
    auto step = [&](auto ctrl_tag, auto rows_tag) {
        constexpr int C = decltype(ctrl_tag)::value, R = decltype(rows_tag)::value;
        const u32 x = (u32)__builtin_amdgcn_update_dpp((int)v, (int)v, C, R, 0xF, false);
        v = MAX ? (x > v ? x : v) : (x < v ? x : v);
    };
    step(std::integral_constant<int, DPP_XOR1>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_XOR2>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_ROW_HALF_MIRROR>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_ROW_MIRROR>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_ROW_BCAST15>(), std::integral_constant<int, 0xA>());
    step(std::integral_constant<int, DPP_ROW_BCAST31>(), std::integral_constant<int, 0xC>());
    return (u32)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

// Histogram bins linear in the key value.  g(o), the key value of order
// word o (negated for largest), is non-decreasing in o; bin(o) = clamp of
// floor(g(o) scale + bias), one fused multiply-add, is then non-decreasing
// in o as well (every rounding step is monotone), and every evaluation of
// it gives the same bin.  So all pairs of a lower bin precede all pairs of a
// higher one, and equal keys share a bin.
template <bool LARGEST>
__device__ __forceinline__ float ord_lin(u32 o)
{
    const float v = ord_value<LARGEST>(o);
    return LARGEST ? -v : v;
}

template <bool LARGEST, u32 NB = BT_BINS>
__device__ __forceinline__ u32 lin_bin(u32 o, float scale, float bias)
{
    const float t = fmaxf(__builtin_fmaf(ord_lin<LARGEST>(o), scale, bias), 0.0f);
    const u32 b = (u32)t;
    return b < NB - 1 ? b : NB - 1;
}

// NB bins over the order words [omin, omax]: false if the range holds a
// NaN, an infinity or a single value (the radix select handles those).
template <bool LARGEST, u32 NB = BT_BINS>
__device__ __forceinline__ bool lin_setup(u32 omin, u32 omax, float &scale, float &bias)
{
    if (omin >= omax || ord_is_nan<LARGEST>(omin) || ord_is_nan<LARGEST>(omax)) return false;
    const float g0 = ord_lin<LARGEST>(omin), g1 = ord_lin<LARGEST>(omax);
    const float span = g1 - g0;
    if (!(span > 0.0f) || !__builtin_isfinite(g0) || !__builtin_isfinite(g1) || !__builtin_isfinite(span))
        return false;
    scale = (float)(NB - 1) / span;
    bias = -g0 * scale;
    return __builtin_isfinite(scale) && __builtin_isfinite(bias);
}

// IPT keys per lane of one sweep step (the tile: BT_THREADS * IPT keys),
// interleaved so that wave w holds columns s0 + (j * BT_WAVES + w) * 64 + lane.
template <bool GUARD, int IPT>
__device__ __forceinline__ void bt_load_step(const u32 *__restrict__ row, u32 s0, u32 len, u32 w,
                                             u32 lane, u32 (&x)[IPT])
{
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const u32 col = s0 + ((u32)j * BT_WAVES + w) * WAVE + lane;
        x[j] = row[GUARD ? (col < len ? col : len - 1) : col];
    }
}

// Fast sweep, one step of one wave: the keys at or below the upper pivot R
// (compared as floats: for a pivot value that is not NaN, the float order and
// the key order agree, -0 and +0 included) are appended with their column to
// the wave's own LDS region; `na` counts those below the lower pivot L.  The
// regions of the waves are independent, so the sweep needs no barrier.
template <bool LARGEST, bool TAIL, int IPT>
__device__ __forceinline__ void bt_fast_step(const u32 (&x)[IPT], u32 s0, u32 len, u32 w, u32 lane,
                                             float fL, float fR, u64 *reg, u32 &cnt, u32 &na)
{
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const u32 col = s0 + ((u32)j * BT_WAVES + w) * WAVE + lane;
        const float f = __uint_as_float(x[j]);
        // largest: NaN keys come first, so "not below R" and "not at or below L"
        bool ab = LARGEST ? !(f < fR) : (f <= fR);
        bool ia = LARGEST ? !(f <= fL) : (f < fL);
        if (TAIL) {
            const bool ok = col < len;
            ab = ab && ok;
            ia = ia && ok;
        }
        const u64 m = ballot(ab);
        // past the region's end every write lands on its last slot: the
        // count then exceeds BT_REG and the caller discards the region
        u32 q = cnt + mbcnt(m);
        q = q < BT_REG - 1 ? q : BT_REG - 1;
        if (ab) {
            u32 *e = (u32 *)(reg + q);
            e[0] = col;
            e[1] = x[j];
        }
        cnt += (u32)__popcll(m);
        na += (u32)__popcll(ballot(ia));
        asm volatile("" : "+s"(cnt), "+s"(na));     // keep the sums current
    }
}

// The whole fast sweep of one wave over the row, loads one step ahead
// (IPT keys per lane per step: the tile size the autotuner picks).
template <bool LARGEST, int IPT>
__device__ __forceinline__ void bt_fast_sweep(const u32 *__restrict__ row, u32 len, float fL, float fR, bool hl,
                              u64 *reg, u32 &cnt_out, u32 &na_out)
{
    constexpr u32 STEP = BT_THREADS * IPT;
    const u32 tid = bt_tid();
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE), lane = tid & (WAVE - 1);
    u32 cnt = 0, na = 0;
    u32 x[IPT], y[IPT];
    auto load = [&](u32 (&v)[IPT], u32 s0) {
        if (s0 + STEP <= len) bt_load_step<false, IPT>(row, s0, len, w, lane, v);
        else bt_load_step<true, IPT>(row, s0, len, w, lane, v);
    };
    auto step = [&](const u32 (&v)[IPT], u32 s0) {
        if (s0 + STEP <= len) bt_fast_step<LARGEST, false, IPT>(v, s0, len, w, lane, fL, fR, reg, cnt, na);
        else bt_fast_step<LARGEST, true, IPT>(v, s0, len, w, lane, fL, fR, reg, cnt, na);
    };
    u32 s0 = 0;
    load(x, 0);
    for (;;) {
        // the next step's loads go out before this step is classified (past
        // the end: the last step again, whose addresses are valid)
        const u32 s1 = s0 + STEP < len ? s0 + STEP : s0;
        load(y, s1);
        step(x, s0);
        if (s1 == s0) break;
        s0 = s1;
        const u32 s2 = s0 + STEP < len ? s0 + STEP : s0;
        load(x, s2);
        step(y, s0);
        if (s2 == s0) break;
        s0 = s2;
    }
    cnt_out = cnt;
    na_out = hl ? na : 0u;          // no lower pivot: nothing lies below it
}

// Write the columns of the fast sweep's candidates up to tau to out[0 ..)
// (at most `limit`): wave v's region holds sh.wt[0][v] pairs; the waves'
// counts are exchanged once, then every wave writes its pairs in region
// order after those of the waves before it.
__device__ __forceinline__ void bt_emit_regions(u64 tau, u32 *out, u32 limit, BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const u32 cw = __builtin_amdgcn_readfirstlane(sh.wt[0][w]);
    u32 pos = 0;
    const u64 *reg = sh.buf + w * BT_REG;
    const u32 nc = (cw + WAVE - 1) / WAVE;          // at most BT_REG / WAVE = 16
    static_assert(BT_REG / WAVE <= 32, "one selection bit per region column");
    u32 bits = 0, c = 0;
    for (u32 j = 0; j < nc; ++j) {
        const u32 i = j * WAVE + lane;
        const bool t = i < cw && reg[i] <= tau;
        bits |= (u32)t << j;
        c += (u32)__popcll(ballot(t));
    }
    if (lane == 0) sh.scan[w] = c;
    lds_sync();
#pragma unroll
    for (int v = 0; v < BT_WAVES; ++v)
        if ((u32)v < w) pos += __builtin_amdgcn_readfirstlane(sh.scan[v]);
    for (u32 j = 0; j < nc; ++j) {
        const bool t = (bits >> j) & 1u;
        const u64 m = ballot(t);
        if (t) {
            const u32 q = pos + mbcnt(m);
            if (q < limit) out[q] = (u32)reg[j * WAVE + lane];
        }
        pos += (u32)__popcll(m);
    }
    // sh.scan is next written after the barrier that ends the row
}

// Rank `rank` (0-based) among the fast sweep's candidates, the pairs
// sh.buf[v BT_REG + (0 .. cnt[v])) of the waves v, which are a prefix of the
// row's order; the band [ordL, ordR] of key order words holds the target
// unless the pivots missed.  One histogram pass: bin 0 counts the order words
// below ordL (by ballots), bins 1 .. by (o - ordL) >> shift, the last bin
// anything above ordR.  A target bin of at most 64 pairs is ranked by one
// wave; otherwise the generic radix select over the slots decides (`ssrc`:
// empty slots read as ~0, above every candidate).
template <class SRC>
__device__ __forceinline__ u64 bt_band_tau(SRC ssrc, const u32 (&cnt)[BT_WAVES], u32 ordL, u32 ordR,
                                           u32 rank, BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const u32 span = ordR - ordL;
    u32 shift = 0;
    while ((span >> shift) > BT_BINS - 3) ++shift;
    auto bin = [&](u64 c) -> u32 {
        const u32 o = (u32)(c >> 32);
        if (o < ordL) return 0u;
        const u32 b = 1u + ((o - ordL) >> shift);
        return b < BT_BINS - 1 ? b : BT_BINS - 1;
    };
    // every histogram bin is zero on entry (all users leave it so)
    if (tid == 0) sh.ccount[0] = 0u;
    u32 below = 0;
#pragma unroll
    for (int v = 0; v < BT_WAVES; ++v) {
        for (u32 i = tid; i < cnt[v]; i += BT_THREADS) {
            const u64 x = sh.buf[(u32)v * BT_REG + i];
            const bool lo = (u32)(x >> 32) < ordL;
            below += (u32)__popcll(ballot(lo));
            if (!lo) atomicAdd(&sh.hist[bin(x)], 1u);
        }
    }
    if (lane == 0 && below) atomicAdd(&sh.hist[0], below);
    lds_sync();
    u32 c[BT_BPT], csum = 0;
#pragma unroll
    for (int q = 0; q < BT_BPT; ++q) {
        c[q] = sh.hist[tid * BT_BPT + q];
        sh.hist[tid * BT_BPT + q] = 0u;      // every bin is left at zero
        csum += c[q];
    }
    u32 tot;
    u32 before = block_excl_scan<BT_THREADS, true>(csum, sh.scan, &tot);
#pragma unroll
    for (int q = 0; q < BT_BPT; ++q) {
        if (before <= rank && rank < before + c[q]) {
            sh.sel_bin[0] = tid * BT_BPT + q;
            sh.sel_before[0] = before;
            sh.sel_count[0] = c[q];
        }
        before += c[q];
    }
    lds_sync();
    const u32 b = __builtin_amdgcn_readfirstlane(sh.sel_bin[0]);
    const u32 nb = __builtin_amdgcn_readfirstlane(sh.sel_count[0]);
    const u32 rr = rank - __builtin_amdgcn_readfirstlane(sh.sel_before[0]);
    if (nb > (u32)WAVE) {
        lds_sync();
        const u64 rk[2] = {(u64)rank, 0ull};
        const bool one[2] = {true, false};
        u64 t2[2];
        bt_select(ssrc, BT_CAP, 64, rk, one, t2, sh);
        return t2[0];
    }
#pragma unroll
    for (int v = 0; v < BT_WAVES; ++v) {
        for (u32 i = tid; i < cnt[v]; i += BT_THREADS) {
            const u64 x = sh.buf[(u32)v * BT_REG + i];
            if (bin(x) == b) sh.cand[0][atomicAdd(&sh.ccount[0], 1u)] = x;
        }
    }
    lds_sync();
    if (w == 0) {
        const u64 mine = lane < nb ? sh.cand[0][lane] : ~0ull;
        const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
        u32 lt = 0;
        for (u32 i = 0; i < nb; ++i) {
            const u64 o = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                          (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
            lt += o < mine ? 1u : 0u;
        }
        if (lane < nb && lt == rr) sh.found[0] = mine;
    }
    lds_sync();
    return sh.found[0];
}

// Pair of rank `rank` (0-based) among the pairs (o[j], j BT_THREADS + tid)
// held in registers (valid while the column is below n): radix select over
// windows of BT_BITS bits of the 64-bit pair from the top, keeping the bucket
// that holds the rank, until it has at most 64 pairs, which one wave ranks.
// Column blocks j at or past ceil(n / BT_THREADS) are skipped as a whole.
// Every histogram bin is zero on entry and on return.
template <int M>
__device__ __forceinline__ u64 bt_reg_select(const u32 (&o)[M], u32 n, u32 rank, BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const u32 jn = (n + BT_THREADS - 1) / BT_THREADS;
    u32 ph = 0, pl = 0;                 // prefix: the bits at and above lowb are fixed
    int lowb = 64;
    u32 rk = rank;
    auto match = [&](u32 oj, u32 col) -> bool {
        if (lowb >= 64) return true;
        if (lowb >= 32) return (oj >> (lowb - 32)) == (ph >> (lowb - 32));
        return oj == ph && (col >> lowb) == (pl >> lowb);
    };
    u32 cnt = n;
    while (cnt > (u32)WAVE && lowb > 0) {
        const int sh_ = lowb > BT_BITS ? lowb - BT_BITS : 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if ((u32)j < jn) {
                const u32 col = (u32)j * BT_THREADS + tid;
                if (col < n && match(o[j], col)) {
                    const u32 d = sh_ >= 32 ? (o[j] >> (sh_ - 32)) & (BT_BINS - 1)
                                            : (u32)(pack(o[j], col) >> sh_) & (BT_BINS - 1);
                    atomicAdd(&sh.hist[d], 1u);
                }
            }
        }
        lds_sync();
        u32 c[BT_BPT], csum = 0;
#pragma unroll
        for (int q = 0; q < BT_BPT; ++q) {
            c[q] = sh.hist[tid * BT_BPT + q];
            sh.hist[tid * BT_BPT + q] = 0u;
            csum += c[q];
        }
        u32 tot;
        u32 before = block_excl_scan<BT_THREADS, true>(csum, sh.scan, &tot);
#pragma unroll
        for (int q = 0; q < BT_BPT; ++q) {
            if (before <= rk && rk < before + c[q]) {
                sh.sel_bin[0] = tid * BT_BPT + q;
                sh.sel_before[0] = before;
                sh.sel_count[0] = c[q];
            }
            before += c[q];
        }
        lds_sync();
        const u64 bsel = (u64)__builtin_amdgcn_readfirstlane(sh.sel_bin[0]) << sh_;
        cnt = __builtin_amdgcn_readfirstlane(sh.sel_count[0]);
        rk -= __builtin_amdgcn_readfirstlane(sh.sel_before[0]);
        ph |= (u32)(bsel >> 32);
        pl |= (u32)bsel;
        lowb = sh_;
    }
    if (lowb == 0) return ((u64)ph << 32) | pl;     // every bit fixed: that pair
    if (tid == 0) sh.ccount[0] = 0u;
    lds_sync();
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn) {
            const u32 col = (u32)j * BT_THREADS + tid;
            if (col < n && match(o[j], col)) sh.cand[0][atomicAdd(&sh.ccount[0], 1u)] = pack(o[j], col);
        }
    }
    lds_sync();
    if (w == 0) {
        const u64 mine = lane < cnt ? sh.cand[0][lane] : ~0ull;
        const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
        u32 lt = 0;
        for (u32 i = 0; i < cnt; ++i) {
            const u64 x = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                          (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
            lt += x < mine ? 1u : 0u;
        }
        if (lane < cnt && lt == rk) sh.found[0] = mine;
    }
    lds_sync();
    return sh.found[0];
}

// First try for a row held in registers: one histogram pass over bins
// linear in the key value between the row's least and greatest key, then,
// if the bin holding rank `rank` has at most 64 pairs, one wave ranks them.
// Returns false, every bin left at zero, when the range allows no linear
// bins or the bin is larger; the radix select then decides.
template <bool LARGEST, int M>
__device__ __forceinline__ bool bt_reg_lin(const u32 (&o)[M], u32 n, u32 rank, BtShared &sh, u64 &tau)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const u32 jn = (n + BT_THREADS - 1) / BT_THREADS;
    u32 mn = ~0u, mx = 0u;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn && (u32)j * BT_THREADS + tid < n) {
            mn = o[j] < mn ? o[j] : mn;
            mx = o[j] > mx ? o[j] : mx;
        }
    }
    mn = bt_wave_ext_u32<false>(mn);
    mx = bt_wave_ext_u32<true>(mx);
    if (lane == 0) {
        sh.wt[0][w] = mn;
        sh.wt[1][w] = mx;
    }
    if (tid == 0) sh.ccount[0] = 0u;
    lds_sync();
    u32 omin = ~0u, omax = 0u;
#pragma unroll
    for (int v = 0; v < BT_WAVES; ++v) {
        const u32 a0 = __builtin_amdgcn_readfirstlane(sh.wt[0][v]);
        const u32 a1 = __builtin_amdgcn_readfirstlane(sh.wt[1][v]);
        omin = a0 < omin ? a0 : omin;
        omax = a1 > omax ? a1 : omax;
    }
    float scale, bias;
    if (!lin_setup<LARGEST>(omin, omax, scale, bias)) return false;
#pragma unroll
    for (int j = 0; j < M; ++j)
        if ((u32)j < jn && (u32)j * BT_THREADS + tid < n)
            atomicAdd(&sh.hist[lin_bin<LARGEST>(o[j], scale, bias)], 1u);
    lds_sync();
    u32 c[BT_BPT], csum = 0;
#pragma unroll
    for (int q = 0; q < BT_BPT; ++q) {
        c[q] = sh.hist[tid * BT_BPT + q];
        sh.hist[tid * BT_BPT + q] = 0u;
        csum += c[q];
    }
    u32 tot;
    u32 before = block_excl_scan<BT_THREADS, true>(csum, sh.scan, &tot);
#pragma unroll
    for (int q = 0; q < BT_BPT; ++q) {
        if (before <= rank && rank < before + c[q]) {
            sh.sel_bin[0] = tid * BT_BPT + q;
            sh.sel_before[0] = before;
            sh.sel_count[0] = c[q];
        }
        before += c[q];
    }
    lds_sync();
    const u32 b = __builtin_amdgcn_readfirstlane(sh.sel_bin[0]);
    const u32 cnt = __builtin_amdgcn_readfirstlane(sh.sel_count[0]);
    const u32 rr = rank - __builtin_amdgcn_readfirstlane(sh.sel_before[0]);
    if (cnt > (u32)WAVE) return false;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const u32 col = (u32)j * BT_THREADS + tid;
        if ((u32)j < jn && col < n && lin_bin<LARGEST>(o[j], scale, bias) == b)
            sh.cand[0][atomicAdd(&sh.ccount[0], 1u)] = pack(o[j], col);
    }
    lds_sync();
    if (w == 0) {
        const u64 mine = lane < cnt ? sh.cand[0][lane] : ~0ull;
        const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
        u32 lt = 0;
        for (u32 i = 0; i < cnt; ++i) {
            const u64 x = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                          (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
            lt += x < mine ? 1u : 0u;
        }
        if (lane < cnt && lt == rr) sh.found[0] = mine;
    }
    lds_sync();
    tau = sh.found[0];
    return true;
}

// Write the columns of the register pairs <= tau in column order to out[0 ..)
// (at most `limit`): lane j of each wave keeps the wave's count of column
// block j, the counts go to LDS in one store, and after one barrier lane j
// finds where the wave's pairs of block j start (the blocks before it, then
// the waves before this one in block j).
template <int M>
__device__ __forceinline__ void bt_reg_emit(const u32 (&o)[M], u32 n, u64 tau, u32 *out, u32 limit,
                                            BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const u32 jn = (n + BT_THREADS - 1) / BT_THREADS;
    const u32 th = (u32)(tau >> 32), tl = (u32)tau;
    static_assert(M <= 32 && BT_WAVES == 4, "one selection bit per column block; four waves");
    u32 bits = 0, myc = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn) {
            const u32 col = (u32)j * BT_THREADS + tid;
            const bool t = col < n && (o[j] < th || (o[j] == th && col <= tl));
            bits |= (u32)t << j;
            const u32 c = (u32)__popcll(ballot(t));
            myc = lane == (u32)j ? c : myc;
        }
    }
    if (lane < jn) sh.ecnt[lane][w] = myc;
    lds_sync();
    u32 all = 0, mine = 0;
    if (lane < jn) {
        const uint4 c4 = *(const uint4 *)sh.ecnt[lane];
        all = c4.x + c4.y + c4.z + c4.w;
        mine = (w > 0 ? c4.x : 0u) + (w > 1 ? c4.y : 0u) + (w > 2 ? c4.z : 0u);
    }
    const u32 incl = wave_incl_scan(all);
    const u32 off = incl - all + mine;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn) {
            const bool t = (bits >> j) & 1u;
            const u64 m = ballot(t);
            const u32 base = (u32)__builtin_amdgcn_readlane((int)off, j);
            if (t) {
                const u32 q = base + mbcnt(m);
                if (q < limit) out[q] = (u32)j * BT_THREADS + tid;
            }
        }
    }
    // ecnt is next written after the barrier that ends the row
}

// A row of at most M BT_THREADS keys, held in registers as key order words;
// thread 0 gets the key bits of the pair of rank k in kbits.
template <bool LARGEST, int M>
__device__ __forceinline__ u64 bt_reg_row(const u32 *__restrict__ row, u32 len, u32 k, u32 *out,
                                          u32 &kbits, BtShared &sh)
{
    const u32 tid = bt_tid();
    const u32 jn = (len + BT_THREADS - 1) / BT_THREADS;
    u32 o[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const u32 col = (u32)j * BT_THREADS + tid;
        // every load is issued before the first is used (a column past the
        // row reads its last key; such slots are never counted)
        o[j] = (u32)j < jn ? row[col < len ? col : len - 1] : 0u;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) o[j] = key_ord<true, LARGEST>(o[j]);
    u64 tau;
    if (!bt_reg_lin<LARGEST, M>(o, len, k - 1, sh, tau)) tau = bt_reg_select<M>(o, len, k - 1, sh);
    if (bt_tid() == 0) kbits = row[(u32)tau];      // in flight during the output
    bt_reg_emit<M>(o, len, tau, out, k, sh);
    return tau;
}

// ---- One wave per row -----------------------------------------------------
// A row of fewer than BT_WAVE_M * 64 keys is solved by one wave alone, its
// key order words in registers (column j * 64 + lane in o[j]): the radix
// select and the output run on wave-level operations and the wave's own LDS,
// with no workgroup barrier, so the four waves of a workgroup work on four
// rows at once.

// Pair of rank `rank` (0-based) among the wave's pairs (o[j], j 64 + lane),
// valid below column n: radix select over windows of BT_BITS bits of the
// pair from the top until the bucket holding the rank has at most 64 pairs,
// which are ranked by comparison.  Every bin of L.hist is zero on entry and
// on return.  Wave-uniform result.
template <int M>
__device__ __forceinline__ u64 bt_wave_select(const u32 (&o)[M], u32 n, u32 rank, BtWaveLds &L)
{
    const u32 lane = bt_tid() & (WAVE - 1);
    const u32 jn = (n + WAVE - 1) / WAVE;
    u32 ph = 0, pl = 0;                 // prefix: the bits at and above lowb are fixed
    int lowb = 64;
    u32 rk = rank, cnt = n;
    auto match = [&](u32 oj, u32 col) -> bool {
        if (lowb >= 64) return true;
        if (lowb >= 32) return (oj >> (lowb - 32)) == (ph >> (lowb - 32));
        return oj == ph && (col >> lowb) == (pl >> lowb);
    };
    while (cnt > (u32)WAVE && lowb > 0) {
        const int sh_ = lowb > BT_BITS ? lowb - BT_BITS : 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if ((u32)j < jn) {
                const u32 col = (u32)j * WAVE + lane;
                if (col < n && match(o[j], col)) {
                    const u32 d = sh_ >= 32 ? (o[j] >> (sh_ - 32)) & (BT_BINS - 1)
                                            : (u32)(pack(o[j], col) >> sh_) & (BT_BINS - 1);
                    atomicAdd(&L.hist[d], 1u);
                }
            }
        }
        // lane l scans bins [16 l, 16 l + 16) and leaves them at zero
        constexpr int BPL = (int)BT_BINS / WAVE;
        uint4 *hp = reinterpret_cast<uint4 *>(&L.hist[lane * BPL]);
        u32 c[BPL], csum = 0;
#pragma unroll
        for (int q = 0; q < BPL / 4; ++q) {
            const uint4 v = hp[q];
            c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
            hp[q] = make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int q = 0; q < BPL; ++q) csum += c[q];
        const u32 incl = wave_incl_scan(csum);
        u32 before = incl - csum;
        const bool hit = before <= rk && rk < incl;
        u32 bin = 0, bcnt = 0, bbefore = 0;
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
            if (before <= rk && rk < before + c[q]) {
                bin = lane * BPL + (u32)q;
                bcnt = c[q];
                bbefore = before;
            }
            before += c[q];
        }
        const int hl = __builtin_ctzll(ballot(hit));
        bin = (u32)__builtin_amdgcn_readlane((int)bin, hl);
        cnt = (u32)__builtin_amdgcn_readlane((int)bcnt, hl);
        rk -= (u32)__builtin_amdgcn_readlane((int)bbefore, hl);
        const u64 bsel = (u64)bin << sh_;
        ph |= (u32)(bsel >> 32);
        pl |= (u32)bsel;
        lowb = sh_;
    }
    if (lowb == 0) return ((u64)ph << 32) | pl;     // every bit fixed: that pair
    // at most 64 candidates: compact them into L.cand (ballot order) and rank
    u32 base = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn) {
            const u32 col = (u32)j * WAVE + lane;
            const bool t = col < n && match(o[j], col);
            const u64 m = ballot(t);
            if (t) L.cand[base + mbcnt(m)] = pack(o[j], col);
            base += (u32)__popcll(m);
        }
    }
    const u64 mine = lane < cnt ? L.cand[lane] : ~0ull;
    const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
    u32 lt = 0;
    for (u32 i = 0; i < cnt; ++i) {
        const u64 x = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                      (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
        lt += x < mine ? 1u : 0u;
    }
    const int fl = __builtin_ctzll(ballot(lane < cnt && lt == rk));
    return ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, fl) << 32) |
           (u32)__builtin_amdgcn_readlane((int)mlo, fl);
}

// First try of the wave mode (a row of more than 64 keys): one histogram of
// BT_WAVE_LIN bins linear in the key value between the row's least and
// greatest key; if the bin holding rank `rank` has at most 64 pairs they are
// compacted and ranked.  Returns false, every bin left at zero, when the
// range allows no linear bins or the bin is larger.
constexpr u32 BT_WAVE_LIN = 256;
template <bool LARGEST, int M>
__device__ __forceinline__ bool bt_wave_lin(const u32 (&o)[M], u32 n, u32 rank, BtWaveLds &L, u64 &tau)
{
    const u32 lane = bt_tid() & (WAVE - 1);
    const u32 jn = (n + WAVE - 1) / WAVE;
    u32 mn = ~0u, mx = 0u;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn && (u32)j * WAVE + lane < n) {
            mn = o[j] < mn ? o[j] : mn;
            mx = o[j] > mx ? o[j] : mx;
        }
    }
    mn = bt_wave_ext_u32<false>(mn);
    mx = bt_wave_ext_u32<true>(mx);
    float scale, bias;
    if (!lin_setup<LARGEST, BT_WAVE_LIN>(mn, mx, scale, bias)) return false;
#pragma unroll
    for (int j = 0; j < M; ++j)
        if ((u32)j < jn && (u32)j * WAVE + lane < n)
            atomicAdd(&L.hist[lin_bin<LARGEST, BT_WAVE_LIN>(o[j], scale, bias)], 1u);
    // lane l scans bins [4 l, 4 l + 4) and leaves them at zero
    static_assert(BT_WAVE_LIN == 4 * WAVE, "four bins per lane");
    uint4 *hp = reinterpret_cast<uint4 *>(&L.hist[lane * 4]);
    const uint4 v = *hp;
    *hp = make_uint4(0u, 0u, 0u, 0u);
    const u32 c[4] = {v.x, v.y, v.z, v.w};
    const u32 csum = v.x + v.y + v.z + v.w;
    const u32 incl = wave_incl_scan(csum);
    u32 before = incl - csum;
    const bool hit = before <= rank && rank < incl;
    u32 bin = 0, bcnt = 0, bbefore = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (before <= rank && rank < before + c[q]) {
            bin = lane * 4 + (u32)q;
            bcnt = c[q];
            bbefore = before;
        }
        before += c[q];
    }
    const int hl = __builtin_ctzll(ballot(hit));
    const u32 b = (u32)__builtin_amdgcn_readlane((int)bin, hl);
    const u32 cnt = (u32)__builtin_amdgcn_readlane((int)bcnt, hl);
    const u32 rk = rank - (u32)__builtin_amdgcn_readlane((int)bbefore, hl);
    if (cnt > (u32)WAVE) return false;
    u32 base = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn) {
            const u32 col = (u32)j * WAVE + lane;
            const bool t = col < n && lin_bin<LARGEST, BT_WAVE_LIN>(o[j], scale, bias) == b;
            const u64 m = ballot(t);
            if (t) L.cand[base + mbcnt(m)] = pack(o[j], col);
            base += (u32)__popcll(m);
        }
    }
    const u64 mine = lane < cnt ? L.cand[lane] : ~0ull;
    const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
    u32 lt = 0;
    for (u32 i = 0; i < cnt; ++i) {
        const u64 x = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                      (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
        lt += x < mine ? 1u : 0u;
    }
    const int fl = __builtin_ctzll(ballot(lane < cnt && lt == rk));
    tau = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, fl) << 32) |
          (u32)__builtin_amdgcn_readlane((int)mlo, fl);
    return true;
}

// One row by one wave: load, select, write the columns up to the pair of
// rank k in column order (ballot compaction, no LDS), and the k-th pair.
template <bool LARGEST, int M>
__device__ __forceinline__ void bt_wave_row(const BtArgs &a, u32 r, const u32 *__restrict__ row, u32 len,
                                            u32 k, BtWaveLds &L)
{
    const u32 lane = bt_tid() & (WAVE - 1);
    const u32 jn = (len + WAVE - 1) / WAVE;
    u32 o[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const u32 col = (u32)j * WAVE + lane;
        o[j] = (u32)j < jn ? row[col < len ? col : len - 1] : 0u;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) o[j] = key_ord<true, LARGEST>(o[j]);
    u64 tau;
    if (len <= (u32)WAVE || !bt_wave_lin<LARGEST, M>(o, len, k - 1, L, tau))
        tau = bt_wave_select<M>(o, len, k - 1, L);
    const u32 th = (u32)(tau >> 32), tl = (u32)tau;
    u32 kbits = 0;
    if (lane == 0) kbits = row[tl];                 // in flight during the output
    u32 *__restrict__ out = a.out_idx + a.out_off[r];
    u32 pos = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if ((u32)j < jn) {
            const u32 col = (u32)j * WAVE + lane;
            const bool t = col < len && (o[j] < th || (o[j] == th && col <= tl));
            const u64 m = ballot(t);
            if (t) {
                const u32 q = pos + mbcnt(m);
                if (q < k) out[q] = col;
            }
            pos += (u32)__popcll(m);
        }
    }
    if (lane == 0) {
        a.kth_idx[r] = tl;
        a.kth_key[r] = kbits;
    }
}

// A row of the wave mode's range: solved if shorter than BT_WAVE_MAXLEN (a
// longer one of the shared class is the workgroup mode's).
template <bool LARGEST>
__device__ __forceinline__ void bt_wave_dispatch(const BtArgs &a, u32 r, BtWaveLds &L)
{
    const u64 off = a.row_off[r];
    const u64 len64 = a.row_off[r + 1] - off;
    if (len64 >= BT_WAVE_MAXLEN) return;
    const u32 k = a.k[r];
    const u32 cls = len_class(len64);
    if (cls < a.cls_lo || cls > a.cls_hi) return;
    if (k == 0 || (u64)k > len64) {
        if ((bt_tid() & (WAVE - 1)) == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_ROW);
        return;
    }
    const u32 len = (u32)len64;
    const u32 *__restrict__ row = a.keys + off;
    if (len <= 16 * WAVE) bt_wave_row<LARGEST, 16>(a, r, row, len, k, L);
    else if (len <= 32 * WAVE) bt_wave_row<LARGEST, 32>(a, r, row, len, k, L);
    else bt_wave_row<LARGEST, BT_WAVE_M>(a, r, row, len, k, L);
    static_assert(BT_WAVE_MAXLEN > 32 * WAVE && BT_WAVE_M % 16 == 0, "wave-mode sizes");
}

// Pivots from the sample by bins linear in the key value.  The sample pairs
// are each thread's (o[j], p[j]), j < cnt; the waves' least and greatest
// order words are in sh.wt[0][], sh.wt[1][] and both candidate counters are
// zero.  One histogram serves both target ranks; when each active target's
// bin holds at most 64 pairs, waves 0 and 1 rank them.  Returns false, every
// bin left at zero, if the range allows no linear bins or a bin is larger.
template <bool LARGEST>
__device__ __forceinline__ bool bt_pivots_lin(const u32 (&o)[BT_SEG], const u32 (&p)[BT_SEG], int cnt,
                                              const u64 rank[2], const bool act[2], u64 res[2], BtShared &sh)
{
    const u32 tid = bt_tid(), lane = tid & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    u32 omin = ~0u, omax = 0u;
#pragma unroll
    for (int v = 0; v < BT_WAVES; ++v) {
        const u32 a0 = __builtin_amdgcn_readfirstlane(sh.wt[0][v]);
        const u32 a1 = __builtin_amdgcn_readfirstlane(sh.wt[1][v]);
        omin = a0 < omin ? a0 : omin;
        omax = a1 > omax ? a1 : omax;
    }
    float scale, bias;
    if (!lin_setup<LARGEST>(omin, omax, scale, bias)) return false;
#pragma unroll
    for (int j = 0; j < BT_SEG; ++j)
        if (j < cnt) atomicAdd(&sh.hist[lin_bin<LARGEST>(o[j], scale, bias)], 1u);
    lds_sync();
    u32 c[BT_BPT], csum = 0;
#pragma unroll
    for (int q = 0; q < BT_BPT; ++q) {
        c[q] = sh.hist[tid * BT_BPT + q];
        sh.hist[tid * BT_BPT + q] = 0u;
        csum += c[q];
    }
    u32 tot;
    u32 before = block_excl_scan<BT_THREADS, true>(csum, sh.scan, &tot);
#pragma unroll
    for (int q = 0; q < BT_BPT; ++q) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (act[t] && (u64)before <= rank[t] && rank[t] < (u64)before + c[q]) {
                sh.sel_bin[t] = tid * BT_BPT + q;
                sh.sel_before[t] = before;
                sh.sel_count[t] = c[q];
            }
        }
        before += c[q];
    }
    lds_sync();
    u32 b[2] = {0u, 0u}, nb[2] = {0u, 0u}, rr[2] = {0u, 0u};
    bool big = false;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!act[t]) continue;
        b[t] = __builtin_amdgcn_readfirstlane(sh.sel_bin[t]);
        nb[t] = __builtin_amdgcn_readfirstlane(sh.sel_count[t]);
        rr[t] = (u32)rank[t] - __builtin_amdgcn_readfirstlane(sh.sel_before[t]);
        big = big || nb[t] > (u32)WAVE;
    }
    if (big) return false;
#pragma unroll
    for (int j = 0; j < BT_SEG; ++j) {
        if (j < cnt) {
            const u32 bn = lin_bin<LARGEST>(o[j], scale, bias);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                if (act[t] && bn == b[t]) sh.cand[t][atomicAdd(&sh.ccount[t], 1u)] = pack(o[j], p[j]);
        }
    }
    lds_sync();
    if (w < 2 && act[w]) {
        const u32 m = nb[w] , want = rr[w];
        const u64 mine = lane < m ? sh.cand[w][lane] : ~0ull;
        const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
        u32 lt = 0;
        for (u32 i = 0; i < m; ++i) {
            const u64 x = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                          (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
            lt += x < mine ? 1u : 0u;
        }
        if (lane < m && lt == want) sh.found[w] = mine;
    }
    lds_sync();
    res[0] = act[0] ? sh.found[0] : 0ull;
    res[1] = act[1] ? sh.found[1] : 0ull;
    return true;
}

template <bool LARGEST>
__device__ __forceinline__ void bt_row(const BtArgs &a, u32 r, BtShared &sh)
{
    const u32 tid = bt_tid();
    const u64 off = a.row_off[r];
    const u64 len64 = a.row_off[r + 1] - off;
    if (len64 < BT_WAVE_MAXLEN) return;          // the wave mode's row (shared class)
    const u32 k = a.k[r];
    const u32 cls = len_class(len64);
    if (cls < a.cls_lo || cls > a.cls_hi) return;
    if (k == 0 || (u64)k > len64 || len64 > 0xFFFFFFFFull) {
        if (tid == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_ROW);
        return;
    }
    const u32 len = (u32)len64;
    const u32 *__restrict__ row = a.keys + off;
    u32 *__restrict__ out = a.out_idx + a.out_off[r];
    auto gsrc = [&](u32 i) -> u64 { return pack(key_ord<true, LARGEST>(row[i]), i); };
    auto lsrc = [&](u32 i) -> u64 { return sh.buf[i]; };
    // fast sweep regions as slots: wave v's candidates at v * BT_REG + [0, count)
    auto ssrc = [&](u32 i) -> u64 {
        return (i & (BT_REG - 1)) < sh.wt[0][i / BT_REG] ? sh.buf[i] : ~0ull;
    };

    u32 na = 0, nb = len;
    u32 kbits = 0;                      // key bits of the pair of rank k (thread 0)
    bool in_lds = false, fast_done = false;
    u64 fast_tau = 0;
    int band_top = 64;                  // pairs in LDS agree at and above this bit
    bool reg_done = false;
    u64 reg_tau = 0;
    u32 reg_kbits = 0;
    if (len <= BT_REG_KEYS / 8) {
        reg_tau = bt_reg_row<LARGEST, BT_REG_KEYS / 8 / BT_THREADS>(row, len, k, out, reg_kbits, sh);
        reg_done = true;
    } else if (len <= BT_REG_KEYS / 2) {
        reg_tau = bt_reg_row<LARGEST, BT_REG_KEYS / 2 / BT_THREADS>(row, len, k, out, reg_kbits, sh);
        reg_done = true;
    } else if (len <= BT_REG_KEYS) {
        reg_tau = bt_reg_row<LARGEST, BT_REG_KEYS / BT_THREADS>(row, len, k, out, reg_kbits, sh);
        reg_done = true;
    } else {
        u32 c_num = a.c_cls[cls];
        const u32 s_target = a.s_cls[cls];
        bool fast_ok = a.fast != 0u;    // until a fast sweep overflows its region
        for (u32 att = 0; att < a.attempts && !in_lds && !fast_done; ++att) {
            // sample -> LDS (stratum q at slot q) and registers, with the
            // waves' least and greatest order words
            const u32 s = s_target < len ? s_target : len;
            u32 pos[BT_SEG], sk[BT_SEG];
            const int cnt = bt_sample(tid, len, s, a.seed, att, r, pos);
#pragma unroll
            for (int j = 0; j < BT_SEG; ++j)
                if (j < cnt) sk[j] = row[pos[j]];
            u32 mn = ~0u, mx = 0u;
#pragma unroll
            for (int j = 0; j < BT_SEG; ++j) {
                if (j < cnt) {
                    sk[j] = key_ord<true, LARGEST>(sk[j]);
                    sh.buf[(u32)j * BT_THREADS + tid] = pack(sk[j], pos[j]);
                    mn = sk[j] < mn ? sk[j] : mn;
                    mx = sk[j] > mx ? sk[j] : mx;
                }
            }
            mn = bt_wave_ext_u32<false>(mn);
            mx = bt_wave_ext_u32<true>(mx);
            {
                const u32 ln = tid & (WAVE - 1), wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
                if (ln == 0) {
                    sh.wt[0][wv] = mn;
                    sh.wt[1][wv] = mx;
                }
            }
            if (tid < 2) sh.ccount[tid] = 0u;
            lds_sync();
            i64 lo, hi;
            pivot_ranks(s, k, len, c_num, lo, hi);
            const bool hl = lo >= 0, hr = hi < (i64)s;
            u64 piv[2];
            {
                const u64 rk[2] = {hl ? (u64)lo : 0ull, hr ? (u64)hi : 0ull};
                const bool ac[2] = {hl, hr};
                if (!bt_pivots_lin<LARGEST>(sk, pos, cnt, rk, ac, piv, sh))
                    bt_select(lsrc, s, 64, rk, ac, piv, sh);
            }
            const u64 L = hl ? uniform64(piv[0]) : 0ull;
            const u64 R = hr ? uniform64(piv[1]) : ~0ull;
            const u32 oL = (u32)(L >> 32), oR = (u32)(R >> 32);
            if (fast_ok && hr && !ord_is_nan<LARGEST>(oR) && !(hl && ord_is_nan<LARGEST>(oL)) &&
                (u64)(hi + 1) * len * BT_FAST_DEN <= (u64)s * BT_FAST_NUM * BT_CAP) {
                // fast sweep: candidates (<= R) into per-wave regions of sh.buf
                const u32 wv = __builtin_amdgcn_readfirstlane(tid / WAVE), ln = tid & (WAVE - 1);
                lds_sync();
                u32 cw, aw;
                u64 *reg = sh.buf + wv * BT_REG;
                if (a.t_cls[cls] == 8)
                    bt_fast_sweep<LARGEST, 8>(row, len, hl ? ord_value<LARGEST>(oL) : 0.0f,
                                              ord_value<LARGEST>(oR), hl, reg, cw, aw);
                else
                    bt_fast_sweep<LARGEST, 16>(row, len, hl ? ord_value<LARGEST>(oL) : 0.0f,
                                               ord_value<LARGEST>(oR), hl, reg, cw, aw);
                // the wave's own region to (ord, column) pairs, in place
                for (u32 i = ln; i < cw && i < BT_REG; i += WAVE) {
                    const u64 e = reg[i];
                    reg[i] = pack(key_ord<true, LARGEST>((u32)(e >> 32)), (u32)e);
                }
                if (ln == 0) {
                    sh.wt[0][wv] = cw;
                    sh.wt[1][wv] = aw;
                }
                lds_sync();
                u32 n_ab = 0, n_a = 0, cnt[BT_WAVES];
                bool over = false;
#pragma unroll
                for (int v = 0; v < BT_WAVES; ++v) {
                    cnt[v] = __builtin_amdgcn_readfirstlane(sh.wt[0][v]);
                    over = over || cnt[v] > BT_REG;
                    n_ab += cnt[v];
                    n_a += __builtin_amdgcn_readfirstlane(sh.wt[1][v]);
                }
                if (!over) {
                    if (n_a >= k || n_ab < k) {
                        c_num *= 2;          // the pivots missed rank k: wider
                        continue;
                    }
                    fast_tau = bt_band_tau(ssrc, cnt, hl ? oL : 0u, oR, k - 1, sh);
                    fast_done = true;
                    break;
                }
                fast_ok = false;             // region overflow: the general sweep, same pivots
                lds_sync();             // (it rewrites sh.wt, read above)
            }
            // one sweep: below L -> output, [L, R] -> LDS band.  Wave w takes
            // keys [s0 + 1024 w, s0 + 1024 w + 1024) of a step as 16 columns of
            // 64 lanes (coalesced); lane bits keep its keys' parts; the waves'
            // counts are exchanged once per step.
            u32 ca = 0, cb = 0;
            {
                const u32 wv = __builtin_amdgcn_readfirstlane(tid / WAVE), ln = tid & (WAVE - 1);
                for (u32 s0 = 0, st = 0; s0 < len; s0 += BT_STEP, ++st) {
                    const u32 base = s0 + wv * (BT_STEP / BT_WAVES);
                    u32 o[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const u32 col = base + (u32)j * WAVE + ln;
                        o[j] = row[col < len ? col : len - 1];
                    }
                    u32 abits = 0, bbits = 0, ta = 0, tb = 0;
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const u32 col = base + (u32)j * WAVE + ln;
                        o[j] = key_ord<true, LARGEST>(o[j]);
                        const u64 c = pack(o[j], col);
                        const bool ok = col < len;
                        const bool ia = ok && hl && c < L;
                        const bool ib = ok && !(hl && c < L) && !(hr && c > R);
                        abits |= (u32)ia << j;
                        bbits |= (u32)ib << j;
                        ta += (u32)__popcll(ballot(ia));
                        tb += (u32)__popcll(ballot(ib));
                        asm volatile("" : "+s"(ta), "+s"(tb));   // keep the sums current
                    }
                    const u32 par = st & 1u;
                    if (ln == 0) sh.wt[par][wv] = ta | (tb << 16);
                    lds_sync();
                    u32 pa = ca, pb = cb, sa = 0, sb = 0;
#pragma unroll
                    for (int v = 0; v < BT_WAVES; ++v) {
                        const u32 x = sh.wt[par][v];
                        if ((u32)v < wv) { pa += x & 0xFFFFu; pb += x >> 16; }
                        sa += x & 0xFFFFu;
                        sb += x >> 16;
                    }
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const u32 col = base + (u32)j * WAVE + ln;
                        const bool ia = (abits >> j) & 1u, ib = (bbits >> j) & 1u;
                        const u64 ma = ballot(ia), mb = ballot(ib);
                        if (ma) {
                            const u32 q = pa + mbcnt(ma);
                            if (ia && q < k) out[q] = col;
                            pa += (u32)__popcll(ma);
                        }
                        if (mb) {
                            const u32 q = pb + mbcnt(mb);
                            if (ib && q < BT_CAP) sh.buf[q] = pack(o[j], col);
                            pb += (u32)__popcll(mb);
                        }
                    }
                    ca += sa;
                    cb += sb;
                }
            }
            lds_sync();
            if (ca >= k || ca + cb < k || cb > BT_CAP) {
                // The attempt is discarded, and the part below L it wrote to
                // out[] will be written again by another attempt or by the
                // exact fallback, possibly by other waves: a barrier that
                // orders global memory too (not only LDS) puts every earlier
                // store before the later ones.  The branch is uniform.
                __syncthreads();
                if (cb > BT_CAP && !(ca >= k || ca + cb < k))
                    c_num = c_num > 1 ? c_num / 2 : 1;   // band too wide for LDS: narrower
                else
                    c_num *= 2;                  // the pivots missed rank k: wider
            } else {
                na = ca;
                nb = cb;
                in_lds = true;
                // every band pair lies in [L, R]: they agree above the highest
                // bit in which L and R differ
                if (hl && hr) band_top = (L == R) ? 0 : 64 - __clzll((long long)(L ^ R));
            }
        }
    }
    u64 tau;
    const bool one[2] = {true, false};
    u64 t2[2];
    // the key of the pair of rank k is loaded before the output is written,
    // so that its latency overlaps the writes
    if (reg_done) {
        tau = reg_tau;
        kbits = reg_kbits;
    } else if (fast_done) {
        tau = fast_tau;
        if (tid == 0) kbits = row[(u32)tau];
        bt_emit_regions(tau, out, k, sh);       // sh.wt[0] still holds the counts
    } else if (in_lds) {
        const u64 rk[2] = {(u64)(k - na - 1), 0ull};
        bt_select(lsrc, nb, band_top, rk, one, t2, sh);
        tau = t2[0];
        if (tid == 0) kbits = row[(u32)tau];
        bt_emit(lsrc, nb, tau, out + na, k - na, sh);
    } else {
        // exact fallback over the row
        const u64 rk[2] = {(u64)(k - 1), 0ull};
        bt_select(gsrc, len, 64, rk, one, t2, sh);
        tau = t2[0];
        if (tid == 0) kbits = row[(u32)tau];
        bt_emit(gsrc, len, tau, out, k, sh);
    }
    if (tid == 0) {
        a.kth_idx[r] = (u32)tau;
        a.kth_key[r] = kbits;
    }
    lds_sync();
}

template <bool LARGEST>
__global__ __launch_bounds__(BT_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_batched(BtArgs a)
{
    __shared__ BtShared sh;
    for (u32 i = threadIdx.x; i < BT_BINS; i += BT_THREADS) sh.hist[i] = 0u;
    lds_sync();
    // order positions [0, n_wg): the classes with workgroup rows (longer
    // than BT_WAVE_MAXLEN); [n_wv0, rows): the classes with wave rows.  The
    // class of BT_WAVE_MAXLEN is in both ranges, and each mode skips the
    // other's rows in it.
    if (threadIdx.x == 0) {
        u32 above = 0;
        for (u32 c = BT_WAVE_CLS + 1; c < (u32)BT_NCLS; ++c) above += a.cls_cnt[c];
        sh.n_wg = above + a.cls_cnt[BT_WAVE_CLS];
        sh.next = above;
    }
    lds_sync();
    const u32 n_wg = __builtin_amdgcn_readfirstlane(sh.n_wg);
    const u32 n_wv0 = __builtin_amdgcn_readfirstlane(sh.next);
    // Workgroup mode: those rows, longest first, from BT_NQ queues, one per
    // XCD (workgroup b is dispatched to XCD b % BT_NQ): queue x hands out the
    // positions x, x + BT_NQ, ... of [0, n_wg), one per grab for the first
    // BT_Q1 of them (the long rows), then BT_QCHUNK per grab.  A grab is a
    // global atomic on the queue's own counter; atomics on one address are
    // serialised, so the workgroups of an XCD use only their own queue (a
    // grid smaller than BT_NQ serves every queue: x = b, b + grid, ...).
    const u32 q_first = blockIdx.x % BT_NQ;
    const u32 q_step = gridDim.x < BT_NQ ? gridDim.x : BT_NQ;
    for (u32 x = q_first; x < BT_NQ; x += q_step) {
        const u32 nx = n_wg > x ? (n_wg - x + BT_NQ - 1) / BT_NQ : 0u;
        u32 *qc = a.queue + x * BT_QSTRIDE;
        while (nx) {
            if (threadIdx.x == 0) sh.next = atomicAdd(qc, 1u);
            lds_sync();
            const u32 g = __builtin_amdgcn_readfirstlane(sh.next);
            lds_sync();
            const u32 q0 = g < BT_Q1 ? g : BT_Q1 + (g - BT_Q1) * BT_QCHUNK;
            if (q0 >= nx) break;
            const u32 q1 = g < BT_Q1 ? q0 + 1 : (q0 + BT_QCHUNK < nx ? q0 + BT_QCHUNK : nx);
            for (u32 q = q0; q < q1; ++q) bt_row<LARGEST>(a, a.order[q * BT_NQ + x], sh);
        }
    }
    // Wave mode: positions [n_wv0, rows), one row per wave, BT_WQCHUNK rows
    // per grab from the second set of queues (the same queue choice).  No
    // workgroup barrier follows: the waves leave independently.
    const u32 lane = bt_tid() & (WAVE - 1);
    const u32 w = __builtin_amdgcn_readfirstlane(bt_tid() / WAVE);
    BtWaveLds &L = reinterpret_cast<BtWaveLds *>(sh.buf)[w];
    {
        uint4 *hp = reinterpret_cast<uint4 *>(L.hist);
        for (u32 i = lane; i < BT_BINS / 4; i += WAVE) hp[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    const u32 n_wv = a.rows - n_wv0;
    for (u32 x = q_first; x < BT_NQ; x += q_step) {
        const u32 nx = n_wv > x ? (n_wv - x + BT_NQ - 1) / BT_NQ : 0u;
        u32 *qc = a.queue + (BT_NQ + x) * BT_QSTRIDE;
        while (nx) {
            u32 g = 0;
            if (lane == 0) g = atomicAdd(qc, BT_WQCHUNK);
            g = __builtin_amdgcn_readfirstlane(g);
            if (g >= nx) break;
            const u32 g1 = g + BT_WQCHUNK < nx ? g + BT_WQCHUNK : nx;
            for (u32 q = g; q < g1; ++q) bt_wave_dispatch<LARGEST>(a, a.order[n_wv0 + q * BT_NQ + x], L);
        }
    }
}

// Zero the class counters and the status word (a kernel, so the call can be
// captured in a graph without memset nodes).
__global__ void k_bt_init(BtArgs a)
{
    const u32 t = threadIdx.x;
    if (t < BT_NCLS) {
        a.cls_cnt[t] = 0u;
        a.cls_fill[t] = 0u;
    }
    if (t < 2 * BT_NQ) a.queue[t * BT_QSTRIDE] = 0u;
    if (t == 0) *a.status = 0u;
}

// Rows per length class (workgroup histogram, one global add per class).
__global__ __launch_bounds__(BT_HIST_THREADS) void k_bt_hist(BtArgs a)
{
    __shared__ u32 h[BT_NCLS];
    const u32 t = threadIdx.x, r = blockIdx.x * BT_HIST_THREADS + t;
    if (t < BT_NCLS) h[t] = 0u;
    __syncthreads();
    if (r < a.rows) atomicAdd(&h[len_class(a.row_off[r + 1] - a.row_off[r])], 1u);
    __syncthreads();
    if (t < BT_NCLS && h[t]) atomicAdd(&a.cls_cnt[t], h[t]);
}

// order[]: rows by decreasing length class (a counting sort; rows of one class
// in no particular order).
__global__ __launch_bounds__(BT_HIST_THREADS) void k_bt_order(BtArgs a)
{
    __shared__ u32 h[BT_NCLS], base[BT_NCLS];
    const u32 t = threadIdx.x, r = blockIdx.x * BT_HIST_THREADS + t;
    if (t < BT_NCLS) h[t] = 0u;
    __syncthreads();
    u32 cls = 0, local = 0;
    if (r < a.rows) {
        cls = len_class(a.row_off[r + 1] - a.row_off[r]);
        local = atomicAdd(&h[cls], 1u);
    }
    __syncthreads();
    if (t < BT_NCLS) {
        // classes above t come first
        u32 start = 0;
        for (int c = BT_NCLS - 1; c > (int)t; --c) start += a.cls_cnt[c];
        base[t] = h[t] ? start + atomicAdd(&a.cls_fill[t], h[t]) : 0u;
    }
    __syncthreads();
    if (r < a.rows) a.order[base[cls] + local] = r;
}

}  // namespace topk

using namespace topk;

namespace {

constexpr size_t BT_ALIGN = 256;
inline size_t bt_align(size_t x) { return (x + BT_ALIGN - 1) / BT_ALIGN * BT_ALIGN; }

struct BtLayout {
    size_t cnt, fill, queue, order, total;
};

BtLayout bt_layout(uint32_t rows)
{
    BtLayout L{};
    size_t off = 0;
    L.cnt = off;
    off = bt_align(off + BT_NCLS * sizeof(uint32_t));
    L.fill = off;
    off = bt_align(off + BT_NCLS * sizeof(uint32_t));
    L.queue = off;
    off = bt_align(off + (size_t)2 * BT_NQ * BT_QSTRIDE * sizeof(uint32_t));
    L.order = off;
    off = bt_align(off + (size_t)rows * sizeof(uint32_t));
    L.total = off;
    return L;
}

// ---- Scratch of topk_select_batched_f32_noalloc ----------------------------
// The same layout as a caller's workspace, for at most BT_NOALLOC_MAX_ROWS
// rows, in a file-scope device array that every call on a device shares.
constexpr uint32_t BT_NOALLOC_MAX_ROWS = 1u << 20;
constexpr size_t BT_NOALLOC_BYTES =
    2 * BT_ALIGN + (size_t)2 * BT_NQ * BT_QSTRIDE * sizeof(uint32_t) +
    (((size_t)BT_NOALLOC_MAX_ROWS * sizeof(uint32_t) + BT_ALIGN - 1) / BT_ALIGN) * BT_ALIGN;

}  // namespace

static __device__ __align__(256) unsigned char scratch[BT_NOALLOC_BYTES];

namespace {

constexpr int BT_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[BT_MAX_DEVICES];    // device address of `scratch` on each device

hipError_t bt_enqueue(const BtArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_bt_init, dim3(1), dim3(64), 0, s, a);
    const u32 hb = (a.rows + BT_HIST_THREADS - 1) / BT_HIST_THREADS;
    hipLaunchKernelGGL(k_bt_hist, dim3(hb), dim3(BT_HIST_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_bt_order, dim3(hb), dim3(BT_HIST_THREADS), 0, s, a);
    if (a.flags & TOPK_LARGEST)
        hipLaunchKernelGGL((k_batched<true>), dim3(grid), dim3(BT_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_batched<false>), dim3(grid), dim3(BT_THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// Look up the device address of `scratch` on `device` (once per device; the
// host-side name of the array is not a device address).  Called by
// topk_create; makes `device` current while it runs and restores the caller's.
int topk_bt_scratch_setup(int device)
{
    static_assert(BT_NOALLOC_BYTES >= 2 * BT_ALIGN + 2 * BT_NQ * BT_QSTRIDE * sizeof(uint32_t) +
                                          BT_NOALLOC_MAX_ROWS * sizeof(uint32_t),
                  "scratch holds the workspace layout of the largest batch");
    if (device < 0 || device >= BT_MAX_DEVICES) return TOPK_E_INVALID;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return TOPK_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return TOPK_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return TOPK_E_HIP;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr) return TOPK_E_HIP;
    if (bt_layout(BT_NOALLOC_MAX_ROWS).total > BT_NOALLOC_BYTES) return TOPK_E_HIP;
    g_scratch_ptr[device] = ptr;
    return TOPK_OK;
}

extern "C" size_t topk_batched_workspace_bytes(const topk_ctx *ctx, uint32_t rows, uint32_t flags)
{
    (void)flags;
    if (!ctx) return 0;
    return bt_layout(rows).total;
}

namespace {

// Kernel arguments of one batched call (after the argument checks).
int bt_args(const topk_ctx *c, const float *keys, const uint64_t *row_off, uint32_t rows,
            const uint32_t *k, const uint64_t *out_off, uint32_t flags, uint32_t *out_idx,
            float *kth_key, uint32_t *kth_idx, uint32_t *status, void *workspace,
            size_t ws_bytes, BtArgs &a)
{
    if (!c || !keys || !row_off || !k || !out_off || !out_idx || !kth_key || !kth_idx ||
        !status || !workspace)
        return TOPK_E_INVALID;
    if (rows == 0) return TOPK_E_INVALID;
    if (flags & ~(uint32_t)(TOPK_LARGEST | TOPK_GRAPH)) return TOPK_E_INVALID;
    if (((uintptr_t)keys & 3u) || ((uintptr_t)row_off & 7u) || ((uintptr_t)out_off & 7u) ||
        ((uintptr_t)workspace & (BT_ALIGN - 1)))
        return TOPK_E_INVALID;
    const BtLayout L = bt_layout(rows);
    if (ws_bytes < L.total) return TOPK_E_WORKSPACE;
    char *w = (char *)workspace;
    a = BtArgs{};
    a.keys = (const u32 *)keys;
    a.row_off = (const u64 *)row_off;
    a.k = k;
    a.out_off = (const u64 *)out_off;
    a.rows = rows;
    a.flags = flags & TOPK_LARGEST;
    a.out_idx = out_idx;
    a.kth_key = (u32 *)kth_key;
    a.kth_idx = kth_idx;
    a.status = status;
    a.cls_cnt = (u32 *)(w + L.cnt);
    a.cls_fill = (u32 *)(w + L.fill);
    a.order = (u32 *)(w + L.order);
    a.queue = (u32 *)(w + L.queue);
    a.seed = c->seed;
    a.attempts = (u32)c->bt_attempts;
    a.fast = (u32)c->bt_fast;
    a.cls_lo = 0;
    a.cls_hi = BT_NCLS - 1;
    for (int i = 0; i < BT_NCLS; ++i) {
        a.s_cls[i] = (u32)(c->bt_s_cls[i] >= 0 ? c->bt_s_cls[i] : c->bt_s_target);
        a.c_cls[i] = (u32)(c->bt_c_cls[i] >= 0 ? c->bt_c_cls[i] : c->bt_c_num);
        a.t_cls[i] = (u32)(c->bt_t_cls[i] >= 0 ? c->bt_t_cls[i] : c->bt_tile);
    }
    return TOPK_OK;
}

int bt_run(topk_ctx *c, const BtArgs &a, bool graph, hipStream_t stream)
{
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    const int grid = (int)(c->num_cu * c->bt_wg_per_cu);   // 4 fit on a CU (LDS, registers)
    if (!graph) return bt_enqueue(a, grid, stream) == hipSuccess ? TOPK_OK : TOPK_E_HIP;

    // one graph per distinct argument set: captured once, then replayed
    std::vector<uint64_t> key = {
        (uint64_t)(uintptr_t)a.keys, (uint64_t)(uintptr_t)a.row_off, a.rows,
        (uint64_t)(uintptr_t)a.k, (uint64_t)(uintptr_t)a.out_off, a.flags,
        (uint64_t)(uintptr_t)a.out_idx, (uint64_t)(uintptr_t)a.kth_key,
        (uint64_t)(uintptr_t)a.kth_idx, (uint64_t)(uintptr_t)a.status,
        (uint64_t)(uintptr_t)a.order, a.seed, a.attempts, a.fast, a.cls_lo, a.cls_hi,
        (uint64_t)grid};
    for (int i = 0; i < BT_NCLS; ++i)
        key.push_back(((uint64_t)a.s_cls[i] << 32) | ((uint64_t)a.t_cls[i] << 24) | a.c_cls[i]);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (!c->capture_stream &&
            hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return TOPK_E_HIP;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return TOPK_E_HIP;
        const hipError_t e1 = bt_enqueue(a, grid, c->capture_stream);
        const hipError_t e2 = hipStreamEndCapture(c->capture_stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return TOPK_E_HIP;
        }
        const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return TOPK_E_HIP;
        if (c->graphs.size() >= BT_GRAPHS_MAX) {
            // evict one cached graph; its launches may still run on any
            // stream, so the device is drained first (rare: only after
            // BT_GRAPHS_MAX distinct argument sets)
            if (hipDeviceSynchronize() != hipSuccess) {
                (void)hipGraphExecDestroy(ge);
                return TOPK_E_HIP;
            }
            (void)hipGraphExecDestroy(c->graphs.begin()->second);
            c->graphs.erase(c->graphs.begin());
        }
        it = c->graphs.emplace(key, ge).first;
    }
    return hipGraphLaunch(it->second, stream) == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}

// Mean of `reps` timed eager calls of the batch (ms), or a negative error.
float bt_time(topk_ctx *c, const BtArgs &a, uint32_t reps, hipStream_t stream, hipEvent_t e0,
              hipEvent_t e1)
{
    std::vector<float> t;
    for (uint32_t i = 0; i < reps; ++i) {
        if (hipEventRecord(e0, stream) != hipSuccess) return -1.0f;
        if (bt_run(c, a, false, stream) != TOPK_OK) return -1.0f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return -1.0f;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
        t.push_back(ms);
    }
    float mean = 0.0f;                  // the mean: repeated attempts count
    for (float x : t) mean += x;
    return mean / (float)t.size();
}

}  // namespace

extern "C" int topk_select_batched_f32(topk_ctx *c, const float *keys, const uint64_t *row_off,
                                       uint32_t rows, const uint32_t *k, const uint64_t *out_off,
                                       uint32_t flags, uint32_t *out_idx, float *kth_key,
                                       uint32_t *kth_idx, uint32_t *status, void *workspace,
                                       size_t ws_bytes, hipStream_t stream)
{
    BtArgs a;
    const int rc = bt_args(c, keys, row_off, rows, k, out_off, flags, out_idx, kth_key, kth_idx,
                           status, workspace, ws_bytes, a);
    if (rc != TOPK_OK) return rc;
    return bt_run(c, a, (flags & TOPK_GRAPH) != 0, stream);
}

extern "C" int topk_tune_batched_f32(topk_ctx *c, const float *keys, const uint64_t *row_off,
                                     uint32_t rows, const uint32_t *k, const uint64_t *out_off,
                                     uint32_t flags, uint32_t *out_idx, float *kth_key,
                                     uint32_t *kth_idx, uint32_t *status, void *workspace,
                                     size_t ws_bytes, uint32_t reps, hipStream_t stream)
{
    BtArgs a;
    int rc = bt_args(c, keys, row_off, rows, k, out_off, flags & ~(uint32_t)TOPK_GRAPH, out_idx,
                     kth_key, kth_idx, status, workspace, ws_bytes, a);
    if (rc != TOPK_OK) return rc;
    if (reps == 0 || reps > 100) return TOPK_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    // rows per length class, from the row offsets
    std::vector<uint64_t> off(rows + 1);
    if (hipStreamSynchronize(stream) != hipSuccess ||
        hipMemcpy(off.data(), row_off, off.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return TOPK_E_HIP;
    std::vector<uint32_t> per(BT_NCLS, 0);
    for (uint32_t r = 0; r < rows; ++r) {
        const uint64_t len = off[r + 1] - off[r];
        const uint32_t cls = len == 0 ? 0u : 64u - (uint32_t)__builtin_clzll(len);
        ++per[cls < (uint32_t)BT_NCLS ? cls : BT_NCLS - 1];
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TOPK_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return TOPK_E_HIP; }
    const int64_t s_cand[] = {256, 512, 1024, 2048};
    const int64_t c_cand[] = {8, 12, 16, 24};
    // classes holding rows of the sampling path (longer than BT_REG_KEYS)
    const uint32_t first = 64u - (uint32_t)__builtin_clzll((uint64_t)BT_REG_KEYS);
    for (uint32_t cls = first; cls < (uint32_t)BT_NCLS && rc == TOPK_OK; ++cls) {
        if (!per[cls]) continue;
        float best = -1.0f;
        int64_t bs = c->bt_s_target, bc = c->bt_c_num;
        for (int64_t sv : s_cand) {
            for (int64_t cv : c_cand) {
                BtArgs t = a;
                t.cls_lo = t.cls_hi = cls;
                t.s_cls[cls] = (u32)sv;
                t.c_cls[cls] = (u32)cv;
                const float ms = bt_time(c, t, reps, stream, e0, e1);
                if (ms < 0.0f) { rc = TOPK_E_HIP; break; }
                if (best < 0.0f || ms < best) { best = ms; bs = sv; bc = cv; }
            }
            if (rc != TOPK_OK) break;
        }
        c->bt_s_cls[cls] = bs;
        c->bt_c_cls[cls] = bc;
        a.s_cls[cls] = (u32)bs;
        a.c_cls[cls] = (u32)bc;
        if (rc != TOPK_OK) break;
        // then the fast sweep's tile under that pair
        int64_t bt = a.t_cls[cls];
        best = -1.0f;
        for (int64_t tv : {8, 16}) {
            BtArgs t = a;
            t.cls_lo = t.cls_hi = cls;
            t.t_cls[cls] = (u32)tv;
            const float ms = bt_time(c, t, reps, stream, e0, e1);
            if (ms < 0.0f) { rc = TOPK_E_HIP; break; }
            if (best < 0.0f || ms < best) { best = ms; bt = tv; }
        }
        c->bt_t_cls[cls] = bt;
        a.t_cls[cls] = (u32)bt;
    }
    // the sampling attempts before the exact fallback, over the whole batch
    if (rc == TOPK_OK) {
        float best = -1.0f;
        int64_t ba = c->bt_attempts;
        for (int64_t av : {1, 2, 4, 8}) {
            BtArgs t = a;
            t.attempts = (u32)av;
            const float ms = bt_time(c, t, reps, stream, e0, e1);
            if (ms < 0.0f) { rc = TOPK_E_HIP; break; }
            if (best < 0.0f || ms < best) { best = ms; ba = av; }
        }
        if (rc == TOPK_OK) {
            c->bt_attempts = ba;
            a.attempts = (u32)ba;
        }
    }
    // then the resident workgroups per CU over the whole batch
    if (rc == TOPK_OK) {
        const int64_t keep = c->bt_wg_per_cu;
        float best = -1.0f;
        int64_t bw = keep;
        for (int64_t wv = 2; wv <= 4; ++wv) {
            c->bt_wg_per_cu = wv;
            const float ms = bt_time(c, a, reps, stream, e0, e1);
            if (ms < 0.0f) { rc = TOPK_E_HIP; break; }
            if (best < 0.0f || ms < best) { best = ms; bw = wv; }
        }
        c->bt_wg_per_cu = rc == TOPK_OK ? bw : keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

extern "C" int topk_select_batched_f32_noalloc(topk_ctx *c, const float *keys,
                                               const uint64_t *row_off, uint32_t rows,
                                               const uint32_t *k, const uint64_t *out_off,
                                               uint32_t flags, uint32_t *out_idx, float *kth_key,
                                               uint32_t *kth_idx, uint32_t *status,
                                               hipStream_t stream)
{
    if (!c) return TOPK_E_INVALID;
    if (flags & ~(uint32_t)TOPK_LARGEST) return TOPK_E_INVALID;   // no graph capture here
    if (rows > BT_NOALLOC_MAX_ROWS) return TOPK_E_WORKSPACE;
    if (c->device < 0 || c->device >= BT_MAX_DEVICES) return TOPK_E_INVALID;
    void *ptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ptr = g_scratch_ptr[c->device];
    }
    if (!ptr) return TOPK_E_HIP;                // topk_create sets it up
    BtArgs a;
    const int rc = bt_args(c, keys, row_off, rows, k, out_off, flags, out_idx, kth_key, kth_idx,
                           status, ptr, BT_NOALLOC_BYTES, a);
    if (rc != TOPK_OK) return rc;
    return bt_run(c, a, false, stream);
}
