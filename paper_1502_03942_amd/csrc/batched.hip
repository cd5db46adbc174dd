// Batched selection: many rows of uneven length, each with its own k, in one
// persistent launch (§1: many similar selections solved together).
//
// Rows are ordered longest first (a counting sort by floor(log2 len)) and
// handed out from a queue to a persistent grid of 256-thread workgroups: one
// row per grab for the long rows, 16 per grab afterwards.  One workgroup solves a row by the sampling method of §2
// with the workgroup as the machine:
//   - a row of at most BT_CAP keys is the base case: its (ord, column) pairs go
//     to LDS and the pair of rank k is found exactly;
//   - a longer row draws a Bernoulli sample of about bt_s_target keys
//     (geometric skips, one segment per thread), takes the pivots at sample
//     ranks k s / len -/+ Delta, and sweeps the row once: the part below the
//     lower pivot goes straight to the output (in column order), the band
//     between the pivots to LDS.  If the band brackets rank k and fits, the
//     band is finished like a short row.  Otherwise the round is repeated with
//     a new sample (spread doubled after a miss, halved after an overflow) and
//     after bt_attempts rounds an exact radix select over the row finishes it.
// Every decision compares the composite key (ord, column), the unique order
// of §2, so the selected set is exactly the oracle's.
//
// Output per row: out_idx[out_off[r] .. + k) holds the selected columns: those
// below the lower pivot in column order, then the rest in column order (a row
// finished directly or by the exact fallback: all in column order);
// kth_key[r] / kth_idx[r] the pair of rank k (key bits as stored).
#include <hip/hip_runtime.h>
#include <string.h>

#include <vector>

#include "common.hpp"
#include "ctx.hpp"
#include "../../include/topk.h"

namespace topk {

constexpr int BT_THREADS = 256;                 // 4 waves
constexpr int BT_WAVES = BT_THREADS / WAVE;
constexpr u32 BT_CAP = 4096;                    // pairs in LDS: a short row or a band
constexpr int BT_BITS = 10;                     // radix digit
constexpr u32 BT_BINS = 1u << BT_BITS;
constexpr int BT_BPT = (int)BT_BINS / BT_THREADS;   // histogram bins per thread in the scan
constexpr int BT_SEG = 8;                       // sample slots per thread
constexpr int BT_IPT = 16;                      // keys per thread per sweep step
constexpr u32 BT_STEP = BT_THREADS * BT_IPT;
constexpr int BT_NCLS = 34;                     // length classes 0 (empty) .. 33
constexpr int BT_HIST_THREADS = 1024;
constexpr u32 BT_Q1 = 4096;                     // queue: rows taken one at a time first
constexpr u32 BT_QCHUNK = 16;                   // then this many per grab

struct BtShared {
    u64 buf[BT_CAP];
    u32 hist[BT_BINS];          // two targets' counts packed (low / high 16 bits)
    u64 cand[2][WAVE];
    u64 rmin[2], rmax[2], found[2];
    u32 ccount[2], sel_bin[2], sel_before[2], sel_count[2];
    u32 scan[BT_WAVES];
    u32 wt[2][BT_WAVES];        // sweep: per-wave (|a| | |b| << 16) of a step, by step parity
    u32 next;                   // next row position handed to this workgroup
};

struct BtArgs {
    const u32 *keys;
    const u64 *row_off;
    const u32 *k;
    const u64 *out_off;
    u32 rows, flags;
    u32 *out_idx, *kth_key, *kth_idx, *status;
    u32 *cls_cnt, *cls_fill, *order, *queue;
    u64 seed;
    u32 s_target, c_num, attempts;
};

__device__ __forceinline__ u32 len_class(u64 len)
{
    const u32 c = len == 0 ? 0u : 64u - (u32)__clzll((long long)len);
    return c < (u32)BT_NCLS ? c : (u32)BT_NCLS - 1;
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
    const u32 tid = threadIdx.x, lane = lane_id();
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const bool packed = n < 65536u;
    u64 pref[2] = {0ull, 0ull};
    int lowb[2] = {top, top};           // bits [lowb, 64) of the candidates equal pref's
    u64 rank[2] = {rank_in[0], rank_in[1]};
    bool done[2] = {!act[0], !act[1]};
    res[0] = res[1] = 0ull;
    for (u32 i = tid; i < BT_BINS; i += BT_THREADS) sh.hist[i] = 0u;
    if (tid < 2) sh.ccount[tid] = 0u;
    if (top >= 64) {
        // pref's bits at or above `top` are those of any pair
        const u64 x0 = n ? src(0) : 0ull;
        pref[0] = pref[1] = x0;
    } else {
        const u64 x0 = n ? src(0) : 0ull;
        pref[0] = pref[1] = top <= 0 ? x0 : (x0 >> top) << top;
    }
    __syncthreads();
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
        __syncthreads();
        // (2) scan: thread t covers bins [BT_BPT t, BT_BPT t + BT_BPT)
        u32 c[BT_BPT], csum = 0;
#pragma unroll
        for (int q = 0; q < BT_BPT; ++q) {
            c[q] = sh.hist[tid * BT_BPT + q];
            sh.hist[tid * BT_BPT + q] = 0u;      // clean for the next pass
            csum += c[q];
        }
        u32 tot;
        u32 before = block_excl_scan<BT_THREADS>(csum, sh.scan, &tot);
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
        __syncthreads();
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
            __syncthreads();
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
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (!gather[t]) continue;
                res[t] = sh.found[t];
                done[t] = true;
            }
            if (tid < 2) sh.ccount[tid] = 0u;
            __syncthreads();
        }
    }
}

// Write the columns of the pairs <= tau among src(0 .. n-1), in source order,
// to out[0 ..) (at most `limit`).  Thread t takes runs of BT_IPT consecutive
// pairs of each step, so source order is thread order within a step.
template <class SRC>
__device__ void bt_emit(SRC src, u32 n, u64 tau, u32 *out, u32 limit, BtShared &sh)
{
    const u32 tid = threadIdx.x;
    u32 cur = 0;
    for (u32 s0 = 0; s0 < n; s0 += BT_STEP) {
        u64 v[BT_IPT];
        u32 c = 0;
#pragma unroll
        for (int j = 0; j < BT_IPT; ++j) {
            const u32 i = s0 + tid * BT_IPT + (u32)j;
            v[j] = i < n ? src(i) : ~0ull;
            c += (i < n && v[j] <= tau) ? 1u : 0u;
        }
        u32 tot;
        u32 pos = cur + block_excl_scan<BT_THREADS>(c, sh.scan, &tot);
#pragma unroll
        for (int j = 0; j < BT_IPT; ++j) {
            const u32 i = s0 + tid * BT_IPT + (u32)j;
            if (i < n && v[j] <= tau) {
                if (pos < limit) out[pos] = (u32)v[j];
                ++pos;
            }
        }
        cur += tot;
    }
}

// Geometric-skip Bernoulli sample of a row (rate s_target / len): thread t
// samples its segment [t L, min(t L + L, len)), L = ceil(len / 256), with
// skips 1 + floor(ln U / ln(1 - rho)), U from Philox4x32-10 at counter
// (j / 4, t, tag, row), key = seed; at most BT_SEG per segment.  The skips of
// a segment are independent, so they are evaluated together (fp32: the
// sample only guides the pivots) and summed.
__device__ __forceinline__ int bt_sample(u32 t, u64 len, u32 s_target, u64 seed, u32 tag,
                                         u32 row, u32 (&pos)[BT_SEG])
{
    const float rho = (float)s_target / (float)len;
    const u64 L = (len + BT_THREADS - 1) / BT_THREADS;
    const u64 s0 = (u64)t * L;
    const u64 e0 = s0 + L < len ? s0 + L : len;
    if (s0 >= e0) return 0;
    const float inv = 1.0f / log1pf(-rho);
    u32 w[BT_SEG];
#pragma unroll
    for (int j = 0; j < BT_SEG; j += 4) {
        const uint4 r4 = philox4x32_10(make_uint4((u32)(j >> 2), t, tag, row), (u32)seed, (u32)(seed >> 32));
        w[j] = r4.x; w[j + 1] = r4.y; w[j + 2] = r4.z; w[j + 3] = r4.w;
    }
    u64 p = s0 - 1;
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < BT_SEG; ++j) {
        const float u = ((float)(w[j] >> 8) + 0.5f) * (1.0f / 16777216.0f);
        const float q = __logf(u) * inv;
        const u64 skip = q >= (float)L ? L + 1 : 1 + (u64)q;
        p += skip;
        if (p < e0) { pos[j] = (u32)p; cnt = j + 1; }
    }
    return cnt;
}

template <bool LARGEST>
__device__ void bt_row(const BtArgs &a, u32 r, BtShared &sh)
{
    const u32 tid = threadIdx.x;
    const u64 off = a.row_off[r];
    const u64 len64 = a.row_off[r + 1] - off;
    const u32 k = a.k[r];
    if (k == 0 || (u64)k > len64 || len64 > 0xFFFFFFFFull) {
        if (tid == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_ROW);
        return;
    }
    const u32 len = (u32)len64;
    const u32 *__restrict__ row = a.keys + off;
    u32 *__restrict__ out = a.out_idx + a.out_off[r];
    auto gsrc = [&](u32 i) -> u64 { return pack(key_ord<true, LARGEST>(row[i]), i); };
    auto lsrc = [&](u32 i) -> u64 { return sh.buf[i]; };

    u32 na = 0, nb = len;
    bool in_lds = false;
    int band_top = 64;                  // pairs in LDS agree at and above this bit
    if (len <= BT_CAP) {
        u32 x[BT_CAP / BT_THREADS];                // all loads first, one wait
#pragma unroll
        for (int j = 0; j < (int)(BT_CAP / BT_THREADS); ++j) {
            const u32 i = (u32)j * BT_THREADS + tid;
            x[j] = i < len ? row[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < (int)(BT_CAP / BT_THREADS); ++j) {
            const u32 i = (u32)j * BT_THREADS + tid;
            if (i < len) sh.buf[i] = pack(key_ord<true, LARGEST>(x[j]), i);
        }
        __syncthreads();
        in_lds = true;
    } else {
        u32 c_num = a.c_num;
        for (u32 att = 0; att < a.attempts && !in_lds; ++att) {
            // sample -> LDS, compacted
            u32 pos[BT_SEG];
            const int cnt = bt_sample(tid, len, a.s_target, a.seed, att, r, pos);
            u32 s;
            const u32 at = block_excl_scan<BT_THREADS>((u32)cnt, sh.scan, &s);
#pragma unroll
            for (int j = 0; j < BT_SEG; ++j)
                if (j < cnt) sh.buf[at + (u32)j] = gsrc(pos[j]);
            __syncthreads();
            i64 lo, hi;
            pivot_ranks(s, k, len, c_num, lo, hi);
            const bool hl = lo >= 0, hr = hi < (i64)s;
            u64 piv[2];
            {
                const u64 rk[2] = {hl ? (u64)lo : 0ull, hr ? (u64)hi : 0ull};
                const bool ac[2] = {hl, hr};
                bt_select(lsrc, s, 64, rk, ac, piv, sh);
            }
            const u64 L = hl ? piv[0] : 0ull;
            const u64 R = hr ? piv[1] : ~0ull;
            // one sweep: below L -> output, [L, R] -> LDS band.  Wave w takes
            // keys [s0 + 1024 w, s0 + 1024 w + 1024) of a step as 16 columns of
            // 64 lanes (coalesced); lane bits keep its keys' parts; the waves'
            // counts are exchanged once per step.
            u32 ca = 0, cb = 0;
            {
                const u32 wv = __builtin_amdgcn_readfirstlane(tid / WAVE), ln = lane_id();
                for (u32 s0 = 0, st = 0; s0 < len; s0 += BT_STEP, ++st) {
                    const u32 base = s0 + wv * (BT_STEP / BT_WAVES);
                    u32 o[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const u32 col = base + (u32)j * WAVE + ln;
                        o[j] = col < len ? row[col] : 0u;
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
                    __syncthreads();
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
            __syncthreads();
            if (ca >= k || ca + cb < k) {
                c_num *= 2;                  // the pivots missed rank k: wider
            } else if (cb > BT_CAP) {
                c_num = c_num > 1 ? c_num / 2 : 1;   // band too wide for LDS: narrower
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
    if (in_lds) {
        const u64 rk[2] = {(u64)(k - na - 1), 0ull};
        bt_select(lsrc, nb, band_top, rk, one, t2, sh);
        tau = t2[0];
        bt_emit(lsrc, nb, tau, out + na, k - na, sh);
    } else {
        // exact fallback over the row
        const u64 rk[2] = {(u64)(k - 1), 0ull};
        bt_select(gsrc, len, 64, rk, one, t2, sh);
        tau = t2[0];
        bt_emit(gsrc, len, tau, out, k, sh);
    }
    if (tid == 0) {
        a.kth_idx[r] = (u32)tau;
        a.kth_key[r] = row[(u32)tau];
    }
    __syncthreads();
}

template <bool LARGEST>
__global__ __launch_bounds__(BT_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_batched(BtArgs a)
{
    __shared__ BtShared sh;
    // rows in longest-first order from a queue: one row per grab for the first
    // BT_Q1 positions (the long rows), then BT_QCHUNK rows per grab
    for (;;) {
        if (threadIdx.x == 0) sh.next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const u32 g = sh.next;
        __syncthreads();
        const u32 p0 = g < BT_Q1 ? g : BT_Q1 + (g - BT_Q1) * BT_QCHUNK;
        if (p0 >= a.rows) break;
        const u32 p1 = g < BT_Q1 ? p0 + 1 : (p0 + BT_QCHUNK < a.rows ? p0 + BT_QCHUNK : a.rows);
        for (u32 p = p0; p < p1; ++p) bt_row<LARGEST>(a, a.order[p], sh);
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
    if (t == 0) {
        *a.status = 0u;
        *a.queue = 0u;
    }
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
    off = bt_align(off + 128);
    L.order = off;
    off = bt_align(off + (size_t)rows * sizeof(uint32_t));
    L.total = off;
    return L;
}

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

extern "C" size_t topk_batched_workspace_bytes(const topk_ctx *ctx, uint32_t rows, uint32_t flags)
{
    (void)flags;
    if (!ctx) return 0;
    return bt_layout(rows).total;
}

extern "C" int topk_select_batched_f32(topk_ctx *c, const float *keys, const uint64_t *row_off,
                                       uint32_t rows, const uint32_t *k, const uint64_t *out_off,
                                       uint32_t flags, uint32_t *out_idx, float *kth_key,
                                       uint32_t *kth_idx, uint32_t *status, void *workspace,
                                       size_t ws_bytes, hipStream_t stream)
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
    BtArgs a{};
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
    a.s_target = (u32)c->bt_s_target;
    a.c_num = (u32)c->bt_c_num;
    a.attempts = (u32)c->bt_attempts;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    const int grid = (int)(c->num_cu * c->bt_wg_per_cu);   // 4 fit on a CU (LDS, registers)
    if (!(flags & TOPK_GRAPH))
        return bt_enqueue(a, grid, stream) == hipSuccess ? TOPK_OK : TOPK_E_HIP;

    // one graph per distinct argument set: captured once, then replayed
    std::vector<uint64_t> key = {
        (uint64_t)(uintptr_t)keys, (uint64_t)(uintptr_t)row_off, rows, (uint64_t)(uintptr_t)k,
        (uint64_t)(uintptr_t)out_off, a.flags, (uint64_t)(uintptr_t)out_idx,
        (uint64_t)(uintptr_t)kth_key, (uint64_t)(uintptr_t)kth_idx, (uint64_t)(uintptr_t)status,
        (uint64_t)(uintptr_t)workspace, a.seed, a.s_target, a.c_num, a.attempts, (uint64_t)grid};
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
        it = c->graphs.emplace(key, ge).first;
    }
    return hipGraphLaunch(it->second, stream) == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}
