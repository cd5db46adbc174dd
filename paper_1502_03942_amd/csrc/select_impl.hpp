// Single-instance sampling selection (Hübschle-Schneider, Sanders, Müller):
// §2 Algorithm "communication efficient selection" with §4.1's Bernoulli
// sampling, mapped onto one gfx950 device.  Kernel templates; each key type
// and order is instantiated in a translation unit of its own (select_*.hip).
//
//   k_sample one lane per (segment, skip): round 1's Bernoulli sample.
//   k_pivot  one 1024-thread workgroup: applies the branch of the Algorithm to
//            the counts of the previous sweep (driver), then either solves a
//            small subproblem directly (finisher) or picks the two pivots by
//            an LDS radix select of two ranks of the current sample.
//   k_sweep  many workgroups: one streaming pass over the subproblem that
//            classifies every element against (l, r), counts a and b with
//            wave ballots, reserves output ranges with one 64-bit atomic per
//            generation of wave-tiles, and writes a's positions to the output
//            and b to the next band buffer; it also draws the next round's
//            sample from b.
//   k_tail   one workgroup that runs the remaining rounds itself (driver,
//            sample, pivots, a workgroup-wide sweep), the exact fallback once
//            the attempt budget is spent, and the finisher.
//
// The host enqueues k_sample, k_pivot, k_sweep, [k_pivot, k_sweep]..., k_tail
// once; the round state lives in device memory, so no round trip to the host
// occurs.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "select.hpp"
#include "radix.hpp"
#include "../../include/topk.h"

namespace topk {

typedef u32 u32x4 __attribute__((ext_vector_type(4)));

struct Smem {
    RadixShared rs;
    u32 scan[PV_THREADS / WAVE];
    u64 L64, R64;
    i64 lo, hi;
    u64 hs_T;
    u32 phase, n_cur, k_cur, src, tag, c_num, cursor, s_total, hs_ok, hs_count;
};

// ---------------------------------------------------------------------------
// Sample drawn while a round's middle part b is formed (§2, "Bernoulli
// sampling": each object independently with probability rho).  Element x
// (input position) is taken iff word 0 of Philox4x32-10 at counter
// (x, 0, tag, 1), key = seed, is below T = rho 2^32.  rho = s_target over the
// expected |b|: the pivots cover sample ranks [bot, top) with bot = lo (0 if
// no lower pivot) and top = hi + 1 (s if no upper pivot), so |b| ~ n (top-bot)/s.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 band_threshold(u64 n_cur, u64 s, i64 lo, i64 hi, u64 s_target)
{
    u64 nb_est = n_cur;
    if (s > 0) {
        const i64 bot = lo >= 0 ? lo : 0;
        const i64 top = hi < (i64)s ? hi + 1 : (i64)s;
        nb_est = n_cur * (u64)(top - bot) / s;
    }
    if (nb_est == 0) nb_est = 1;
    return (s_target << 32) / nb_est;
}

__device__ __forceinline__ bool hash_taken(u64 seed, u32 tag, u32 x, u64 T)
{
    const uint4 r = philox4x32_10(make_uint4(x, 0u, tag, 1u), (u32)seed, (u32)(seed >> 32));
    return (u64)r.x < T;
}

// Append the taken elements of this wave (lane flag `take`, pair `e`) to the
// collected sample; positions beyond S_MAX are counted but not stored.
__device__ __forceinline__ void sample_append(const SelArgs &a, State *st, bool take, u64 e)
{
    const u64 m = ballot(take);
    if (m) {
        const int first = __ffsll((unsigned long long)m) - 1;
        u32 base = 0;
        if ((int)lane_id() == first) base = atomicAdd(&st->hs_count, (u32)__popcll(m));
        base = __shfl(base, first, WAVE);
        if (take) {
            const u32 q = base + mbcnt(m);
            if (q < (u32)S_MAX) a.hs_buf[q] = e;
        }
    }
}

// ---------------------------------------------------------------------------
// State machine pieces (thread 0 of the driving workgroup).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void state_init(const SelArgs &a, State *st)
{
    st->phase = PH_PIVOT;
    st->n_cur = a.n;
    st->k_cur = a.k;
    st->cursor = 0;
    st->src = 0;
    st->tag = 0;
    st->c_num = a.c_num0;
    st->na = st->nb = 0;
    st->nrec = 0;
    st->hs_ok = 0;
    st->resv = 0;
    st->gen = 0;
    st->hs_count = 0;
}

// Branch of the Algorithm after a sweep: recurse into b when the pivots
// bracket rank k_cur (n_a < k_cur <= n_a + n_b) and b is narrower than its
// buffer and than the subproblem.  Otherwise repeat the round on the same
// subproblem with a fresh stream: after a miss (the Algorithm's recursions
// into a or c) with c doubled, after a too wide b with c halved.
__device__ __forceinline__ void driver_eval(const SelArgs &a, State *st)
{
    if (st->phase != PH_SWEEP) return;
    const u32 tag = st->tag;
    const u32 na = (u32)(st->resv >> 32), nb = (u32)st->resv;
    const u32 n = st->n_cur, k = st->k_cur;
    st->na = na;
    st->nb = nb;
    const bool miss = na >= k || (u64)na + nb < k;
    const bool wide = nb > a.band_cap || nb == n;
    const bool ok = !miss && !wide;
    if (tag < R_TRACE) {
        st->rec[tag].na = na;
        st->rec[tag].nb = nb;
        st->rec[tag].ok = ok ? 1u : 0u;
    }
    st->tag = tag + 1;
    st->hs_ok = (ok && st->hs_count <= (u32)S_MAX) ? 1u : 0u;
    if (ok) {
        st->cursor += na;
        st->k_cur = k - na;
        st->n_cur = nb;
        st->src = (st->src == 1) ? 2u : 1u;
        st->c_num = a.c_num0;
    } else if (miss) {
        const u32 c = st->c_num * 2u;
        st->c_num = c > 4096u ? 4096u : c;
    } else {
        st->c_num = st->c_num / 2u;
    }
    st->phase = PH_PIVOT;
}

__device__ __forceinline__ void load_state(const State *st, Smem &sm)
{
    sm.phase = st->phase;
    sm.n_cur = st->n_cur;
    sm.k_cur = st->k_cur;
    sm.src = st->src;
    sm.tag = st->tag;
    sm.c_num = st->c_num;
    sm.cursor = st->cursor;
    sm.hs_ok = st->hs_ok;
    sm.hs_count = st->hs_count;
}

// element `p` of the current subproblem as an (ord, position) pair
template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ u64 fetch_elem(const SelArgs &a, u32 src, u64 p)
{
    if (src == 0) return pack(key_ord<IS_F32, LARGEST>(a.keys[p]), (u32)p);
    return pack(a.band_ord[src - 1][p], a.band_idx[src - 1][p]);
}

// v[j] = element p(j) of source src for every j < N, all loads issued before
// the first is used (src uniform: one branch around the whole gather).
template <bool IS_F32, bool LARGEST, int N, class POS>
__device__ __forceinline__ void fetch_elems(const SelArgs &a, u32 src, POS p, u64 (&v)[N])
{
    src = __builtin_amdgcn_readfirstlane(src);
    if (src == 0) {
        u32 x[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = a.keys[p(j)];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = pack(key_ord<IS_F32, LARGEST>(x[j]), (u32)p(j));
    } else {
        const u32 *__restrict__ bo = a.band_ord[src - 1];
        const u32 *__restrict__ bi = a.band_idx[src - 1];
        u32 o[N], i[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            o[j] = bo[p(j)];
            i[j] = bi[p(j)];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = pack(o[j], i[j]);
    }
}

// ---------------------------------------------------------------------------
// Sample and pivots (§2 "Bernoulli sampling", FR-selection; §4.1 samples the
// current subproblem at rate s_target / n_cur).  Thread t owns segment t of
// ceil(n/1024) consecutive positions and walks it with geometric skips
// 1 + floor(ln U / ln(1 - rho)), U from Philox4x32-10 counter
// (draw/4, t, attempt, 0) and key = seed; it keeps at most SEG_CAP positions.
// ---------------------------------------------------------------------------
// Geometric-skip Bernoulli sampler of one segment (§2 sampling; each of the
// n positions is taken independently with probability rho = s_target / n).
// Segment t of NSEG covers [t L, min(t L + L, n)), L = ceil(n / NSEG); skip
// j of the segment is 1 + floor(ln U / ln(1 - rho)) with U = (w + 1/2) 2^-32,
// w the word j % 4 of Philox4x32-10 at counter (j / 4, t, tag, 0), key =
// seed.  At most SEG_CAP positions per segment.  Returns their count.
__device__ __forceinline__ int skip_sample(u32 t, u32 n, u32 s_target, u64 seed, u32 tag,
                                           u32 (&pos)[SEG_CAP])
{
    const double rho = (double)s_target / (double)n;
    const u64 L = ((u64)n + NSEG - 1) / NSEG;
    const u64 s0 = (u64)t * L;
    const u64 e0 = s0 + L < (u64)n ? s0 + L : (u64)n;
    int cnt = 0;
    if (s0 >= e0) return 0;
    if (rho >= 1.0) {
#pragma unroll
        for (int j = 0; j < SEG_CAP; ++j)
            if (s0 + j < e0) { pos[j] = (u32)(s0 + j); cnt = j + 1; }
        return cnt;
    }
    const double ln1mrho = log1p(-rho);
    i64 p = (i64)s0 - 1;
    bool stop = false;
    uint4 r4 = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int j = 0; j < SEG_CAP; ++j) {
        if (!stop) {
            if ((j & 3) == 0)
                r4 = philox4x32_10(make_uint4((u32)(j >> 2), t, tag, 0u), (u32)seed, (u32)(seed >> 32));
            const u32 w = (j & 3) == 0 ? r4.x : (j & 3) == 1 ? r4.y : (j & 3) == 2 ? r4.z : r4.w;
            const double u = ((double)w + 0.5) * (1.0 / 4294967296.0);
            const double q = log(u) / ln1mrho;
            if (q >= (double)((i64)e0 - 1 - p)) {
                stop = true;
            } else {
                p = p + 1 + (i64)q;
                pos[j] = (u32)p;
                cnt = j + 1;
            }
        }
    }
    return cnt;
}

// Round 1's sample with one lane per (segment, skip): the skips of a segment
// do not depend on each other, only their running sum does, so lane j of a
// 16-lane row computes skip j (the same fp64 operations as skip_sample) and
// a row prefix sum gives the positions.  A skip is clamped to L + 1, which
// leaves every position past the segment's end past it.
template <bool IS_F32, bool LARGEST>
__global__ __launch_bounds__(WAVE) void k_sample(SelArgs a)
{
    static_assert(SEG_CAP == 16, "one DPP row per segment");
    const u32 g = blockIdx.x * WAVE + threadIdx.x;
    const u32 t = g / SEG_CAP, j = g % SEG_CAP;
    const u32 n = a.n;
    const double rho = (double)a.s_target / (double)n;
    const u64 L = ((u64)n + NSEG - 1) / NSEG;
    const u64 s0 = (u64)t * L;
    const u64 e0 = s0 + L < (u64)n ? s0 + L : (u64)n;
    u32 skip;
    if (rho >= 1.0) {
        skip = 1u;
    } else {
        const uint4 r4 = philox4x32_10(make_uint4(j >> 2, t, 0u, 0u), (u32)a.seed, (u32)(a.seed >> 32));
        const u32 w = (j & 3) == 0 ? r4.x : (j & 3) == 1 ? r4.y : (j & 3) == 2 ? r4.z : r4.w;
        const double u = ((double)w + 0.5) * (1.0 / 4294967296.0);
        const double q = log(u) / log1p(-rho);
        skip = q >= (double)L ? (u32)L + 1u : 1u + (u32)(u64)q;
    }
    // inclusive sum over the row (the segment)
    u32 sum = skip;
    sum += dpp<DPP_ROW_SHR1>(sum);
    sum += dpp<DPP_ROW_SHR2>(sum);
    sum += dpp<DPP_ROW_SHR4>(sum);
    sum += dpp<DPP_ROW_SHR8>(sum);
    const u64 p = s0 - 1 + (u64)sum;
    const bool ok = s0 < e0 && p < e0;
    if (ok) a.hs_buf[t * SEG_CAP + j] = fetch_elem<IS_F32, LARGEST>(a, 0u, (u32)p);
    const u64 m = ballot(ok);
    if (j == 0) a.seg_cnt[t] = (u32)__popcll(m & (0xFFFFull << (lane_id() & 48u)));
}

template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ void sample_and_pivot(const SelArgs &a, State *st, Smem &sm)
{
    const u32 tid = threadIdx.x;
    const u32 n = sm.n_cur, k = sm.k_cur, src = sm.src, tag = sm.tag;
    const bool collected = sm.hs_ok != 0;   // sample drawn while this subproblem was formed
    // round 1's sample drawn by k_sample (segment t in hs_buf[t SEG_CAP ..])
    const bool pre = a.presampled && tag == 0 && src == 0;
    u32 pos[SEG_CAP];
    int cnt = 0;
    if (collected) {
        const u32 hc = sm.hs_count;
#pragma unroll
        for (int j = 0; j < SEG_CAP; ++j)
            if (tid + (u32)j * PV_THREADS < hc) cnt = j + 1;
    } else if (pre) {
        cnt = (int)a.seg_cnt[tid];
    } else {
        cnt = skip_sample(tid, n, a.s_target, a.seed, tag, pos);
    }
    // every load is issued before the first is used: slots past cnt read an
    // in-bounds element (the sample buffer holds S_MAX pairs; position 0
    // exists) and are then marked empty
    u64 v[SEG_CAP];
    if (collected) {
#pragma unroll
        for (int j = 0; j < SEG_CAP; ++j) v[j] = a.hs_buf[tid + (u32)j * PV_THREADS];
    } else if (pre) {
#pragma unroll
        for (int j = 0; j < SEG_CAP; ++j) v[j] = a.hs_buf[tid * SEG_CAP + (u32)j];
    } else {
        fetch_elems<IS_F32, LARGEST, SEG_CAP>(
            a, src, [&](int j) -> u64 { return j < cnt ? pos[j] : 0u; }, v);
    }
#pragma unroll
    for (int j = 0; j < SEG_CAP; ++j) v[j] = j < cnt ? v[j] : ~0ull;

    u32 s_total;
    const u32 excl = block_excl_scan<PV_THREADS>((u32)cnt, sm.scan, &s_total);
    if (a.trace_pos && tag < R_TRACE) {
        // the sampled objects (input positions) of this attempt
        u32 *tp = a.trace_pos + (u64)tag * TRACE_STRIDE + excl;
#pragma unroll
        for (int j = 0; j < SEG_CAP; ++j)
            if (j < cnt) tp[j] = (u32)v[j];
    }
    if (tid == 0) {
        i64 lo, hi;
        pivot_ranks(s_total, k, n, sm.c_num, lo, hi);
        sm.lo = lo;
        sm.hi = hi;
        sm.s_total = s_total;
    }
    __syncthreads();
    const i64 lo = sm.lo, hi = sm.hi;
    const bool act[2] = {lo >= 0, hi < (i64)s_total};
    const u64 ranks[2] = {act[0] ? (u64)lo : 0ull, act[1] ? (u64)hi : 0ull};
    u64 piv[2];
    radix_select<SEG_CAP>(v, cnt, ranks, act, piv, sm.rs);
    if (tid == 0) {
        const u64 Lp = act[0] ? piv[0] : 0ull;
        const u64 Rp = act[1] ? piv[1] : ~0ull;
        sm.L64 = Lp;
        sm.R64 = Rp;
        st->l_ord = (u32)(Lp >> 32);
        st->l_idx = (u32)Lp;
        st->r_ord = (u32)(Rp >> 32);
        st->r_idx = (u32)Rp;
        st->has_l = act[0];
        st->has_r = act[1];
        if (tag < R_TRACE) {
            RoundRec &R = st->rec[tag];
            R.n_cur = n; R.k_cur = k; R.s = s_total; R.c_num = sm.c_num;
            R.lo = lo; R.hi = hi;
            R.l_idx = act[0] ? (u32)Lp : 0u;
            R.r_idx = act[1] ? (u32)Rp : 0u;
            R.has_l = act[0]; R.has_r = act[1];
            R.na = R.nb = R.ok = 0u;
            R.tag = tag;
            st->nrec = tag + 1;
        }
        st->phase = PH_SWEEP;
        // the coming sweep reserves output space and draws the next sample
        st->resv = 0ull;
        st->gen = 0u;
        st->hs_count = 0u;
        st->hs_T = band_threshold(n, s_total, lo, hi, a.s_target);
        sm.hs_T = st->hs_T;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Finisher (§2 base case): a subproblem of n_cur <= t_fin elements is loaded
// into registers (thread t holds a run of consecutive positions), tau = its
// element of rank k_cur is found by radix select, and every element <= tau is
// written in sequence order after the cursor.
// ---------------------------------------------------------------------------
template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ void finish(const SelArgs &a, State *st, Smem &sm)
{
    const u32 tid = threadIdx.x;
    const u32 n = sm.n_cur, k = sm.k_cur, src = sm.src;
    const u32 per = (n + PV_THREADS - 1) / PV_THREADS;
    const u64 b0 = (u64)tid * per;
    const int cnt = b0 >= n ? 0 : (int)((u64)n - b0 < per ? (u64)n - b0 : per);
    // every load is issued before the first is used (slots past cnt read
    // position n - 1, then are marked empty)
    u64 v[FIN_ITEMS];
    fetch_elems<IS_F32, LARGEST, FIN_ITEMS>(
        a, src, [&](int j) -> u64 { return j < cnt ? b0 + (u64)j : (u64)n - 1; }, v);
#pragma unroll
    for (int j = 0; j < FIN_ITEMS; ++j) v[j] = j < cnt ? v[j] : ~0ull;
    const u64 ranks[2] = {(u64)k - 1, 0ull};
    const bool act[2] = {true, false};
    u64 tau2[2];
    radix_select<FIN_ITEMS>(v, cnt, ranks, act, tau2, sm.rs);
    const u64 tau = tau2[0];
    u32 c = 0;
#pragma unroll
    for (int j = 0; j < FIN_ITEMS; ++j) c += (j < cnt && v[j] <= tau) ? 1u : 0u;
    u32 tot;
    u32 off = block_excl_scan<PV_THREADS>(c, sm.scan, &tot);
    const u64 base = (u64)sm.cursor + off;
    const bool wkeys = (a.flags & TOPK_WRITE_KEYS) && a.out_keys;
    u32 m = 0;
#pragma unroll
    for (int j = 0; j < FIN_ITEMS; ++j) {
        if (j < cnt && v[j] <= tau) {
            const u32 idx = (u32)v[j];
            if (base + m < a.k) {
                a.out_idx[base + m] = idx;
                if (wkeys) a.out_keys[base + m] = a.keys[idx];
            }
            ++m;
        }
        if (j < cnt && v[j] == tau) {
            const u32 idx = (u32)v[j];
            *a.kth_idx = idx;
            *a.kth_key = a.keys[idx];
        }
    }
    if (tid == 0) {
        st->phase = PH_DONE;
        if (a.status) *a.status = (tot == k) ? TOPK_STATUS_OK : TOPK_STATUS_INTERNAL;
    }
}

// ---------------------------------------------------------------------------
// Workgroup-wide sweep for the tail kernel: the same partition as k_sweep,
// done by one workgroup in order, with a running offset instead of look-back.
// ---------------------------------------------------------------------------
template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ void block_sweep(const SelArgs &a, State *st, Smem &sm)
{
    const u32 tid = threadIdx.x;
    const u32 n = sm.n_cur, src = sm.src;
    const u32 di = (src == 1) ? 1u : 0u;     // destination band buffer
    const u64 L64 = sm.L64, R64 = sm.R64;
    const bool wkeys = (a.flags & TOPK_WRITE_KEYS) && a.out_keys;
    u64 run_a = 0, run_b = 0;
    for (u64 base = 0; base < n; base += (u64)PV_THREADS * 4) {
        u64 e[4];
        bool fa[4], fb[4];
        u32 ta = 0, tb = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const u64 p = base + (u64)tid * 4 + u;
            const bool valid = p < n;
            e[u] = valid ? fetch_elem<IS_F32, LARGEST>(a, src, p) : 0ull;
            const bool below = e[u] < L64;
            const bool above = e[u] > R64;
            fa[u] = valid && below;
            fb[u] = valid && !below && !above;
            ta += fa[u];
            tb += fb[u];
        }
        u32 tot;
        const u32 ex = block_excl_scan<PV_THREADS>(ta | (tb << 16), sm.scan, &tot);
        u64 pa = (u64)sm.cursor + run_a + (ex & 0xFFFFu);
        u64 pb = run_b + (ex >> 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const u32 idx = (u32)e[u];
            if (fa[u]) {
                if (pa < a.k) {
                    a.out_idx[pa] = idx;
                    if (wkeys) a.out_keys[pa] = a.keys[idx];
                }
                ++pa;
            }
            if (fb[u]) {
                if (pb < a.band_cap) {
                    a.band_ord[di][pb] = (u32)(e[u] >> 32);
                    a.band_idx[di][pb] = idx;
                }
                ++pb;
            }
            sample_append(a, st, fb[u] && hash_taken(a.seed, sm.tag + 1, idx, sm.hs_T), e[u]);
        }
        run_a += tot & 0xFFFFu;
        run_b += tot >> 16;
    }
    if (tid == 0) st->resv = (run_a << 32) | run_b;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Exact fallback once the attempt budget r_max is spent (§4.1 bounds the
// number of rounds only with high probability).  tau, the object of rank
// k_cur of the current subproblem, is found by a radix select that streams
// the subproblem from memory: 8-bit digits of the (ord, position) pair from
// the top, each pass counting the objects that share the digits fixed so far,
// until the bucket holding the rank has at most S_MAX objects.  Those are
// gathered into the sample buffer and ranked in registers.  tau then becomes
// both pivots, so the round that follows keeps b = {tau}, succeeds, and
// leaves a subproblem of one object for the finisher.  One workgroup; the
// path is reached only after r_max failed attempts.
// ---------------------------------------------------------------------------
template <bool IS_F32, bool LARGEST>
__device__ __noinline__ void exact_pivot(const SelArgs &a, State *st, Smem &sm)
{
    constexpr int DB = 8;
    constexpr u32 NB = 1u << DB;
    const u32 tid = threadIdx.x;
    const u32 n = sm.n_cur, src = sm.src, tag = sm.tag;
    u32 *hist = sm.rs.rhist[0];             // NB bins (rhist holds 2 x RS_BINS)
    u32 *gcount = &sm.rs.rhist[1][0];       // gathered objects
    u64 rank = (u64)sm.k_cur - 1;
    u64 pref = 0;
    int lowb = 64;                          // bits [lowb, 64) of the candidates equal pref's
    u64 cnt = n;
    auto match = [&](u64 e) { return lowb >= 64 || (e >> lowb) == (pref >> lowb); };
    while (cnt > (u64)S_MAX && lowb > 0) {
        const int sh = lowb - DB;
        for (u32 i = tid; i < NB; i += PV_THREADS) hist[i] = 0u;
        __syncthreads();
        for (u64 p = tid; p < n; p += PV_THREADS) {
            const u64 e = fetch_elem<IS_F32, LARGEST>(a, src, p);
            if (match(e)) atomicAdd(&hist[(u32)(e >> sh) & (NB - 1)], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            u64 before = 0;
            u32 b = 0;
            for (; b < NB - 1; ++b) {
                const u32 c = hist[b];
                if (before + c > rank) break;
                before += c;
            }
            sm.rs.sel_bin[0] = b;
            sm.rs.sel_count[0] = hist[b];
            sm.rs.found[0] = before;
        }
        __syncthreads();
        pref |= (u64)sm.rs.sel_bin[0] << sh;
        lowb = sh;
        rank -= sm.rs.found[0];
        cnt = sm.rs.sel_count[0];
        __syncthreads();
    }
    u64 tau;
    if (lowb == 0) {
        tau = pref;                         // every bit fixed: one object
    } else {
        // gather the bucket (at most S_MAX objects) and rank it in registers
        if (tid == 0) *gcount = 0u;
        __syncthreads();
        for (u64 p = tid; p < n; p += PV_THREADS) {
            const u64 e = fetch_elem<IS_F32, LARGEST>(a, src, p);
            if (match(e)) a.hs_buf[atomicAdd(gcount, 1u)] = e;
        }
        __syncthreads();
        const u32 m = *gcount;
        __syncthreads();                    // radix_select clears rhist (and the count)
        u64 v[SEG_CAP];
        int c = 0;
#pragma unroll
        for (int j = 0; j < SEG_CAP; ++j) {
            const u32 q = tid * SEG_CAP + (u32)j;
            v[j] = q < m ? a.hs_buf[q] : ~0ull;
            c = q < m ? j + 1 : c;
        }
        const u64 ranks[2] = {rank, 0ull};
        const bool act[2] = {true, false};
        u64 t2[2];
        radix_select<SEG_CAP>(v, c, ranks, act, t2, sm.rs);
        tau = t2[0];
    }
    if (tid == 0) {
        sm.L64 = tau;
        sm.R64 = tau;
        st->l_ord = st->r_ord = (u32)(tau >> 32);
        st->l_idx = st->r_idx = (u32)tau;
        st->has_l = st->has_r = 1u;
        if (tag < R_TRACE) {
            RoundRec &R = st->rec[tag];
            R.n_cur = n; R.k_cur = sm.k_cur; R.s = 0u; R.c_num = sm.c_num;
            R.lo = ROUND_EXACT; R.hi = ROUND_EXACT;
            R.l_idx = R.r_idx = (u32)tau;
            R.has_l = R.has_r = 1u;
            R.na = R.nb = R.ok = 0u;
            R.tag = tag;
            st->nrec = tag + 1;
        }
        st->phase = PH_SWEEP;
        st->resv = 0ull;
        st->gen = 0u;
        st->hs_count = 0u;
        st->hs_T = 0ull;                    // no sample is drawn from b = {tau}
        sm.hs_T = 0ull;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
template <bool IS_F32, bool LARGEST>
__global__ __launch_bounds__(PV_THREADS) void k_pivot(SelArgs a)
{
    __shared__ Smem sm;
    State *st = a.st;
    if (threadIdx.x == 0) {
        if (a.first) state_init(a, st);
        driver_eval(a, st);
        load_state(st, sm);
    }
    __syncthreads();
    if (sm.phase != PH_PIVOT) return;
    if (sm.n_cur <= a.t_fin) {
        finish<IS_F32, LARGEST>(a, st, sm);
        return;
    }
    // attempt budget spent: the subproblem stays as it is (the sweeps that
    // follow see no PH_SWEEP and return) until k_tail's exact fallback
    if (sm.tag >= a.r_max) return;
    sample_and_pivot<IS_F32, LARGEST>(a, st, sm);
}

// A round of the tail kernel (pivots, or the exact fallback's pivot, then the
// workgroup-wide sweep).  Rare after the multi-workgroup rounds, so kept out
// of line: its registers are not the finisher's (which would spill).
template <bool IS_F32, bool LARGEST>
__device__ __noinline__ void tail_round(const SelArgs &a, State *st, Smem &sm)
{
    if (sm.tag >= a.r_max) exact_pivot<IS_F32, LARGEST>(a, st, sm);
    else sample_and_pivot<IS_F32, LARGEST>(a, st, sm);
    block_sweep<IS_F32, LARGEST>(a, st, sm);
}

template <bool IS_F32, bool LARGEST>
__global__ __launch_bounds__(PV_THREADS) void k_tail(SelArgs a)
{
    __shared__ Smem sm;
    State *st = a.st;
    bool first = a.first != 0;
    for (;;) {
        if (threadIdx.x == 0) {
            if (first) state_init(a, st);
            driver_eval(a, st);
            load_state(st, sm);
        }
        first = false;
        __syncthreads();
        if (sm.phase != PH_PIVOT) return;
        if (sm.n_cur <= a.t_fin) {
            finish<IS_F32, LARGEST>(a, st, sm);
            return;
        }
        tail_round<IS_F32, LARGEST>(a, st, sm);
    }
}

// ---------------------------------------------------------------------------
// The hot loop: partition of the current input into a, b, c (§2 Algorithm;
// the partition is the part of the running time that scales with n).
//
// Geometry.  A wave-tile is 64 * COLS consecutive elements; element (j, lane)
// is base + 64 j + lane, so every load instruction reads 256 contiguous bytes
// and the rank of an element among the a (or b) elements of its wave-tile, in
// sequence order, is a count over the columns before j plus one mbcnt.  Data
// wave dw of workgroup g takes wave-tiles (t G + g) W + dw, t = 0, 1, ...
// (W data waves per workgroup, G workgroups); iteration t of all data waves
// of a workgroup is its generation t.
//
// Classification.  Pass 1 compares each key with the pivots strictly: below
// l goes to a, above r to c, the rest (including keys equal to a pivot) to b.
// f32 keys are compared as floats while no pivot is NaN (-0 == +0 and NaN
// above all follow from the IEEE predicates), else through their order
// transform; u32 keys and band ords as integers.  A key equal to a pivot
// belongs to a or c by its position (§2: ties are broken by the object), so a
// wave-tile whose b holds such a key classifies again with positions; that
// happens for the few wave-tiles holding a pivot unless keys repeat.
//
// Per lane, the a-membership of the lane's 64 elements is kept as bits in
// two registers (a transposed mask), so pass 1 spends two compares per
// column on elements outside b.  b is compacted in sequence order into an
// LDS stash.  Pass 2 of a wave-tile runs after pass 1 of the next one, once
// the control wave has reserved its output ranges: it rebuilds each column's
// a-mask from the bits, writes the positions of a, and copies the stash to
// the band with coalesced stores while drawing the next round's sample from
// it (element-wise Philox decisions).  A stash overflow reloads the wave-tile.
// ---------------------------------------------------------------------------
struct Piv {
    u32 lo, li, ro, ri;     // pivot ords and positions (selection order); absent
                            // pivots are sentinels no (ord, position) pair passes
    float lv, rv;           // f32 input and fast: pivot values (an absent pivot
                            // that the fast compare allows is -inf)
    bool hl, hr;            // pivot present
    bool fast;              // f32 input: compare as floats (see load_pivots)
};

__device__ __forceinline__ u32 bits_from_ord(u32 o)
{
    return (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
}

// The float compare needs non-NaN pivots and, in smallest order, a right
// pivot (no float threshold leaves NaN out of c), in largest order a left
// pivot (none leaves NaN out of a).  The other absent pivot becomes -inf:
// nothing is below it (smallest) and nothing after it (largest).
template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ Piv load_pivots(const State *st)
{
    Piv p;
    p.hl = st->has_l != 0;
    p.hr = st->has_r != 0;
    p.lo = p.hl ? st->l_ord : 0u;
    p.li = p.hl ? st->l_idx : 0u;
    p.ro = p.hr ? st->r_ord : 0xFFFFFFFFu;
    p.ri = p.hr ? st->r_idx : 0xFFFFFFFFu;
    p.fast = false;
    p.lv = p.rv = 0.f;
    if (IS_F32) {
        const u32 ls = LARGEST ? ~p.lo : p.lo, rs = LARGEST ? ~p.ro : p.ro;  // ascending ords
        const bool lnan = p.hl && ls == 0xFFFFFFFFu, rnan = p.hr && rs == 0xFFFFFFFFu;
        p.fast = !lnan && !rnan && (LARGEST ? p.hl : p.hr);
        const float ninf = __uint_as_float(0xFF800000u);
        p.lv = p.hl ? __uint_as_float(bits_from_ord(ls)) : ninf;
        p.rv = p.hr ? __uint_as_float(bits_from_ord(rs)) : ninf;
    }
    return p;
}

// Selection-order ord of an element as loaded.  KIND 0: f32 key bits, 1: u32
// key, 2: band ord (already one).
template <int KIND, bool LARGEST>
__device__ __forceinline__ u32 ord_of(u32 x)
{
    return KIND == 0 ? key_ord<true, LARGEST>(x) : KIND == 1 ? (LARGEST ? ~x : x) : x;
}

// Membership of one element: ia = in a, ic = in c.  TIES: break ties with a
// pivot by position i (else keys equal to a pivot are in b).
template <int KIND, bool LARGEST, bool FAST, bool TIES>
__device__ __forceinline__ void classify(u32 x, u32 i, const Piv &p, bool &ia, bool &ic)
{
    if (KIND == 0 && FAST) {
        const float f = __uint_as_float(x);
        ia = LARGEST ? !(f <= p.lv) : (f < p.lv);
        ic = LARGEST ? (f < p.rv) : !(f <= p.rv);
        if (TIES) {
            ia = ia || (p.hl && f == p.lv && i < p.li);
            ic = ic || (p.hr && f == p.rv && i > p.ri);
        }
    } else {
        const u32 o = ord_of<KIND, LARGEST>(x);
        ia = o < p.lo;
        ic = o > p.ro;
        if (TIES) {
            ia = ia || (p.hl && o == p.lo && i < p.li);
            ic = ic || (p.hr && o == p.ro && i > p.ri);
        }
    }
}

// Does x equal a present pivot (so that its position decides its part)?
template <int KIND, bool LARGEST, bool FAST>
__device__ __forceinline__ bool equals_pivot(u32 x, const Piv &p)
{
    if (KIND == 0 && FAST) {
        const float f = __uint_as_float(x);
        return (p.hl && f == p.lv) || (p.hr && f == p.rv);
    }
    const u32 o = ord_of<KIND, LARGEST>(x);
    return (p.hl && o == p.lo) || (p.hr && o == p.ro);
}

// f(std::integral_constant<int, J>()) for J = 0 .. N-1, unrolled.
template <class F, int... J>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, J...>)
{
    (f(std::integral_constant<int, J>()), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>());
}

// mbcnt(mask) + base
__device__ __forceinline__ u32 mbcnt_add(u64 mask, u32 base)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, base));
}

// LDS of a sweep workgroup: per data wave two wave-tile slots.
struct WSlot {
    u64 stash[SW_STASH + WAVE]; // b of the wave-tile in sequence order: key bits
                                // (band: ord) << 32 | position; a column is
                                // stashed whole while fewer than SW_STASH precede it
    u32 cnt;                    // |a| | |b| << 16 of the wave-tile
    u32 base_a, base_b;         // reserved output positions (relative to the round's start)
    u32 state;                  // 0 free, 1 counted (posted), 2 space reserved
};
constexpr u32 SW_GRING = 4;     // generation numbers published ahead (ring)
struct SwShared {
    WSlot slot[SW_DW][SW_SLOTS];    // [data wave][generation % SW_SLOTS]
    u32 gnum[SW_GRING];             // workgroup's generation t: wave-tiles gnum W + dw
    u32 gseq[SW_GRING];             // t + 1 once gnum[t % SW_GRING] is published
};

__device__ __forceinline__ u32 lds_acquire(u32 *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_release(u32 *p, u32 v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One sweep workgroup: wave 0 reserves output space, waves 1..SW_DW stream.
// The reservation is one global atomic on a 64-bit counter |a| << 32 | |b|
// per generation of the workgroup, so pass 2 of a wave-tile (which waits for
// it) trails pass 1 by one wave-tile and wave-tiles of one workgroup never
// wait for another workgroup.  Inside a generation the output is in sequence
// order; the order of the generations' ranges follows the reservations.
template <int KIND, bool IS_F32, bool LARGEST, bool FAST>
__device__ __forceinline__ void sweep_waves(const SelArgs &a, State *st, const Piv &p, u32 n,
                                            u32 src, u32 tag, SwShared &sh)
{
    constexpr int COLS = KIND == 2 ? SW_COLS_BAND : SW_COLS_IN;
    static_assert(COLS <= 64 && (COLS <= 32 || COLS % 32 == 0), "a-bits: two 32-bit words");
    constexpr u32 WSPAN = (u32)WAVE * COLS;
    const u32 lane = lane_id();
    const u32 w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const u32 nwt = (u32)(((u64)n + WSPAN - 1) / WSPAN);
    // A workgroup whose first generation holds no wave-tile has nothing to do
    // (generation numbers only grow): it leaves before touching a counter, so
    // a grid sized for the largest subproblem costs little on a small one.
    if ((u64)blockIdx.x * SW_DW >= (u64)nwt) return;

    if (w == 0) {
        // ------------- control wave: one reservation per generation -------------
        // Generation t of this workgroup is the generation number g_t: its
        // wave-tiles are g_t W + dw (W = SW_DW).  g_0 = blockIdx; later ones
        // come from a global counter (so faster workgroups take more), published
        // SW_GRING - 1 generations ahead.  Once every data wave that has a
        // wave-tile in generation t has posted its counts, one atomic reserves
        // the output ranges of the whole generation.
        u32 *gctr = &st->gen;
        auto publish = [&](u32 t, u32 g) {
            if (lane == 0) {
                sh.gnum[t % SW_GRING] = g;
                lds_release(&sh.gseq[t % SW_GRING], t + 1u);
            }
        };
        if (lane < SW_GRING) sh.gseq[lane] = 0u;     // LDS keeps an earlier kernel's values
        publish(0u, blockIdx.x);
        __syncthreads();
        auto fetch = [&]() -> u32 {
            u32 g = 0;
            if (lane == 0) g = atomicAdd(gctr, 1u) + gridDim.x;
            return __builtin_amdgcn_readfirstlane(__shfl(g, 0, WAVE));
        };
        for (u32 t = 1; t < SW_GRING - 1; ++t) publish(t, fetch());
        u64 *resv = &st->resv;
        for (u32 t = 0;; ++t) {
            const u32 gt = __builtin_amdgcn_readfirstlane(sh.gnum[t % SW_GRING]);
            const u64 t0 = (u64)gt * (u64)SW_DW;
            if (t0 >= nwt) break;       // numbers only grow: nothing after it either
            publish(t + SW_GRING - 1, fetch());
            const u32 expected = (u64)nwt - t0 < (u64)SW_DW ? (u32)((u64)nwt - t0) : (u32)SW_DW;
            const bool mine = lane < expected;
            WSlot *S = &sh.slot[mine ? lane : 0u][t % SW_SLOTS];
            while (ballot(mine && lds_acquire(&S->state) != 1u)) __builtin_amdgcn_s_sleep(1);
            const u32 c = mine ? S->cnt : 0u;
            const u32 ca = c & 0xFFFFu, cb = c >> 16;
            const u32 ia = wave_incl_scan(ca), ib = wave_incl_scan(cb);
            const u32 ta = __shfl(ia, WAVE - 1, WAVE), tb = __shfl(ib, WAVE - 1, WAVE);
            u64 base = 0;
            if (lane == 0) base = atomicAdd((unsigned long long *)resv, ((u64)ta << 32) | tb);
            const u32 bh = __shfl((u32)(base >> 32), 0, WAVE), bl = __shfl((u32)base, 0, WAVE);
            if (mine) {
                S->base_a = bh + ia - ca;
                S->base_b = bl + ib - cb;
                lds_release(&S->state, 2u);
            }
        }
        return;
    }

    // ---------------- data waves ----------------
    const u32 dw = w - 1;
    if (lane == 0)
        for (int i = 0; i < SW_SLOTS; ++i) sh.slot[dw][i].state = 0u;
    __syncthreads();
    // wave-tile of this data wave in the workgroup's generation t (or nwt)
    auto tile_of = [&](u32 t) -> u32 {
        u32 *q = &sh.gseq[t % SW_GRING];
        while (lds_acquire(q) != t + 1u) __builtin_amdgcn_s_sleep(1);
        const u64 wt = (u64)__builtin_amdgcn_readfirstlane(sh.gnum[t % SW_GRING]) * SW_DW + dw;
        return wt < (u64)nwt ? (u32)wt : nwt;
    };
    const u64 cursor = st->cursor;
    const u64 hs_T = st->hs_T;
    const u32 di = (src == 1) ? 1u : 0u;
    u32 *__restrict__ dord = a.band_ord[di];
    u32 *__restrict__ didx = a.band_idx[di];
    const u32 *__restrict__ sord = KIND == 2 ? a.band_ord[src - 1] : a.keys;
    const u32 *__restrict__ sidx = KIND == 2 ? a.band_idx[src - 1] : a.keys;
    const bool wkeys = (a.flags & TOPK_WRITE_KEYS) && a.out_keys;
    u32 x[COLS], ix[COLS];

    // Loads of one wave-tile; only the last (ragged) wave-tile tests bounds.
    auto issue = [&](u32 wt) {
        const u64 wb = (u64)wt * WSPAN;
        const u32 *__restrict__ pw = sord + wb;
        const u32 *__restrict__ pi = sidx + wb;
        u32 ln = lane;
        asm volatile("" : "+v"(ln));
        if ((u64)n - wb >= WSPAN) {
#pragma unroll
            for (int j = 0; j < COLS; ++j) {
                x[j] = __builtin_nontemporal_load(pw + j * WAVE + ln);
                if (KIND == 2) ix[j] = __builtin_nontemporal_load(pi + j * WAVE + ln);
            }
        } else {
            int rem = (int)((u64)n - wb);
            asm volatile("" : "+s"(rem));
#pragma unroll
            for (int j = 0; j < COLS; ++j) {
                const bool ok = (int)ln < rem - j * WAVE;
                x[j] = ok ? __builtin_nontemporal_load(pw + j * WAVE + ln) : 0u;
                if (KIND == 2) ix[j] = ok ? __builtin_nontemporal_load(pi + j * WAVE + ln) : 0u;
            }
        }
    };

    // Pass 1 over the loaded (full) wave-tile, ties left in b: a-bits (column
    // j in bit W - 1 - j % 32 of A[j / 32], W = min(COLS, 32)), b into the
    // stash; returns |b|.
    auto pass1 = [&](WSlot &S, u32 ib, u32 &A0, u32 &A1) -> u32 {
        u32 ln = lane;
        asm volatile("" : "+v"(ln));
        u32 a0 = 0, a1 = 0, tb = 0;
        static_for<COLS>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            bool ia, ic;
            classify<KIND, LARGEST, FAST, false>(x[j], 0u, p, ia, ic);
            if (j < 32) a0 = a0 + a0 + (u32)ia;
            else        a1 = a1 + a1 + (u32)ia;
            asm volatile("" : "+v"(a0), "+v"(a1));   // materialize now (else every mask stays live)
            const u64 mb = ~(ballot(ia) | ballot(ic));
            if (mb) {
                if (tb < (u32)SW_STASH && !(ia || ic)) {
                    u32 xk = x[j];
                    asm volatile("" : "+v"(xk));    // a register of its own (else keys load into pairs)
                    const u32 ie = KIND == 2 ? ix[j] : ib + (u32)(j * WAVE) + ln;
                    S.stash[mbcnt_add(mb, tb)] = pack(xk, ie);
                }
                tb += (u32)__popcll(mb);
            }
            __builtin_amdgcn_sched_barrier(0);
        });
        A0 = a0;
        A1 = a1;
        return tb;
    };

    // Pass 1 with ties broken by position, over the wave-tile still in x[]
    // (wave-tiles whose b holds a key equal to a pivot, and the last one).
    auto pass1_ties = [&](WSlot &S, u64 wb, u32 &A0, u32 &A1) -> u32 {
        u32 ln = lane;
        asm volatile("" : "+v"(ln));
        const int rem = (u64)n - wb < WSPAN ? (int)((u64)n - wb) : (int)WSPAN;
        u32 a0 = 0, a1 = 0, tb = 0;
        static_for<COLS>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const u32 ie = KIND == 2 ? ix[j] : (u32)wb + (u32)(j * WAVE) + ln;
            const bool ok = (int)ln < rem - j * WAVE;
            bool ia, ic;
            classify<KIND, LARGEST, FAST, true>(x[j], ie, p, ia, ic);
            ia = ia && ok;
            ic = ic || !ok;
            if (j < 32) a0 = a0 + a0 + (u32)ia;
            else        a1 = a1 + a1 + (u32)ia;
            asm volatile("" : "+v"(a0), "+v"(a1));
            const bool ibb = !(ia || ic);
            const u64 mb = ballot(ibb);
            if (mb) {
                if (tb < (u32)SW_STASH && ibb) {
                    u32 xk = x[j];
                    asm volatile("" : "+v"(xk));
                    S.stash[mbcnt_add(mb, tb)] = pack(xk, ie);
                }
                tb += (u32)__popcll(mb);
            }
            asm volatile("" : "+s"(tb));
            __builtin_amdgcn_sched_barrier(0);
        });
        A0 = a0;
        A1 = a1;
        return tb;
    };

    // Pass 1 with the tie and overflow checks; posts the counts.
    auto count_tile = [&](u32 wt, WSlot &S, u32 &A0, u32 &A1) {
        const u64 wb = (u64)wt * WSPAN;
        u32 tb;
        bool redo = (u64)n - wb < WSPAN;
        if (!redo) {
            tb = pass1(S, (u32)wb, A0, A1);
            redo = tb > (u32)SW_STASH;
            if (!redo && (p.hl || p.hr)) {
                // keys equal to a pivot were left in b: look for them in the stash
                bool eq = false;
                for (u32 q0 = 0; q0 < tb; q0 += WAVE) {
                    const u32 q = q0 + lane;
                    eq = eq || (q < tb && equals_pivot<KIND, LARGEST, FAST>((u32)(S.stash[q] >> 32), p));
                }
                redo = ballot(eq) != 0;
            }
        }
        if (redo) tb = pass1_ties(S, wb, A0, A1);
        const u32 ta = wave_sum_u32((u32)__popc(A0) + (u32)__popc(A1));
        if (lane == 0) {
            S.cnt = ta | (tb << 16);
            lds_release(&S.state, 1u);
        }
    };

    // Pass 2: write a and b of a counted wave-tile.  Band input runs it right
    // after pass 1 (positions still in ix[]); key input one wave-tile later.
    auto write_tile = [&](u32 wt, WSlot &P, u32 A0, u32 A1) {
        while (lds_acquire(&P.state) != 2u) __builtin_amdgcn_s_sleep(1);
        const u64 wb = (u64)wt * WSPAN;
        const u32 *__restrict__ pw = sord + wb;
        const u32 *__restrict__ pi = sidx + wb;
        const u32 cnt = P.cnt, ca = cnt & 0xFFFFu, cb = cnt >> 16;
        u32 ln = lane;
        asm volatile("" : "+v"(ln));
        if (ca) {
            const u64 abase = cursor + P.base_a;
            const bool fits = abase + ca <= a.k;   // else a round that misses: clip at k
            u32 *__restrict__ oi = a.out_idx + abase;
            u32 ra = 0;
            // column j went in as bit (columns in its word - 1 - j % 32)
            constexpr int WBITS = COLS < 32 ? COLS : 32;
            auto abit = [&](int j) -> bool {
                return ((((j < 32) ? A0 : A1) >> (WBITS - 1 - (j & 31))) & 1u) != 0;
            };
            if (!wkeys) {
                // positions only (band input: still in registers)
                auto put = [&](auto clip_tag) {
                    constexpr bool CLIP = decltype(clip_tag)::value;
                    const u32 lim = CLIP ? (u32)(a.k - abase) : 0u;   // abase < k when clipping
                    static_for<COLS>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        const bool ia = abit(j);
                        const u64 ma = ballot(ia);
                        if (ma) {
                            if (ia) {
                                const u32 q = mbcnt_add(ma, ra);
                                if (!CLIP || q < lim)
                                    oi[q] = KIND == 2 ? ix[j] : (u32)wb + (u32)(j * WAVE) + ln;
                            }
                            ra += (u32)__popcll(ma);
                        }
                    });
                };
                if (fits) put(std::false_type());
                else if (abase < a.k) put(std::true_type());
            } else {
                // keys are read again: per group of columns all loads first,
                // then one wait
                constexpr int G = 16;
                static_for<COLS / G>([&](auto gc) {
                    constexpr int g = decltype(gc)::value;
                    u32 kv[G];
                    static_for<G>([&](auto uc) {
                        constexpr int u = decltype(uc)::value, j = g * G + u;
                        kv[u] = 0u;
                        if (abit(j)) kv[u] = KIND == 2 ? a.keys[ix[j]] : pw[j * WAVE + ln];
                    });
                    static_for<G>([&](auto uc) {
                        constexpr int u = decltype(uc)::value, j = g * G + u;
                        const bool ia = abit(j);
                        const u64 ma = ballot(ia);
                        if (ma) {
                            if (ia) {
                                const u32 q = mbcnt_add(ma, ra);
                                if (fits || abase + q < a.k) {
                                    oi[q] = KIND == 2 ? ix[j] : (u32)wb + (u32)(j * WAVE) + ln;
                                    a.out_keys[abase + q] = kv[u];
                                }
                            }
                            ra += (u32)__popcll(ma);
                        }
                    });
                    __builtin_amdgcn_sched_barrier(0);
                });
            }
        }
        if (cb == 0) {
        } else if (cb <= (u32)SW_STASH) {
            // b from the stash: contiguous, coalesced writes.  The next
            // round's sample decisions of the whole wave-tile come first, so
            // one atomic reserves their place in the collected sample (a hot
            // counter: one round trip per wave-tile, not per column).
            static_assert(SW_STASH <= 32 * WAVE, "one take bit per stash column");
            const u64 pb0 = P.base_b;
            u32 tbits = 0, ntake = 0;
            if (hs_T) {
                for (u32 q0 = 0, c = 0; q0 < cb; q0 += WAVE, ++c) {
                    const u32 q = q0 + ln;
                    const bool tk = q < cb && hash_taken(a.seed, tag + 1, (u32)P.stash[q], hs_T);
                    tbits |= (u32)tk << c;
                    ntake += (u32)__popcll(ballot(tk));
                }
            }
            u32 sq = 0;
            if (ntake) {
                if (ln == 0) sq = atomicAdd(&st->hs_count, ntake);
                sq = __builtin_amdgcn_readfirstlane(sq);
            }
            for (u32 q0 = 0, c = 0; q0 < cb; q0 += WAVE, ++c) {
                const u32 q = q0 + ln;
                const bool have = q < cb;
                const u64 e = have ? P.stash[q] : 0ull;
                const u32 o = ord_of<KIND, LARGEST>((u32)(e >> 32)), iv = (u32)e;
                const u64 dst = pb0 + q;
                if (have && dst < a.band_cap) {
                    dord[dst] = o;
                    didx[dst] = iv;
                }
                const bool tk = (tbits >> c) & 1u;
                const u64 mt = ballot(tk);
                if (tk) {
                    const u32 sp = sq + mbcnt(mt);
                    if (sp < (u32)S_MAX) a.hs_buf[sp] = pack(o, iv);
                }
                sq += (u32)__popcll(mt);
            }
        } else {
            // b did not fit the stash: read the wave-tile again, one column at a time
            u64 pb = P.base_b;
#pragma unroll 1
            for (u32 j = 0; j < (u32)COLS; ++j) {
                const u32 e = j * WAVE + ln;
                const bool ok = wb + e < (u64)n;
                const u32 xv = ok ? pw[e] : 0u;
                const u32 iv = KIND == 2 ? (ok ? pi[e] : 0u) : (u32)wb + e;
                bool ia, ic;
                classify<KIND, LARGEST, FAST, true>(xv, iv, p, ia, ic);
                const bool ibb = ok && !(ia || ic);
                const u64 mb = ballot(ibb);
                if (mb) {
                    const u32 o = ord_of<KIND, LARGEST>(xv);
                    const u64 q = pb + mbcnt(mb);
                    if (ibb && q < a.band_cap) {
                        dord[q] = o;
                        didx[q] = iv;
                    }
                    sample_append(a, st, ibb && hash_taken(a.seed, tag + 1, iv, hs_T), pack(o, iv));
                    pb += (u64)__popcll(mb);
                }
            }
        }
        if (lane == 0) lds_release(&P.state, 0u);
    };

    u32 cur = tile_of(0u);
    if (cur < nwt) issue(cur);
    // key input: pass 2 of the wave-tile of iteration i runs in iteration
    // i + 2 (q1 = iteration - 2, q0 = iteration - 1)
    u32 q0t = 0, q0a0 = 0, q0a1 = 0, q1t = 0, q1a0 = 0, q1a1 = 0, npend = 0;
    for (u32 it = 0;; ++it) {
        const u32 sl = it % SW_SLOTS;
        u32 ca0 = 0, ca1 = 0;
        if (KIND == 2) {
            // band input: the reservation wait is exposed, band positions need no reload
            if (cur >= nwt) break;
            count_tile(cur, sh.slot[dw][sl], ca0, ca1);
            write_tile(cur, sh.slot[dw][sl], ca0, ca1);
            cur = tile_of(it + 1u);
            asm volatile("" ::: "memory");
            if (cur < nwt) issue(cur);
            continue;
        }
        const bool have = cur < nwt;
        if (have) count_tile(cur, sh.slot[dw][sl], ca0, ca1);
        if (npend == 2) {
            write_tile(q1t, sh.slot[dw][(it + 1) % SW_SLOTS], q1a0, q1a1);
            npend = 1;
        }
        if (!have) {
            if (npend == 1) write_tile(q0t, sh.slot[dw][(it + 2) % SW_SLOTS], q0a0, q0a1);
            break;
        }
        const u32 nxt = tile_of(it + 1u);
        asm volatile("" ::: "memory");   // the next loads stay after pass 2 (register budget)
        if (nxt < nwt) issue(nxt);
        q1t = q0t; q1a0 = q0a0; q1a1 = q0a1;
        q0t = cur; q0a0 = ca0; q0a1 = ca1;
        ++npend;
        cur = nxt;
    }
}

// FIRST only names the instance enqueued for the first round (which reads
// the input) apart from later rounds' instances in profiles.
template <bool IS_F32, bool LARGEST, bool FIRST>
__global__ __launch_bounds__(SW_THREADS) void k_sweep(SelArgs a)
{
    State *st = a.st;
    if (st->phase != PH_SWEEP) return;
    const u32 n = st->n_cur, src = st->src, tag = st->tag;
    __shared__ SwShared sh;
    const Piv p = load_pivots<IS_F32, LARGEST>(st);
    if (src != 0)
        sweep_waves<2, IS_F32, LARGEST, true>(a, st, p, n, src, tag, sh);
    else if (!IS_F32)
        sweep_waves<1, IS_F32, LARGEST, true>(a, st, p, n, src, tag, sh);
    else if (p.fast)
        sweep_waves<0, IS_F32, LARGEST, true>(a, st, p, n, src, tag, sh);
    else
        sweep_waves<0, IS_F32, LARGEST, false>(a, st, p, n, src, tag, sh);
}

// ---------------------------------------------------------------------------
static inline int tm_begin(KernelTimer *tm, int kind, hipStream_t s)
{
    if (!tm || tm->level == 0 || tm->used >= tm->cap) return -1;
    if (tm->level == 1 && kind != KT_SWEEP_FIRST) return -1;
    const int i = tm->used++;
    tm->kind[i] = kind;
    (void)hipEventRecord(tm->ev[2 * i], s);
    return i;
}

static inline void tm_end(KernelTimer *tm, int i, hipStream_t s)
{
    if (i >= 0) (void)hipEventRecord(tm->ev[2 * i + 1], s);
}

template <bool F, bool LG>
hipError_t launch_impl(SelArgs a, const SelLaunch &L, hipStream_t s, KernelTimer *tm)
{
    a.first = 1;
    int t;
    if (a.n <= a.t_fin || L.r_fast <= 0) {
        t = tm_begin(tm, KT_TAIL, s);
        hipLaunchKernelGGL((k_tail<F, LG>), dim3(1), dim3(PV_THREADS), 0, s, a);
        tm_end(tm, t, s);
        return hipGetLastError();
    }
    t = tm_begin(tm, KT_PIVOT_FIRST, s);
    a.presampled = 1;
    hipLaunchKernelGGL((k_sample<F, LG>), dim3(NSEG * SEG_CAP / WAVE), dim3(WAVE), 0, s, a);
    hipLaunchKernelGGL((k_pivot<F, LG>), dim3(1), dim3(PV_THREADS), 0, s, a);
    tm_end(tm, t, s);
    a.first = 0;
    for (int r = 0; r < L.r_fast; ++r) {
        if (r == 0) {
            t = tm_begin(tm, KT_SWEEP_FIRST, s);
            hipLaunchKernelGGL((k_sweep<F, LG, true>), dim3(L.sweep_grid[r]), dim3(SW_THREADS), 0, s, a);
        } else {
            t = tm_begin(tm, KT_SWEEP, s);
            hipLaunchKernelGGL((k_sweep<F, LG, false>), dim3(L.sweep_grid[r]), dim3(SW_THREADS), 0, s, a);
        }
        tm_end(tm, t, s);
        if (r + 1 < L.r_fast) {
            t = tm_begin(tm, KT_PIVOT, s);
            hipLaunchKernelGGL((k_pivot<F, LG>), dim3(1), dim3(PV_THREADS), 0, s, a);
            tm_end(tm, t, s);
        }
    }
    t = tm_begin(tm, KT_TAIL, s);
    hipLaunchKernelGGL((k_tail<F, LG>), dim3(1), dim3(PV_THREADS), 0, s, a);
    tm_end(tm, t, s);
    return hipGetLastError();
}

// Workgroups of k_sweep that fit on one CU at once.
template <bool F, bool LG>
int sweep_blocks_per_cu()
{
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep<F, LG, true>, SW_THREADS, 0);
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

// One key type and order per translation unit.
#define TOPK_INSTANTIATE_SELECT(F, LG)                                                   \
    template hipError_t launch_impl<F, LG>(SelArgs, const SelLaunch &, hipStream_t,     \
                                           KernelTimer *);                              \
    template int sweep_blocks_per_cu<F, LG>();

}  // namespace topk
