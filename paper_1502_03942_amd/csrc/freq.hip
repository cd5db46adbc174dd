// Top-k most frequent objects (§7: PAC and EC) and top-k sum aggregation
// (§8) on one gfx950 device.
//
// One device stands in for the paper's p PEs, so its distributed hash table
// (which spreads objects over PEs) becomes a direct-mapped count table over
// the object universe [0, U) in HBM.  Counting (and summing) by object runs
// in one of two ways:
//   partitioned (U <= 2^25, the default): the elements are first split into
//        partitions by the low bits of the object, then each partition is
//        counted in LDS with a direct counter per object (k_fa_*); no device
//        atomic per element, whatever the skew of the stream;
//   hashed: each workgroup aggregates in an LDS hash table (the local
//        aggregation §7.4 recommends before insertion) and adds its entries
//        to the table with one atomic per object; the objects that miss the
//        table go straight to it (k_freq_count, k_sum_aggregate).
//
//   PAC: the Bernoulli sample (per-element Philox decisions) counted by
//        object, the library's own selection of the k largest counts (§7.1
//        selects with the Algorithm of §2), k_freq_rank.
//   EC:  the same, selecting k* objects, then k_freq_exact (one more sweep
//        counting the k* candidates exactly, LDS hash set) and k_freq_rank
//        of the candidates by exact count.
//   Sum: sums by key, k_sum_sample (the weighted sample of §8), selection
//        and ranking as PAC or EC, exact sums from the table.
//
// "Most frequent" is the order of §2 with the count as the value: larger
// counts first, ties by ascending object.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <type_traits>

#include "common.hpp"
#include "ctx.hpp"
#include "../../include/topk.h"

namespace topk {

typedef uint16_t u16;
typedef u32 fq_u32x4 __attribute__((ext_vector_type(4)));

constexpr int FQ_THREADS = 512;
constexpr u32 FQ_SLOTS = 4096;                  // LDS hash table of a counting workgroup
constexpr u32 FQ_EMPTY = 0xFFFFFFFFu;
constexpr int FQ_PROBES = 8;                    // then the object goes straight to the table
constexpr u32 FQ_KSTAR_MAX = 4096;              // candidates of EC
constexpr u32 FQ_SET_SLOTS = 2 * FQ_KSTAR_MAX;  // LDS hash set of the candidates
constexpr int FQ_RANK_THREADS = 1024;
constexpr u32 FA_BITS = 13, FA_W = 1u << FA_BITS;  // objects per partition (one LDS counter each)
constexpr u32 FA_NB_MAX = 4096;                   // partitions at most: U <= 2^25
constexpr u32 FA_UNIT = 1u << 18;                 // elements per counting unit at most
constexpr u32 FA_UNITS_MAX = (1u << 14) + FA_NB_MAX;   // units at most (n < 2^32)
constexpr u32 FD_COUNT_MAX = 1u << 15;            // direct counting: U at most (counts)
constexpr u32 FD_SUM_MAX = 1u << 14;              // direct counting: U at most (sums)
constexpr int FD_THREADS = 1024;
constexpr int FA_SCAN_P = 64;                     // partitions per scan workgroup

struct FqArgs {
    const u32 *keys;        // objects (u32 < U)
    const u32 *values;      // sum aggregation: value of each object occurrence
    u64 n;
    u32 U, k, kstar;
    u64 T;                  // sampling threshold: rho = T / 2^32 (T >= 2^32: everything)
    u64 seed;
    u32 *counts;            // [U] sample counts (frequent) or weighted samples (sum)
    u64 *sums;              // [U] sums by key (sum aggregation)
    u64 *n_sampled;         // [1]
    u64 *total;             // [1] sum of all values (sum aggregation)
    u32 *cand;              // [kstar] selected objects (selection output, any order)
    u64 *exact;             // [kstar] exact counts (EC) of the candidates
    u32 *out_ids;
    u32 *out_counts;        // frequent: [k] counts
    u64 *out_vals;          // sum: [k] sample counts or exact sums
    u32 *status;
    u64 s_target;           // sum aggregation: desired sample size
    // partitioned counting
    u32 nb_log;             // log2 of the number of partitions NB
    u32 *whist;             // [G][NB] elements per (workgroup, partition), then offsets
    u32 *ptot;              // [NB] partition sizes
    u32 *pstart;            // [NB] partition starts
    u32 *ubase;             // [NB + 1] first unit of each partition
    u32 *unit_part;         // [FA_UNITS_MAX] partition of each unit
    u32 *nunits;            // [1]
    u64 *wsum;              // [G] sum aggregation: values per workgroup
    u16 *pq;                // [n] object index within its partition
    u32 *pv;                // [n] sum aggregation: value
    void *partial;          // per unit (partitioned) or per workgroup (direct): counts / sums
    u64 *wtaken;            // [G] direct counting: sampled elements per workgroup
    u32 *samp;              // [n] partitioned counting of a sample: each workgroup's
                            // sampled objects, from its first element's index on
    u32 *wcount;            // [G] their number
};

// Sum of a u64 over the wave (wave-uniform): three 24-bit pieces, so no
// piece's sum over 64 lanes can overflow 32 bits.
__device__ __forceinline__ u64 fq_wave_sum_u64(u64 x)
{
    const u32 p0 = wave_sum_u32((u32)x & 0xFFFFFFu);
    const u32 p1 = wave_sum_u32((u32)(x >> 24) & 0xFFFFFFu);
    const u32 p2 = wave_sum_u32((u32)(x >> 48));
    return (u64)p0 + ((u64)p1 << 24) + ((u64)p2 << 48);
}

// Add v of every thread of the workgroup (NT threads) to *dst with one device
// atomic per workgroup (atomics on one word serialise across the device).
// Called by every thread; `red` is LDS of NT / 64 words.
template <int NT>
__device__ __forceinline__ void fq_block_add(unsigned long long *dst, u64 v, u64 *red)
{
    const u64 w = fq_wave_sum_u64(v);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int i = 0; i < NT / WAVE; ++i) t += red[i];
        if (t) atomicAdd(dst, (unsigned long long)t);
    }
}

__device__ __forceinline__ u32 fq_hash(u32 key, u32 bits)
{
    return (key * 0x9E3779B1u) >> (32 - bits);     // Fibonacci hashing
}

// Bernoulli decisions of four consecutive positions 4g .. 4g+3 (§2 Bernoulli
// sampling, each independently with probability T / 2^32): word j of
// Philox4x32-10 at counter (g, 0, tag 0, 2), key = seed, below T.
__device__ __forceinline__ u32 fq_take4(u64 g, u64 seed, u64 T)
{
    if (T >= (1ull << 32)) return 0xFu;
    const uint4 r = philox4x32_10(make_uint4((u32)g, 0u, 0u, 2u), (u32)seed, (u32)(seed >> 32));
    return ((u64)r.x < T ? 1u : 0u) | ((u64)r.y < T ? 2u : 0u) | ((u64)r.z < T ? 4u : 0u) |
           ((u64)r.w < T ? 8u : 0u);
}

// ---------------------------------------------------------------------------
// Clear the tables (a kernel, not a memset: the launches stay capturable).
// ---------------------------------------------------------------------------
__global__ void k_freq_clear(FqArgs a)
{
    const u64 i0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 step = (u64)gridDim.x * blockDim.x;
    for (u64 i = i0; i < a.U; i += step) {
        a.counts[i] = 0u;
        if (a.sums) a.sums[i] = 0ull;
    }
    for (u64 i = i0; i < a.kstar; i += step) a.exact[i] = 0ull;
    if (i0 == 0) {
        *a.n_sampled = 0ull;
        if (a.total) *a.total = 0ull;
        *a.status = 0u;
    }
}

// LDS hash table of one workgroup: object -> count (or sum).
template <typename V>
struct FqTable {
    u32 key[FQ_SLOTS];
    V val[FQ_SLOTS];
};

template <typename V>
__device__ __forceinline__ void fq_table_clear(FqTable<V> &t)
{
    for (u32 i = threadIdx.x; i < FQ_SLOTS; i += blockDim.x) {
        t.key[i] = FQ_EMPTY;
        t.val[i] = (V)0;
    }
}

// Add v to object x: in the LDS table when x has (or finds) a slot within
// FQ_PROBES probes, else straight to the device table.
template <typename V>
__device__ __forceinline__ void fq_add(FqTable<V> &t, u32 x, V v, V *dev)
{
    constexpr u32 BITS = 12;
    static_assert((1u << BITS) == FQ_SLOTS, "table size");
    u32 h = fq_hash(x, BITS);
    for (int p = 0; p < FQ_PROBES; ++p) {
        u32 kx = t.key[h];
        if (kx == FQ_EMPTY) kx = atomicCAS(&t.key[h], FQ_EMPTY, x);
        if (kx == FQ_EMPTY || kx == x) {
            atomicAdd(&t.val[h], v);
            return;
        }
        h = (h + 1) & (FQ_SLOTS - 1);
    }
    atomicAdd(&dev[x], v);
}

template <typename V>
__device__ __forceinline__ void fq_table_flush(FqTable<V> &t, V *dev)
{
    for (u32 i = threadIdx.x; i < FQ_SLOTS; i += blockDim.x) {
        const u32 x = t.key[i];
        const V v = t.val[i];
        if (x != FQ_EMPTY && v) atomicAdd(&dev[x], v);
    }
}

// The workgroup's contiguous range of 4-element groups.
__device__ __forceinline__ void fq_range(u64 n, u64 &g0, u64 &g1)
{
    const u64 groups = (n + 3) / 4;
    const u64 per = (groups + gridDim.x - 1) / gridDim.x;
    g0 = (u64)blockIdx.x * per;
    g1 = g0 + per < groups ? g0 + per : groups;
}

// Elements 4g .. 4g+3 (those below n): one 16-byte load when whole.
__device__ __forceinline__ void fq_load4(const u32 *__restrict__ p, u64 g, u64 n, u32 (&x)[4], u32 &valid)
{
    const u64 e = 4 * g;
    if (e + 4 <= n) {
        const fq_u32x4 v = __builtin_nontemporal_load((const fq_u32x4 *)(p + e));
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        valid = 0xFu;
    } else {
        valid = 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            x[j] = e + j < n ? p[e + j] : 0u;
            valid |= (e + j < n ? 1u : 0u) << j;
        }
    }
}

// ---------------------------------------------------------------------------
// PAC / EC step 1 (§7.1): Bernoulli sample, counted by object.
// ---------------------------------------------------------------------------
template <bool ALL>
__global__ __launch_bounds__(FQ_THREADS) void k_freq_count(FqArgs a)
{
    __shared__ FqTable<u32> t;
    fq_table_clear(t);
    __syncthreads();
    u64 g0, g1;
    fq_range(a.n, g0, g1);
    u32 taken = 0, bad = 0;
    for (u64 g = g0 + threadIdx.x; g < g1; g += FQ_THREADS) {
        u32 x[4], valid;
        fq_load4(a.keys, g, a.n, x, valid);
        const u32 take = valid & (ALL ? 0xFu : fq_take4(g, a.seed, a.T));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if ((take >> j) & 1u) {
                if (x[j] < a.U) {
                    fq_add<u32>(t, x[j], 1u, a.counts);
                    ++taken;
                } else {
                    bad = 1u;
                }
            }
        }
    }
    __shared__ u64 red[FQ_THREADS / WAVE];
    if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
    fq_block_add<FQ_THREADS>((unsigned long long *)a.n_sampled, taken, red);
    __syncthreads();
    fq_table_flush(t, a.counts);
}

// ---------------------------------------------------------------------------
// Partitioned counting (and summing) by object.  Partition p of NB (a power
// of two) holds the objects x with x mod NB = p; within it, object x is
// x / NB < FA_W.  Splitting by the low bits puts the most frequent objects of
// a skewed stream (which may well be neighbours) into different partitions.
//   k_fa_hist     per workgroup of the counting grid, the sampled elements
//                 of its range by partition (whist[wg][p]); sums: the
//                 workgroup's total of the values
//   k_fa_scan     whist[.][p] -> offsets within partition p; ptot[p]
//   k_fa_starts   partition starts, the units (at most FA_UNIT elements of
//                 one partition), the sample size and the total of values
//   k_fa_scatter  the same elements (the same decisions) to their partition:
//                 the object's index within it (u16), sums: the value
//   k_fa_count    per unit, a direct LDS counter (sum) per object of the
//                 partition, added to the table (one atomic per object and
//                 unit; stores when the partition is one unit)
// Elements with an object >= U are flagged and left out; sums leave out
// values of 0 (they add nothing).
// ---------------------------------------------------------------------------
// The workgroup's sampled elements with an object below U (sums: and a
// value above 0), f(object, value) each; FA_GB groups of four per thread and
// step, every load of a step issued before the first is used.
constexpr int FA_GB = 4;
template <int NT, bool ALL, bool SUM, class F>
__device__ __forceinline__ void fa_for_taken(const FqArgs &a, F f)
{
    u64 g0, g1;
    fq_range(a.n, g0, g1);
    u32 bad = 0;
    for (u64 gs = g0 + threadIdx.x; gs < g1; gs += (u64)FA_GB * NT) {
        u32 x[FA_GB][4], v[FA_GB][4], valid[FA_GB];
#pragma unroll
        for (int b = 0; b < FA_GB; ++b) {
            const u64 g = gs + (u64)b * NT;
            // a group past the range reads group g0 again (valid: nothing taken)
            fq_load4(a.keys, g < g1 ? g : g0, a.n, x[b], valid[b]);
            if (SUM) fq_load4(a.values, g < g1 ? g : g0, a.n, v[b], valid[b]);
            if (g >= g1) valid[b] = 0u;
        }
#pragma unroll
        for (int b = 0; b < FA_GB; ++b) {
            const u64 g = gs + (u64)b * NT;
            const u32 take = valid[b] & (ALL || !valid[b] ? 0xFu : fq_take4(g, a.seed, a.T));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if ((take >> j) & 1u) {
                    if (x[b][j] >= a.U) bad = 1u;
                    else if (!SUM || v[b][j]) f(x[b][j], SUM ? v[b][j] : 1u);
                }
            }
        }
    }
    if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
}

template <bool ALL, bool SUM>
__global__ __launch_bounds__(FQ_THREADS) void k_fa_hist(FqArgs a)
{
    __shared__ u32 hist[FA_NB_MAX];
    __shared__ u64 wtot[FQ_THREADS / WAVE];
    const u32 NB = 1u << a.nb_log;
    for (u32 i = threadIdx.x; i < NB; i += FQ_THREADS) hist[i] = 0u;
    __syncthreads();
    u64 tot = 0;
    if (ALL) {
        fa_for_taken<FQ_THREADS, ALL, SUM>(a, [&](u32 x, u32 v) {
            atomicAdd(&hist[x & (NB - 1)], 1u);
            tot += v;
        });
    } else {
        // a sample: its objects are also written, compacted, to the
        // workgroup's part of samp[] (pass 2 reads only those)
        __shared__ u32 lcnt;
        if (threadIdx.x == 0) lcnt = 0u;
        __syncthreads();
        u64 g0, g1;
        fq_range(a.n, g0, g1);
        u32 *dst = a.samp + 4 * g0;
        u32 bad = 0;
        for (u64 gb = g0; gb < g1; gb += (u64)FA_GB * FQ_THREADS) {
            u32 x[FA_GB][4], valid[FA_GB];
#pragma unroll
            for (int b = 0; b < FA_GB; ++b) {
                const u64 g = gb + (u64)b * FQ_THREADS + threadIdx.x;
                fq_load4(a.keys, g < g1 ? g : g0, a.n, x[b], valid[b]);
                if (g >= g1) valid[b] = 0u;
            }
#pragma unroll
            for (int b = 0; b < FA_GB; ++b) {
                const u64 g = gb + (u64)b * FQ_THREADS + threadIdx.x;
                const u32 take = valid[b] ? valid[b] & fq_take4(g, a.seed, a.T) : 0u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool tk = (take >> j) & 1u;
                    if (tk && x[b][j] >= a.U) bad = 1u;
                    const bool use = tk && x[b][j] < a.U;
                    if (use) atomicAdd(&hist[x[b][j] & (NB - 1)], 1u);
                    const u64 m = ballot(use);
                    if (m) {
                        u32 base = 0;
                        if (lane_id() == 0) base = atomicAdd(&lcnt, (u32)__popcll(m));
                        base = __builtin_amdgcn_readfirstlane(base);
                        if (use) dst[base + mbcnt(m)] = x[b][j];
                    }
                }
            }
        }
        if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
        __syncthreads();
        if (threadIdx.x == 0) a.wcount[blockIdx.x] = lcnt;
    }
    if (SUM) {
        const u64 t = fq_wave_sum_u64(tot);
        if (lane_id() == 0) wtot[threadIdx.x / WAVE] = t;
    }
    __syncthreads();
    if (SUM && threadIdx.x == 0) {
        u64 t = 0;
        for (int i = 0; i < FQ_THREADS / WAVE; ++i) t += wtot[i];
        a.wsum[blockIdx.x] = t;
    }
    u32 *row = a.whist + (u64)blockIdx.x * NB;
    for (u32 p = threadIdx.x; p < NB; p += FQ_THREADS) row[p] = hist[p];
}

// Workgroup b: partitions [64 b, 64 b + 64); thread (p, segment) walks the
// counting workgroups [seg S, seg S + S) of its partition, S = ceil(G / 16).
__global__ __launch_bounds__(1024) void k_fa_scan(FqArgs a, u32 G)
{
    __shared__ u32 segsum[16][FA_SCAN_P];
    const u32 NB = 1u << a.nb_log;
    const u32 pl = threadIdx.x % FA_SCAN_P, seg = threadIdx.x / FA_SCAN_P;
    const u32 p = blockIdx.x * FA_SCAN_P + pl;
    const u32 S = (G + 15) / 16;
    const u32 w0 = seg * S < G ? seg * S : G, w1 = w0 + S < G ? w0 + S : G;
    u32 sum = 0;
    if (p < NB)
        for (u32 w = w0; w < w1; ++w) sum += a.whist[(u64)w * NB + p];
    segsum[seg][pl] = sum;
    __syncthreads();
    u32 run = 0, tot = 0;
    for (u32 i = 0; i < 16; ++i) {
        const u32 c = segsum[i][pl];
        run += i < seg ? c : 0u;
        tot += c;
    }
    if (p < NB) {
        for (u32 w = w0; w < w1; ++w) {
            u32 *q = a.whist + (u64)w * NB + p;
            const u32 c = *q;
            *q = run;
            run += c;
        }
        if (seg == 0) a.ptot[p] = tot;
    }
}

// One workgroup of 1024 threads: thread t covers partitions [4 t, 4 t + 4).
__global__ __launch_bounds__(1024) void k_fa_starts(FqArgs a, u32 G, u32 sum)
{
    __shared__ u32 scan[1024 / WAVE];
    __shared__ u64 vt[1024 / WAVE];
    const u32 NB = 1u << a.nb_log;
    static_assert(FA_NB_MAX == 4 * 1024, "four partitions per thread");
    u32 c[4], nu[4], cs = 0, us = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const u32 p = 4 * threadIdx.x + (u32)i;
        c[i] = p < NB ? a.ptot[p] : 0u;
        nu[i] = (c[i] + FA_UNIT - 1) / FA_UNIT;
        cs += c[i];
        us += nu[i];
    }
    u32 ctot, utot;
    u32 cb = block_excl_scan<1024>(cs, scan, &ctot);
    u32 ub = block_excl_scan<1024>(us, scan, &utot);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const u32 p = 4 * threadIdx.x + (u32)i;
        if (p < NB) {
            a.pstart[p] = cb;
            a.ubase[p] = ub;
            for (u32 j = 0; j < nu[i]; ++j) a.unit_part[ub + j] = p;
        }
        cb += c[i];
        ub += nu[i];
    }
    if (threadIdx.x == 0) {
        a.ubase[NB] = utot;
        *a.nunits = utot;
        if (!sum) *a.n_sampled = ctot;      // sums: the weighted sample counts it later
    }
    if (sum) {
        u64 t = 0;
        for (u32 w = threadIdx.x; w < G; w += 1024) t += a.wsum[w];
        t = fq_wave_sum_u64(t);
        if (lane_id() == 0) vt[threadIdx.x / WAVE] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 m = 0;
            for (int i = 0; i < 1024 / WAVE; ++i) m += vt[i];
            *a.total = m;
        }
    }
}

// Pass 2 in tiles of FA_TILE elements per workgroup: every element gets its
// rank within its partition in the tile (an LDS atomic), the tile is staged
// in LDS in partition order, then copied out so that each partition's run
// of the tile goes to consecutive positions (stores in runs, not scattered
// over NB regions).
constexpr int FA_TG = 4;                                 // groups of four per thread and tile
constexpr u32 FA_TILE = (u32)FQ_THREADS * 4 * FA_TG;     // 8192 elements
template <bool ALL, bool SUM>
__global__ __launch_bounds__(FQ_THREADS) void k_fa_scatter(FqArgs a)
{
    __shared__ u32 cur[FA_NB_MAX];      // next position of each partition (device)
    __shared__ u32 tcnt[FA_NB_MAX];     // tile: elements per partition, then their start
    __shared__ u32 stage_x[FA_TILE];
    __shared__ u32 stage_v[SUM ? FA_TILE : 1];
    __shared__ u32 scan[FQ_THREADS / WAVE];
    const u32 NB = 1u << a.nb_log, sh = a.nb_log, tid = threadIdx.x;
    const u32 *row = a.whist + (u64)blockIdx.x * NB;
    for (u32 p = tid; p < NB; p += FQ_THREADS) {
        cur[p] = a.pstart[p] + row[p];
        tcnt[p] = 0u;
    }
    __syncthreads();
    // the elements: a sample was compacted by pass 1 (every one taken, every
    // object below U); else the workgroup's range of the input
    u64 g0, g1;
    fq_range(a.n, g0, g1);
    const u32 *src = a.keys;
    u64 nsrc = a.n;
    if (!ALL) {
        src = a.samp + 4 * g0;
        nsrc = a.wcount[blockIdx.x];
        g0 = 0;
        g1 = (nsrc + 3) / 4;
    }
    u32 bad = 0;
    constexpr int E = 4 * FA_TG;
    const u32 per_p = (NB + FQ_THREADS - 1) / FQ_THREADS;   // partitions per thread in the scan
    // (1) the tile's elements; the next tile's loads are issued before this
    // tile is processed
    u32 x[FA_TG][4], v[FA_TG][4], valid[FA_TG];
    auto load_tile = [&](u64 gs, u32 (&xx)[FA_TG][4], u32 (&vv)[FA_TG][4], u32 (&ok)[FA_TG]) {
#pragma unroll
        for (int b = 0; b < FA_TG; ++b) {
            const u64 g = gs + (u64)b * FQ_THREADS + tid;
            fq_load4(src, g < g1 ? g : g0, nsrc, xx[b], ok[b]);
            if (SUM) fq_load4(a.values, g < g1 ? g : g0, a.n, vv[b], ok[b]);
            if (g >= g1) ok[b] = 0u;
        }
    };
    if (g0 < g1) load_tile(g0, x, v, valid);
    for (u64 gs = g0; gs < g1; gs += (u64)FQ_THREADS * FA_TG) {
        u32 xn[FA_TG][4], vn[FA_TG][4], validn[FA_TG];
        const u64 gn = gs + (u64)FQ_THREADS * FA_TG;
        if (gn < g1) load_tile(gn, xn, vn, validn);
        u32 rk[E];
        bool use[E];
#pragma unroll
        for (int b = 0; b < FA_TG; ++b) {
            const u32 take = valid[b];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = 4 * b + j;
                const bool t = (take >> j) & 1u;
                if (t && x[b][j] >= a.U) bad = 1u;
                use[e] = t && x[b][j] < a.U && (!SUM || v[b][j] != 0u);
                // (2) rank within the partition in this tile
                rk[e] = use[e] ? atomicAdd(&tcnt[x[b][j] & (NB - 1)], 1u) : 0u;
            }
        }
        __syncthreads();
        // (3) partition starts within the tile (exclusive scan of tcnt)
        u32 loc = 0;
        for (u32 i = 0; i < per_p; ++i) {
            const u32 p = tid * per_p + i;
            loc += p < NB ? tcnt[p] : 0u;
        }
        u32 ttot;
        u32 run = block_excl_scan<FQ_THREADS, true>(loc, scan, &ttot);
        for (u32 i = 0; i < per_p; ++i) {
            const u32 p = tid * per_p + i;
            if (p < NB) {
                const u32 c = tcnt[p];
                tcnt[p] = run;
                run += c;
            }
        }
        lds_sync();
        // (4) stage in partition order
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (use[e]) {
                const u32 xe = x[e / 4][e % 4];
                const u32 at = tcnt[xe & (NB - 1)] + rk[e];
                stage_x[at] = xe;
                if (SUM) stage_v[at] = v[e / 4][e % 4];
            }
        }
        lds_sync();
        // (5) copy out: slot i of partition p goes to cur[p] + (i - start of p)
        for (u32 i = tid; i < ttot; i += FQ_THREADS) {
            const u32 xe = stage_x[i];
            const u32 p = xe & (NB - 1);
            const u32 pos = cur[p] + (i - tcnt[p]);
            a.pq[pos] = (u16)(xe >> sh);
            if (SUM) a.pv[pos] = stage_v[i];
        }
        lds_sync();
        // (6) advance the cursors, clear the tile counts
        for (u32 i = 0; i < per_p; ++i) {
            const u32 p = tid * per_p + i;
            if (p < NB) {
                const u32 nxt = p + 1 < NB ? tcnt[p + 1] : ttot;
                cur[p] += nxt - tcnt[p];
            }
        }
        lds_sync();
        for (u32 i = 0; i < per_p; ++i) {
            const u32 p = tid * per_p + i;
            if (p < NB) tcnt[p] = 0u;
        }
        lds_sync();
        if (gn < g1) {
#pragma unroll
            for (int b = 0; b < FA_TG; ++b) {
                valid[b] = validn[b];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    x[b][j] = xn[b][j];
                    if (SUM) v[b][j] = vn[b][j];
                }
            }
        }
    }
    if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
}

// ---------------------------------------------------------------------------
// EC step 2 (§7.2): count the k* candidates exactly over the whole input.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(FQ_THREADS) void k_freq_exact(FqArgs a)
{
    constexpr u32 BITS = 13;
    static_assert((1u << BITS) == FQ_SET_SLOTS, "set size");
    __shared__ u32 skey[FQ_SET_SLOTS];
    __shared__ u32 scnt[FQ_SET_SLOTS];
    __shared__ u16 sidx[FQ_SET_SLOTS];
    for (u32 i = threadIdx.x; i < FQ_SET_SLOTS; i += FQ_THREADS) {
        skey[i] = FQ_EMPTY;
        scnt[i] = 0u;
    }
    __syncthreads();
    // the candidates (distinct objects) into the set
    for (u32 c = threadIdx.x; c < a.kstar; c += FQ_THREADS) {
        const u32 x = a.cand[c];
        u32 h = fq_hash(x, BITS);
        while (atomicCAS(&skey[h], FQ_EMPTY, x) != FQ_EMPTY) h = (h + 1) & (FQ_SET_SLOTS - 1);
        sidx[h] = (u16)c;
    }
    __syncthreads();
    // every element (FA_GB groups of four per thread and step, loads first);
    // load factor <= 1/2: a miss ends at an empty slot
    fa_for_taken<FQ_THREADS, true, false>(a, [&](u32 x, u32) {
        u32 h = fq_hash(x, BITS);
        for (;;) {
            const u32 kx = skey[h];
            if (kx == x) { atomicAdd(&scnt[h], 1u); break; }
            if (kx == FQ_EMPTY) break;
            h = (h + 1) & (FQ_SET_SLOTS - 1);
        }
    });
    __syncthreads();
    for (u32 i = threadIdx.x; i < FQ_SET_SLOTS; i += FQ_THREADS)
        if (skey[i] != FQ_EMPTY && scnt[i]) atomicAdd((unsigned long long *)&a.exact[sidx[i]],
                                                      (unsigned long long)scnt[i]);
}

// Count the lanes in `act` into LDS counter q (sums: add v into it).  The
// lanes holding the same object as the wave's first active lane are merged
// into one atomic when there are several (a skewed stream puts most of a
// wave on a few objects, whose LDS atomics would serialise); the rest add
// one by one.
__device__ __forceinline__ void fa_lds_count(u32 *cnt, u32 q, bool act)
{
    const u64 am = ballot(act);
    if (!am) return;
    const int l0 = __builtin_ctzll(am);
    const u32 q0 = (u32)__builtin_amdgcn_readlane((int)q, l0);
    const bool same = act && q == q0;
    const u64 sm = ballot(same);
    if (__popcll(sm) > 1) {
        if ((int)lane_id() == l0) atomicAdd(&cnt[q0], (u32)__popcll(sm));
        act = act && !same;
    }
    if (act) atomicAdd(&cnt[q], 1u);
}

__device__ __forceinline__ void fa_lds_sum(unsigned long long *cnt, u32 q, u32 v, bool act)
{
    const u64 am = ballot(act);
    if (!am) return;
    const int l0 = __builtin_ctzll(am);
    const u32 q0 = (u32)__builtin_amdgcn_readlane((int)q, l0);
    const bool same = act && q == q0;
    const u64 sm = ballot(same);
    if (__popcll(sm) > 1) {
        // the group's values in two 16-bit halves (each wave sum < 2^22)
        const u32 lo = wave_sum_u32(same ? (v & 0xFFFFu) : 0u);
        const u32 hi = wave_sum_u32(same ? (v >> 16) : 0u);
        if ((int)lane_id() == l0) atomicAdd(&cnt[q0], ((unsigned long long)hi << 16) + lo);
        act = act && !same;
    }
    if (act) atomicAdd(&cnt[q], (unsigned long long)v);
}

template <bool SUM>
__global__ __launch_bounds__(FQ_THREADS) void k_fa_count(FqArgs a)
{
    __shared__ unsigned long long lds[SUM ? FA_W : FA_W / 2];
    u32 *cnt = reinterpret_cast<u32 *>(lds);
    unsigned long long *sums = lds;
    const u32 nu = *a.nunits;
    for (u32 u = blockIdx.x; u < nu; u += gridDim.x) {
        const u32 p = a.unit_part[u];
        const u32 tot = a.ptot[p];
        const u32 c0 = (u - a.ubase[p]) * FA_UNIT;
        const u32 s0 = a.pstart[p] + c0;
        const u32 s1 = a.pstart[p] + (tot - c0 < FA_UNIT ? tot : c0 + FA_UNIT);
        for (u32 i = threadIdx.x; i < FA_W; i += FQ_THREADS) {
            if (SUM) sums[i] = 0ull;
            else cnt[i] = 0u;
        }
        __syncthreads();
        // the wave's elements in 64-element columns, FA_CB columns per step
        // (uniform trip count; all loads of a step before the first use)
        constexpr int FA_CB = 16;
        const u32 wv = threadIdx.x / WAVE, ln = lane_id();
        for (u32 b = s0 + wv * WAVE * FA_CB; b < s1; b += FQ_THREADS * FA_CB) {
            u32 q[FA_CB], v[FA_CB];
#pragma unroll
            for (int j = 0; j < FA_CB; ++j) {
                const u32 i = b + (u32)j * WAVE + ln;
                q[j] = i < s1 ? (u32)a.pq[i] : 0u;
                if (SUM) v[j] = i < s1 ? a.pv[i] : 0u;
            }
#pragma unroll
            for (int j = 0; j < FA_CB; ++j) {
                const bool act = b + (u32)j * WAVE + ln < s1;
                if (SUM) fa_lds_sum(sums, q[j], v[j], act);
                else fa_lds_count(cnt, q[j], act);
            }
        }
        __syncthreads();
        // the unit's counters (sums) to its row of partials: coalesced, no atomics
        if (SUM) {
            u64 *row = (u64 *)a.partial + (u64)u * FA_W;
            for (u32 i = threadIdx.x; i < FA_W; i += FQ_THREADS) row[i] = sums[i];
        } else {
            u32 *row = (u32 *)a.partial + (u64)u * FA_W;
            for (u32 i = threadIdx.x; i < FA_W; i += FQ_THREADS) row[i] = cnt[i];
        }
        __syncthreads();
    }
}

// counts[x] (sums[x]) of partition p = x mod NB: the sum of its units' rows
// at x / NB.  Workgroup (p, c) covers q in [256 c, 256 c + 256).
template <bool SUM>
__global__ __launch_bounds__(256) void k_fa_reduce(FqArgs a)
{
    const u32 NB = 1u << a.nb_log, per = FA_W / 256;
    const u32 p = blockIdx.x / per, q = (blockIdx.x % per) * 256 + threadIdx.x;
    const u32 x = (q << a.nb_log) | p;
    if (p >= NB || x >= a.U) return;
    const u32 u0 = a.ubase[p], u1 = a.ubase[p + 1];
    if (SUM) {
        u64 t = 0;
        for (u32 u = u0; u < u1; ++u) t += ((const u64 *)a.partial)[(u64)u * FA_W + q];
        a.sums[x] = t;
    } else {
        u32 t = 0;
        for (u32 u = u0; u < u1; ++u) t += ((const u32 *)a.partial)[(u64)u * FA_W + q];
        a.counts[x] = t;
    }
}

// ---------------------------------------------------------------------------
// Direct counting for small universes (U <= FD_COUNT_MAX counts, FD_SUM_MAX
// sums): every workgroup counts its range into one LDS counter per object
// and writes them as its row of partials; k_fd_reduce adds the rows.  One
// pass over the input, no device atomics.
// ---------------------------------------------------------------------------
template <bool ALL, bool SUM>
__global__ __launch_bounds__(FD_THREADS) void k_fd_count(FqArgs a)
{
    __shared__ unsigned long long lds[FD_COUNT_MAX / 2];
    __shared__ u64 wred[FD_THREADS / WAVE];
    static_assert(FD_SUM_MAX * 8 <= FD_COUNT_MAX * 4, "LDS holds either table");
    u32 *cnt = reinterpret_cast<u32 *>(lds);
    unsigned long long *sums = lds;
    for (u32 i = threadIdx.x; i < a.U; i += FD_THREADS) {
        if (SUM) sums[i] = 0ull;
        else cnt[i] = 0u;
    }
    __syncthreads();
    u64 tot = 0;
    // one LDS atomic per element
    fa_for_taken<FD_THREADS, ALL, SUM>(a, [&](u32 x, u32 v) {
        if (SUM) atomicAdd(&sums[x], (unsigned long long)v);
        else atomicAdd(&cnt[x], 1u);
        tot += SUM ? v : 1u;
    });
    const u64 wt = fq_wave_sum_u64(tot);
    if (lane_id() == 0) wred[threadIdx.x / WAVE] = wt;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int i = 0; i < FD_THREADS / WAVE; ++i) t += wred[i];
        if (SUM) a.wsum[blockIdx.x] = t;
        else a.wtaken[blockIdx.x] = t;
    }
    if (SUM) {
        u64 *row = (u64 *)a.partial + (u64)blockIdx.x * a.U;
        for (u32 i = threadIdx.x; i < a.U; i += FD_THREADS) row[i] = sums[i];
    } else {
        u32 *row = (u32 *)a.partial + (u64)blockIdx.x * a.U;
        for (u32 i = threadIdx.x; i < a.U; i += FD_THREADS) row[i] = cnt[i];
    }
}

// Column x of the partials: workgroup (64 columns) x (4 row segments), each
// thread adds a segment with eight loads in flight, LDS adds the segments.
template <bool SUM>
__global__ __launch_bounds__(256) void k_fd_reduce(FqArgs a, u32 G)
{
    using V = typename std::conditional<SUM, u64, u32>::type;
    __shared__ V part[4][64];
    const u32 c = threadIdx.x % 64, sgm = threadIdx.x / 64;
    const u32 x = blockIdx.x * 64 + c;
    const u32 r0 = sgm * ((G + 3) / 4), r1 = r0 + (G + 3) / 4 < G ? r0 + (G + 3) / 4 : G;
    const V *P = (const V *)a.partial;
    V t = 0;
    if (x < a.U) {
        u32 w = r0;
        for (; w + 8 <= r1; w += 8) {
            V q[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) q[i] = P[(u64)(w + i) * a.U + x];
#pragma unroll
            for (int i = 0; i < 8; ++i) t += q[i];
        }
        for (; w < r1; ++w) t += P[(u64)w * a.U + x];
    }
    part[sgm][c] = t;
    __syncthreads();
    if (sgm == 0 && x < a.U) {
        const V s4 = part[0][c] + part[1][c] + part[2][c] + part[3][c];
        if (SUM) a.sums[x] = s4;
        else a.counts[x] = (u32)s4;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        u64 tt = 0;
        for (u32 w = 0; w < G; ++w) tt += SUM ? a.wsum[w] : a.wtaken[w];
        if (SUM) *a.total = tt;
        else *a.n_sampled = tt;
    }
}

// ---------------------------------------------------------------------------
// Final ranking of m candidates by (value descending, object ascending); the
// first k are written in that order.  One workgroup: each candidate's rank is
// the number of candidates before it (m <= FQ_KSTAR_MAX).
//   MODE 0: values = counts[cand]        (PAC, frequent objects)
//   MODE 1: values = exact[]             (EC, frequent objects)
//   MODE 2: values = counts[cand]        (PAC, sum aggregation: sample counts)
//   MODE 3: values = sums[cand]          (exact sums)
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(FQ_RANK_THREADS) void k_freq_rank(FqArgs a, u32 m)
{
    __shared__ u64 sv[FQ_KSTAR_MAX];
    __shared__ u32 sid[FQ_KSTAR_MAX];
    for (u32 i = threadIdx.x; i < m; i += FQ_RANK_THREADS) {
        const u32 x = a.cand[i];
        sid[i] = x;
        sv[i] = MODE == 1 ? a.exact[i] : MODE == 3 ? a.sums[x] : (u64)a.counts[x];
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < m; i += FQ_RANK_THREADS) {
        const u64 vi = sv[i];
        const u32 xi = sid[i];
        u32 r = 0;
        for (u32 j = 0; j < m; ++j) {
            const u64 vj = sv[j];
            r += (vj > vi || (vj == vi && sid[j] < xi)) ? 1u : 0u;
        }
        if (r < a.k) {
            a.out_ids[r] = xi;
            if (MODE <= 1) a.out_counts[r] = (u32)vi;
            else a.out_vals[r] = vi;
        }
    }
}

// ---------------------------------------------------------------------------
// Sum aggregation (§8): sums by key, then the weighted sample.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(FQ_THREADS) void k_sum_aggregate(FqArgs a)
{
    __shared__ FqTable<unsigned long long> t;
    fq_table_clear(t);
    __syncthreads();
    u64 g0, g1;
    fq_range(a.n, g0, g1);
    u64 tot = 0;
    u32 bad = 0;
    for (u64 g = g0 + threadIdx.x; g < g1; g += FQ_THREADS) {
        u32 x[4], v[4], valid;
        fq_load4(a.keys, g, a.n, x, valid);
        fq_load4(a.values, g, a.n, v, valid);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if ((valid >> j) & 1u) {
                if (x[j] < a.U) {
                    if (v[j]) fq_add<unsigned long long>(t, x[j], (unsigned long long)v[j],
                                                         (unsigned long long *)a.sums);
                    tot += v[j];
                } else {
                    bad = 1u;
                }
            }
        }
    }
    // the total of all values (v_avg = total / s)
    __shared__ u64 red[FQ_THREADS / WAVE];
    if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
    fq_block_add<FQ_THREADS>((unsigned long long *)a.total, tot, red);
    __syncthreads();
    fq_table_flush(t, (unsigned long long *)a.sums);
}

// floor(v s / m) and v s mod m for v <= m < 2^63, s < 2^32: the product is
// accumulated bit by bit of s modulo m (every intermediate stays below 2m).
__device__ __forceinline__ void mul_divmod(u64 v, u64 s, u64 m, u64 &q, u64 &r)
{
    q = 0;
    r = 0;
    for (int b = 31; b >= 0; --b) {
        q <<= 1;
        r <<= 1;
        if (r >= m) { r -= m; q += 1; }
        if ((s >> b) & 1u) {
            r += v;
            if (r >= m) { r -= m; q += 1; }
        }
    }
}

// floor(r 2^32 / m) for r < m < 2^63.
__device__ __forceinline__ u64 frac32(u64 r, u64 m)
{
    u64 q = 0;
    for (int b = 0; b < 32; ++b) {
        r <<= 1;
        q <<= 1;
        if (r >= m) { r -= m; q |= 1u; }
    }
    return q;
}

// Weighted sample (§8 "Sampling"): with v_avg = m / s, key x with sum v gets
// floor(v / v_avg) samples plus one with probability v / v_avg - that; the
// extra one is taken iff word 0 of Philox4x32-10 at counter (x, 0, 0, 3) is
// below floor(r 2^32 / m), r = v s mod m.
constexpr int FQ_SAMPLE_THREADS = 256;
__global__ __launch_bounds__(FQ_SAMPLE_THREADS) void k_sum_sample(FqArgs a)
{
    u64 m = *a.total;
    const u64 i0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >> 63) {                  // outside the exact integer arithmetic below
        if (i0 == 0) atomicOr(a.status, (u32)TOPK_STATUS_SUM_RANGE);
        m = 0;
    }
    const u64 step = (u64)gridDim.x * blockDim.x;
    u32 taken = 0;
    for (u64 x = i0; x < a.U; x += step) {
        u32 c = 0;
        const u64 v = a.sums[x];
        if (m && v) {
            u64 q, r;
            mul_divmod(v, a.s_target, m, q, r);
            const uint4 w = philox4x32_10(make_uint4((u32)x, 0u, 0u, 3u), (u32)a.seed, (u32)(a.seed >> 32));
            c = (u32)q + ((u64)w.x < frac32(r, m) ? 1u : 0u);
        }
        a.counts[x] = c;
        taken += c;
    }
    __shared__ u64 red[FQ_SAMPLE_THREADS / WAVE];
    fq_block_add<FQ_SAMPLE_THREADS>((unsigned long long *)a.n_sampled, taken, red);
}

}  // namespace topk

using namespace topk;

namespace {

constexpr size_t FQ_ALIGN = 256;
inline size_t fq_align(size_t x) { return (x + FQ_ALIGN - 1) / FQ_ALIGN * FQ_ALIGN; }

int fq_grid(const topk_ctx *c) { return c->num_cu * 4; }

// How the table is filled: context parameter "fq_mode" 0 picks by U (direct
// counting for small universes, partitioned up to FA_NB_MAX partitions, else
// hashed); 1 hashed; 2 partitioned (hashed beyond it); 3 direct (else as 0).
enum FqMethod { FQ_HASHED, FQ_PARTITIONED, FQ_DIRECT };
FqMethod fq_method(const topk_ctx *c, uint32_t U, bool sum)
{
    const bool direct_ok = U <= (sum ? FD_SUM_MAX : FD_COUNT_MAX);
    const bool part_ok = (uint64_t)U <= (uint64_t)FA_NB_MAX * FA_W;
    switch (c->fq_mode) {
    case 1: return FQ_HASHED;
    case 2: return part_ok ? FQ_PARTITIONED : FQ_HASHED;
    default: return direct_ok ? FQ_DIRECT : part_ok ? FQ_PARTITIONED : FQ_HASHED;
    }
}

int fq_nb_log(uint32_t U)
{
    const uint32_t need = (U + FA_W - 1) / FA_W;
    int l = 0;
    while ((1u << l) < need) ++l;
    return l;
}

struct FqLayout {
    size_t counts, sums, scal, cand, exact, sel, total;
    size_t sel_bytes;
    FqMethod method;
    int nb_log;
    size_t whist, ptot, pstart, ubase, unit_part, wsum, wtaken, pq, pv, partial, samp, wcount;
};

FqLayout fq_layout(const topk_ctx *c, uint64_t n, uint32_t U, bool sum)
{
    FqLayout L{};
    size_t off = 0;
    L.counts = off;
    off = fq_align(off + (size_t)U * sizeof(uint32_t));
    L.sums = off;
    if (sum) off = fq_align(off + (size_t)U * sizeof(uint64_t));
    L.scal = off;                   // n_sampled, total, kth key, kth idx, units
    off = fq_align(off + 64);
    L.method = fq_method(c, U, sum);
    L.nb_log = L.method == FQ_PARTITIONED ? fq_nb_log(U) : -1;
    const size_t vb = sum ? sizeof(uint64_t) : sizeof(uint32_t);
    if (L.method == FQ_DIRECT) {
        const size_t G = (size_t)c->num_cu;
        L.wsum = off;
        off = fq_align(off + G * sizeof(uint64_t));
        L.wtaken = off;
        off = fq_align(off + G * sizeof(uint64_t));
        L.partial = off;
        off = fq_align(off + G * (size_t)U * vb);
    }
    if (L.method == FQ_PARTITIONED) {
        const size_t NB = (size_t)1 << L.nb_log, G = (size_t)fq_grid(c);
        L.whist = off;
        off = fq_align(off + G * NB * sizeof(uint32_t));
        L.ptot = off;
        off = fq_align(off + NB * sizeof(uint32_t));
        L.pstart = off;
        off = fq_align(off + NB * sizeof(uint32_t));
        L.ubase = off;
        off = fq_align(off + (NB + 1) * sizeof(uint32_t));
        L.unit_part = off;
        off = fq_align(off + FA_UNITS_MAX * sizeof(uint32_t));
        L.wsum = off;
        off = fq_align(off + G * sizeof(uint64_t));
        L.pq = off;
        off = fq_align(off + (size_t)n * sizeof(uint16_t));
        L.pv = off;
        if (sum) off = fq_align(off + (size_t)n * sizeof(uint32_t));
        const size_t units = (size_t)((n + FA_UNIT - 1) / FA_UNIT) + NB;
        L.partial = off;
        off = fq_align(off + units * FA_W * vb);
        if (!sum) {                 // a sample's objects, compacted per workgroup
            L.samp = off;
            off = fq_align(off + (size_t)n * sizeof(uint32_t));
            L.wcount = off;
            off = fq_align(off + G * sizeof(uint32_t));
        }
    }
    L.cand = off;
    off = fq_align(off + FQ_KSTAR_MAX * sizeof(uint32_t));
    L.exact = off;
    off = fq_align(off + FQ_KSTAR_MAX * sizeof(uint64_t));
    L.sel = off;
    L.sel_bytes = topk_workspace_bytes(c, U, 0);
    off = fq_align(off + L.sel_bytes);
    L.total = off;
    return L;
}

// Point the partitioned-counting fields of `a` into the workspace.
void fq_bind_partitioned(FqArgs &a, const FqLayout &L, char *w)
{
    a.nb_log = (u32)L.nb_log;
    a.whist = (u32 *)(w + L.whist);
    a.ptot = (u32 *)(w + L.ptot);
    a.pstart = (u32 *)(w + L.pstart);
    a.ubase = (u32 *)(w + L.ubase);
    a.unit_part = (u32 *)(w + L.unit_part);
    a.nunits = (u32 *)(w + L.scal + 32);
    a.wsum = (u64 *)(w + L.wsum);
    a.pq = (u16 *)(w + L.pq);
    a.pv = (u32 *)(w + L.pv);
    a.partial = w + L.partial;
    a.samp = (u32 *)(w + L.samp);
    a.wcount = (u32 *)(w + L.wcount);
}

void fq_bind_direct(FqArgs &a, const FqLayout &L, char *w)
{
    a.wsum = (u64 *)(w + L.wsum);
    a.wtaken = (u64 *)(w + L.wtaken);
    a.partial = w + L.partial;
}

template <bool ALL, bool SUM>
void fq_count_direct(const topk_ctx *c, const FqArgs &a, hipStream_t stream)
{
    const int G = c->num_cu;
    hipLaunchKernelGGL((k_fd_count<ALL, SUM>), dim3(G), dim3(FD_THREADS), 0, stream, a);
    hipLaunchKernelGGL((k_fd_reduce<SUM>), dim3((a.U + 63) / 64), dim3(256), 0, stream, a, (u32)G);
}

// The partitioned counting of the (sampled) elements into a.counts (sums:
// a.sums and a.total); a.counts / a.sums are clear.
template <bool ALL, bool SUM>
void fq_count_partitioned(const topk_ctx *c, const FqArgs &a, hipStream_t stream)
{
    const int G = fq_grid(c);
    const u32 NB = 1u << a.nb_log;
    hipLaunchKernelGGL((k_fa_hist<ALL, SUM>), dim3(G), dim3(FQ_THREADS), 0, stream, a);
    hipLaunchKernelGGL(k_fa_scan, dim3((NB + FA_SCAN_P - 1) / FA_SCAN_P), dim3(1024), 0, stream, a, (u32)G);
    hipLaunchKernelGGL(k_fa_starts, dim3(1), dim3(1024), 0, stream, a, (u32)G, SUM ? 1u : 0u);
    hipLaunchKernelGGL((k_fa_scatter<ALL, SUM>), dim3(G), dim3(FQ_THREADS), 0, stream, a);
    hipLaunchKernelGGL((k_fa_count<SUM>), dim3(c->num_cu * 4), dim3(FQ_THREADS), 0, stream, a);
    hipLaunchKernelGGL((k_fa_reduce<SUM>), dim3(NB * (FA_W / 256)), dim3(256), 0, stream, a);
}

// Shared part of both problems: select the kk objects with the largest
// counts[] (ties by ascending object: the selection's position rule) into
// a.cand, in any order.
int fq_select(topk_ctx *c, const FqArgs &a, const FqLayout &L, char *w, uint32_t kk,
              hipStream_t stream)
{
    uint32_t *kth = (uint32_t *)(w + L.scal + 16);
    return topk_select_u32(c, a.counts, a.U, kk, TOPK_LARGEST, a.cand, nullptr, kth, kth + 1,
                           nullptr, w + L.sel, L.sel_bytes, stream);
}

}  // namespace

extern "C" {

size_t topk_frequent_workspace_bytes(const topk_ctx *ctx, uint64_t n, uint32_t U)
{
    if (!ctx) return 0;
    return fq_layout(ctx, n, U, false).total;
}

size_t topk_sum_workspace_bytes(const topk_ctx *ctx, uint64_t n, uint32_t U)
{
    if (!ctx) return 0;
    return fq_layout(ctx, n, U, true).total;
}

int topk_frequent_u32(topk_ctx *c, const uint32_t *keys, uint64_t n, uint32_t U, uint32_t k,
                      uint32_t kstar, uint64_t T, uint32_t *out_ids, uint32_t *out_counts,
                      uint32_t *sample_counts, uint64_t *n_sampled, uint32_t *status,
                      void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!c || !keys || !out_ids || !out_counts || !status || !workspace) return TOPK_E_INVALID;
    if (n == 0 || n > 0xFFFFFFFFull || U == 0 || k == 0 || k > U || k > FQ_KSTAR_MAX ||
        U > 0x80000000u)
        return TOPK_E_INVALID;
    if (kstar != 0 && (kstar < k || kstar > U || kstar > FQ_KSTAR_MAX)) return TOPK_E_INVALID;
    if (T == 0 || T > (1ull << 32)) return TOPK_E_INVALID;
    if (((uintptr_t)keys & 15u) || ((uintptr_t)workspace & (FQ_ALIGN - 1))) return TOPK_E_INVALID;
    const FqLayout L = fq_layout(c, n, U, false);
    if (ws_bytes < L.total) return TOPK_E_WORKSPACE;
    char *w = (char *)workspace;
    FqArgs a{};
    a.keys = keys;
    a.n = n;
    a.U = U;
    a.k = k;
    a.kstar = kstar;
    a.T = T;
    a.seed = c->seed;
    a.counts = sample_counts ? sample_counts : (u32 *)(w + L.counts);
    a.n_sampled = n_sampled ? n_sampled : (u64 *)(w + L.scal);
    a.cand = (u32 *)(w + L.cand);
    a.exact = (u64 *)(w + L.exact);
    a.out_ids = out_ids;
    a.out_counts = out_counts;
    a.status = status;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    const int grid = fq_grid(c);
    hipLaunchKernelGGL(k_freq_clear, dim3(grid), dim3(256), 0, stream, a);
    if (L.method == FQ_DIRECT) {
        fq_bind_direct(a, L, w);
        if (T >= (1ull << 32)) fq_count_direct<true, false>(c, a, stream);
        else fq_count_direct<false, false>(c, a, stream);
    } else if (L.method == FQ_PARTITIONED) {
        fq_bind_partitioned(a, L, w);
        if (T >= (1ull << 32)) fq_count_partitioned<true, false>(c, a, stream);
        else fq_count_partitioned<false, false>(c, a, stream);
    } else if (T >= (1ull << 32)) {
        hipLaunchKernelGGL((k_freq_count<true>), dim3(grid), dim3(FQ_THREADS), 0, stream, a);
    } else {
        hipLaunchKernelGGL((k_freq_count<false>), dim3(grid), dim3(FQ_THREADS), 0, stream, a);
    }
    if (hipGetLastError() != hipSuccess) return TOPK_E_HIP;
    const uint32_t kk = kstar ? kstar : k;
    int rc = fq_select(c, a, L, w, kk, stream);
    if (rc != TOPK_OK) return rc;
    if (kstar) {
        hipLaunchKernelGGL(k_freq_exact, dim3(grid), dim3(FQ_THREADS), 0, stream, a);
        hipLaunchKernelGGL((k_freq_rank<1>), dim3(1), dim3(FQ_RANK_THREADS), 0, stream, a, kk);
    } else {
        hipLaunchKernelGGL((k_freq_rank<0>), dim3(1), dim3(FQ_RANK_THREADS), 0, stream, a, kk);
    }
    return hipGetLastError() == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}

int topk_sum_top_u32(topk_ctx *c, const uint32_t *keys, const uint32_t *values, uint64_t n,
                     uint32_t U, uint32_t k, uint32_t kstar, uint64_t s, uint32_t *out_ids,
                     uint64_t *out_vals, uint64_t *sums, uint32_t *samples, uint32_t *status,
                     void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!c || !keys || !values || !out_ids || !out_vals || !status || !workspace)
        return TOPK_E_INVALID;
    if (n == 0 || n > 0xFFFFFFFFull || U == 0 || k == 0 || k > U || k > FQ_KSTAR_MAX ||
        U > 0x80000000u)
        return TOPK_E_INVALID;
    if (kstar != 0 && (kstar < k || kstar > U || kstar > FQ_KSTAR_MAX)) return TOPK_E_INVALID;
    if (s == 0 || s > 0x7FFFFFFFull) return TOPK_E_INVALID;
    if (((uintptr_t)keys & 15u) || ((uintptr_t)values & 15u) ||
        ((uintptr_t)workspace & (FQ_ALIGN - 1)))
        return TOPK_E_INVALID;
    const FqLayout L = fq_layout(c, n, U, true);
    if (ws_bytes < L.total) return TOPK_E_WORKSPACE;
    char *w = (char *)workspace;
    FqArgs a{};
    a.keys = keys;
    a.values = values;
    a.n = n;
    a.U = U;
    a.k = k;
    a.kstar = kstar;
    a.seed = c->seed;
    a.s_target = s;
    a.counts = samples ? samples : (u32 *)(w + L.counts);
    a.sums = sums ? sums : (u64 *)(w + L.sums);
    a.n_sampled = (u64 *)(w + L.scal);
    a.total = (u64 *)(w + L.scal + 8);
    a.cand = (u32 *)(w + L.cand);
    a.exact = (u64 *)(w + L.exact);
    a.out_ids = out_ids;
    a.out_vals = out_vals;
    a.status = status;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    const int grid = fq_grid(c);
    hipLaunchKernelGGL(k_freq_clear, dim3(grid), dim3(256), 0, stream, a);
    if (L.method == FQ_DIRECT) {
        fq_bind_direct(a, L, w);
        fq_count_direct<true, true>(c, a, stream);
    } else if (L.method == FQ_PARTITIONED) {
        fq_bind_partitioned(a, L, w);
        fq_count_partitioned<true, true>(c, a, stream);
    } else {
        hipLaunchKernelGGL(k_sum_aggregate, dim3(grid), dim3(FQ_THREADS), 0, stream, a);
    }
    hipLaunchKernelGGL(k_sum_sample, dim3(grid), dim3(FQ_SAMPLE_THREADS), 0, stream, a);
    if (hipGetLastError() != hipSuccess) return TOPK_E_HIP;
    const uint32_t kk = kstar ? kstar : k;
    int rc = fq_select(c, a, L, w, kk, stream);
    if (rc != TOPK_OK) return rc;
    if (kstar)
        hipLaunchKernelGGL((k_freq_rank<3>), dim3(1), dim3(FQ_RANK_THREADS), 0, stream, a, kk);
    else
        hipLaunchKernelGGL((k_freq_rank<2>), dim3(1), dim3(FQ_RANK_THREADS), 0, stream, a, kk);
    return hipGetLastError() == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}

// Expected sample sizes of §7 and §8 for an (eps, delta)-approximation.
double topk_sample_size(int method, uint64_t n, uint32_t k, uint32_t kstar, double eps,
                        double delta)
{
    if (n == 0 || !(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0)) return -1.0;
    const double dn = (double)n;
    switch (method) {
    case TOPK_SAMPLE_PAC: {
        if (k == 0) return -1.0;
        const double a = 3.0 / k * log(4.0 * dn / delta), b = 2.0 * log(2.0 * k / delta);
        return 4.0 / (eps * eps) * (a > b ? a : b);
    }
    case TOPK_SAMPLE_EC:
        if (kstar == 0) return -1.0;
        return 2.0 / (eps * eps * kstar) * log(dn / delta);
    case TOPK_SAMPLE_SUM:
        return 1.0 / eps * sqrt(2.0 * log(2.0 * dn / delta));
    default:
        return -1.0;
    }
}

uint64_t topk_sample_threshold(uint64_t n, double sample_size)
{
    if (n == 0 || !(sample_size > 0.0)) return 1ull << 32;
    const double t = ceil(sample_size * 4294967296.0 / (double)n);
    if (!(t < 4294967296.0)) return 1ull << 32;
    return t < 1.0 ? 1ull : (uint64_t)t;
}

}  // extern "C"
