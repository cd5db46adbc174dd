// Top-k most frequent objects (§7: PAC and EC) and top-k sum aggregation
// (§8) on one gfx950 device.
//
// One device stands in for the paper's p PEs, so its distributed hash table
// (which spreads objects over PEs) becomes a direct-mapped count table over
// the object universe [0, U) in HBM; each workgroup first aggregates in an
// LDS hash table (the local aggregation §7.4 recommends before insertion)
// and adds its entries to the table with one atomic per object.
//
//   PAC: k_freq_count (Bernoulli sample by per-element Philox decisions,
//        counted by object), the library's own selection of the k largest
//        counts (§7.1 selects with the Algorithm of §2), k_freq_rank.
//   EC:  the same, selecting k* objects, then k_freq_exact (one more sweep
//        counting the k* candidates exactly, LDS hash set) and k_freq_rank
//        of the candidates by exact count.
//   Sum: k_sum_aggregate (sums by key), k_sum_sample (the weighted sample of
//        §8), selection and ranking as PAC or EC, exact sums from the table.
//
// "Most frequent" is the order of §2 with the count as the value: larger
// counts first, ties by ascending object.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

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
};

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
    const u32 ws = wave_sum_u32(taken);
    if (lane_id() == 0 && ws) atomicAdd((unsigned long long *)a.n_sampled, (unsigned long long)ws);
    if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
    __syncthreads();
    fq_table_flush(t, a.counts);
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
    u64 g0, g1;
    fq_range(a.n, g0, g1);
    for (u64 g = g0 + threadIdx.x; g < g1; g += FQ_THREADS) {
        u32 x[4], valid;
        fq_load4(a.keys, g, a.n, x, valid);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if ((valid >> j) & 1u) {
                // load factor <= 1/2: a miss ends at an empty slot
                u32 h = fq_hash(x[j], BITS);
                for (;;) {
                    const u32 kx = skey[h];
                    if (kx == x[j]) { atomicAdd(&scnt[h], 1u); break; }
                    if (kx == FQ_EMPTY) break;
                    h = (h + 1) & (FQ_SET_SLOTS - 1);
                }
            }
        }
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < FQ_SET_SLOTS; i += FQ_THREADS)
        if (skey[i] != FQ_EMPTY && scnt[i]) atomicAdd((unsigned long long *)&a.exact[sidx[i]],
                                                      (unsigned long long)scnt[i]);
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
    const u32 lo = wave_sum_u32((u32)tot), hi = wave_sum_u32((u32)(tot >> 32));
    if (lane_id() == 0) atomicAdd((unsigned long long *)a.total, ((unsigned long long)hi << 32) + lo);
    if (ballot(bad != 0u) && lane_id() == 0) atomicOr(a.status, (u32)TOPK_STATUS_BAD_KEY);
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
__global__ void k_sum_sample(FqArgs a)
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
    const u32 ws = wave_sum_u32(taken);
    if (lane_id() == 0 && ws) atomicAdd((unsigned long long *)a.n_sampled, (unsigned long long)ws);
}

}  // namespace topk

using namespace topk;

namespace {

constexpr size_t FQ_ALIGN = 256;
inline size_t fq_align(size_t x) { return (x + FQ_ALIGN - 1) / FQ_ALIGN * FQ_ALIGN; }

struct FqLayout {
    size_t counts, sums, scal, cand, exact, sel, total;
    size_t sel_bytes;
};

FqLayout fq_layout(const topk_ctx *c, uint32_t U, bool sum)
{
    FqLayout L{};
    size_t off = 0;
    L.counts = off;
    off = fq_align(off + (size_t)U * sizeof(uint32_t));
    L.sums = off;
    if (sum) off = fq_align(off + (size_t)U * sizeof(uint64_t));
    L.scal = off;                   // n_sampled, total, kth key, kth idx
    off = fq_align(off + 64);
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

int fq_grid(const topk_ctx *c) { return c->num_cu * 4; }

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

size_t topk_frequent_workspace_bytes(const topk_ctx *ctx, uint32_t U)
{
    if (!ctx) return 0;
    return fq_layout(ctx, U, false).total;
}

size_t topk_sum_workspace_bytes(const topk_ctx *ctx, uint32_t U)
{
    if (!ctx) return 0;
    return fq_layout(ctx, U, true).total;
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
    const FqLayout L = fq_layout(c, U, false);
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
    if (T >= (1ull << 32))
        hipLaunchKernelGGL((k_freq_count<true>), dim3(grid), dim3(FQ_THREADS), 0, stream, a);
    else
        hipLaunchKernelGGL((k_freq_count<false>), dim3(grid), dim3(FQ_THREADS), 0, stream, a);
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
    const FqLayout L = fq_layout(c, U, true);
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
    hipLaunchKernelGGL(k_sum_aggregate, dim3(grid), dim3(FQ_THREADS), 0, stream, a);
    hipLaunchKernelGGL(k_sum_sample, dim3(grid), dim3(256), 0, stream, a);
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
