// Selection over locally sorted input on one gfx950 device:
//   msSelect  (§4.2, Appendix A, Algorithm "musel"): the object of global
//             rank k among p sorted sequences, by quickselect with random
//             pivots located by binary search in every sequence;
//   amsSelect (§4.3, Algorithm "approxMusel"): the k smallest objects for some
//             k in [kmin, kmax], the pivot being the minimum (or maximum) of a
//             geometric-deviate sample of the sequences.
// Both run d trials per round together (§4.3 "Multiple Concurrent Trials",
// Theorem "vectorMusel"): d pivots are located at once, and the recursion
// continues between the best pivot below the target and the best one above.
//
// The sequences are the rows of a CSR batch; an object is identified by its
// position in the concatenation, so the order is (value, position) as in §2
// and a row sorted by value is sorted in it.  The result is a prefix of every
// row ("split": the selected length per row).  One workgroup of 1024 threads
// runs every round (thread t owns rows t, t + 1024, ...); the path is bound
// by the latency of the dependent binary-search loads, so every thread keeps
// the loads of all its (row, pivot) searches in flight together.
#include <hip/hip_runtime.h>
#include <math.h>

#include "common.hpp"
#include "ctx.hpp"
#include "../../include/topk.h"

namespace topk {

constexpr int MS_THREADS = 1024;
constexpr int MS_ITEMS = 8;                  // (row, pivot) searches per thread per round
constexpr u32 MS_ROWS_MAX = 8192;
constexpr u32 MS_ROUND_CAP = 1u << 20;       // a failsafe: every exact round removes a pivot
constexpr u32 AMS_ROUNDS = 64;               // flexible rounds before the exact finish

struct MsArgs {
    const u32 *keys;
    const u64 *row_off;
    u32 p;
    u64 k, kmin, kmax;
    u64 seed;
    u32 *split;          // [p]
    u32 *kth_pos;        // [1] msSelect: position of the object of rank k
    u32 *kth_key;        // [1] its key bits
    u64 *k_out;          // [1] amsSelect: the k chosen (the sum of the split)
    u32 *rounds;         // [1] or null
    u32 *status;
};

struct MsShared {
    u64 piv[MS_ITEMS];        // pivot objects: ord << 32 | position
    u32 prow[MS_ITEMS];       // row of each pivot
    u32 cnt[MS_ITEMS];        // active objects below (exact) / at or below (flexible) a pivot
    u64 rnd[MS_ITEMS];        // exact: pivot ranks among the active objects
    u32 scan[MS_THREADS / WAVE];
    int hit, ilo, ihi;        // decision of the round
    double rho;
    int maxmode;              // flexible: 1 = max-based estimator
};

template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ u64 ms_elem(const u32 *__restrict__ keys, u64 base, u32 pos)
{
    return pack(key_ord<IS_F32, LARGEST>(keys[base + pos]), (u32)(base + pos));
}

// For every item e (row q = e / D, pivot i = e % D): the first position in
// the row window [L[e], H[e]) whose object is not below v_i (UPPER: not at
// or below v_i), i.e. lower (upper) bound.  The loads of all items of a
// step are issued before any is compared.
template <bool IS_F32, bool LARGEST, bool UPPER, int QR, int D>
__device__ __forceinline__ void ms_bounds(const u32 *__restrict__ keys, const u64 (&base)[QR],
                                          u32 (&L)[QR * D], u32 (&H)[QR * D], const u64 *v)
{
    for (int step = 0; step < 33; ++step) {
        u32 x[QR * D];
        bool any = false;
#pragma unroll
        for (int e = 0; e < QR * D; ++e) {
            const u32 mid = (L[e] + H[e]) >> 1;
            x[e] = L[e] < H[e] ? keys[base[e / D] + mid] : 0u;
            any = any || L[e] < H[e];
        }
        if (!any) break;
#pragma unroll
        for (int e = 0; e < QR * D; ++e) {
            if (L[e] < H[e]) {
                const u32 mid = (L[e] + H[e]) >> 1;
                const u64 el = pack(key_ord<IS_F32, LARGEST>(x[e]), (u32)(base[e / D] + mid));
                const bool right = UPPER ? el <= v[e % D] : el < v[e % D];
                if (right) L[e] = mid + 1; else H[e] = mid;
            }
        }
    }
}

__global__ void k_clear_word(u32 *w) { *w = 0u; }

template <bool IS_F32, bool LARGEST, int QR, bool FLEX>
__global__ __launch_bounds__(MS_THREADS) void k_msselect(MsArgs a)
{
    constexpr int D = MS_ITEMS / QR;
    __shared__ MsShared sh;
    __shared__ u32 has[MS_ITEMS];            // flexible: some row sampled for the trial
    const u32 tid = threadIdx.x, lane = lane_id();
    u64 base[QR];
    u32 lo[QR], hi[QR];
    bool own[QR];
    // n: the objects of all rows (contiguous: row_off[p] - row_off[0]); the
    // positions must fit 32 bits
    const u64 first = a.row_off[0], end = a.row_off[a.p];
    const u64 n = end - first;
    bool exact = !FLEX;
    u64 k_cur = a.k, kmin = a.kmin, kmax = a.kmax;
    const bool bad = end > 0xFFFFFFFFull ||
                     (FLEX ? (kmin == 0 || kmin > kmax || kmin > n) : (k_cur == 0 || k_cur > n));
    if (bad) {
        if (tid == 0) *a.status = TOPK_STATUS_BAD_ARG;
        return;
    }
    if (FLEX && kmax > n) kmax = n;
#pragma unroll
    for (int q = 0; q < QR; ++q) {
        const u32 r = tid + (u32)q * MS_THREADS;
        own[q] = r < a.p;
        base[q] = own[q] ? a.row_off[r] : 0ull;
        const u32 len = own[q] ? (u32)(a.row_off[r + 1] - base[q]) : 0u;
        lo[q] = 0;
        // msSelect needs only the first k objects of each sequence
        hi[q] = (!FLEX && (u64)len > k_cur) ? (u32)k_cur : len;
    }
    u32 fl_round = 0;
    for (u32 round = 0;; ++round) {
        if (round >= MS_ROUND_CAP) {
            if (tid == 0) *a.status = TOPK_STATUS_INTERNAL;
            return;
        }
        // active objects of this thread's rows, their prefix over the workgroup
        u32 mine = 0;
#pragma unroll
        for (int q = 0; q < QR; ++q) mine += hi[q] - lo[q];
        u32 total;
        const u32 excl = block_excl_scan<MS_THREADS>(mine, sh.scan, &total);
        if (tid < MS_ITEMS) {
            // exact: every pivot is written by its owner; flexible: set with
            // the estimator below (it depends on the mode)
            sh.cnt[tid] = 0u;
            has[tid] = 0u;
        }
        if (exact && total == 1) {
            // the one active object is the answer (k_cur = 1)
#pragma unroll
            for (int q = 0; q < QR; ++q) {
                if (!own[q]) continue;
                const bool one = hi[q] - lo[q] == 1;
                if (one && a.kth_pos) {             // (the flexible call has no k-th object output)
                    const u32 pos = (u32)(base[q] + lo[q]);
                    *a.kth_pos = pos;
                    *a.kth_key = a.keys[pos];
                }
                a.split[tid + (u32)q * MS_THREADS] = lo[q] + (one ? 1u : 0u);
            }
            if (tid == 0 && a.rounds) *a.rounds = round;
            if (FLEX) {
                // only reached after the flexible rounds were spent: k = kmin
                u32 s = 0;
#pragma unroll
                for (int q = 0; q < QR; ++q)
                    if (own[q]) s += lo[q] + ((hi[q] - lo[q] == 1) ? 1u : 0u);
                u32 tot;
                (void)block_excl_scan<MS_THREADS>(s, sh.scan, &tot);
                if (tid == 0) *a.k_out = tot;
            }
            return;
        }
        bool none[D];
        if (exact) {
            // d pivots uniformly among the active objects: ranks from
            // Philox4x32-10 at counter (round, i, 0, 6), key = seed
            if (tid < (u32)D) {
                const uint4 w = philox4x32_10(make_uint4(round, tid, 0u, 6u), (u32)a.seed, (u32)(a.seed >> 32));
                sh.rnd[tid] = __umul64hi(((u64)w.x << 32) | w.y, (u64)total);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const u64 u = sh.rnd[i];
                if (u >= excl && u < (u64)excl + mine) {
                    u32 off = (u32)(u - excl);
                    bool found = false;
#pragma unroll
                    for (int q = 0; q < QR; ++q) {
                        const u32 wq = hi[q] - lo[q];
                        if (!found && off < wq) {
                            sh.piv[i] = ms_elem<IS_F32, LARGEST>(a.keys, base[q], lo[q] + off);
                            sh.prow[i] = tid + (u32)q * MS_THREADS;
                            found = true;
                        } else if (!found) {
                            off -= wq;
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < D; ++i) none[i] = false;
        } else {
            // flexible: the estimator of Algorithm "approxMusel" per trial
            if (tid == 0) {
                const double dn = (double)total, dmin = (double)kmin, dmax = (double)kmax;
                const bool mx = !(dmin < dn - dmax);
                double rho;
                if (!mx) rho = 1.0 - pow((dmin - 1.0) / dmax, 1.0 / (dmax - dmin + 1.0));
                else if (dn - dmax <= 0.0) rho = 1.0;
                else rho = 1.0 - pow((dn - dmax) / (dn - dmin + 1.0), 1.0 / (dmax - dmin + 1.0));
                sh.rho = rho;
                sh.maxmode = mx ? 1 : 0;
                // the identity of the trial reductions: -inf for the maximum,
                // +inf for the minimum
                for (int i = 0; i < MS_ITEMS; ++i) sh.piv[i] = mx ? 0ull : ~0ull;
            }
            __syncthreads();
            const double rho = sh.rho;
            const bool mx = sh.maxmode != 0;
            const double l1 = rho < 1.0 ? log1p(-rho) : 0.0;
            u64 best[D];
            bool got[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                best[i] = mx ? 0ull : ~0ull;
                got[i] = false;
            }
#pragma unroll
            for (int q = 0; q < QR; ++q) {
                if (!own[q] || hi[q] == lo[q]) continue;
                const u32 r = tid + (u32)q * MS_THREADS;
#pragma unroll
                for (int i0 = 0; i0 < D; i0 += 4) {
                    // geometric deviates x on {1, 2, ...} (rank of the first
                    // object of a Bernoulli(rho) sample of the row, from its
                    // start or its end): Philox4x32-10 at counter
                    // (row, round, trial / 4, 7), key = seed; x = 1 +
                    // floor(ln U / ln(1 - rho))
                    const uint4 w = philox4x32_10(make_uint4(r, round, (u32)i0 >> 2, 7u), (u32)a.seed,
                                                  (u32)(a.seed >> 32));
                    const u32 ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int i = i0 + t;
                        if (i >= D) continue;
                        u64 x = 1;
                        if (rho < 1.0) {
                            const double u = ((double)ws[t] + 0.5) * (1.0 / 4294967296.0);
                            const double g = floor(log(u) / l1);
                            x = g >= 4294967296.0 ? (1ull << 32) : 1ull + (u64)g;
                        }
                        const u32 wq = hi[q] - lo[q];
                        if (x <= wq) {
                            const u32 pos = mx ? hi[q] - (u32)x : lo[q] + (u32)x - 1u;
                            const u64 el = ms_elem<IS_F32, LARGEST>(a.keys, base[q], pos);
                            best[i] = mx ? (el > best[i] ? el : best[i]) : (el < best[i] ? el : best[i]);
                            got[i] = true;
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const u64 b = mx ? wave_max_u64(best[i]) : wave_min_u64(best[i]);
                const bool g = ballot(got[i]) != 0;
                if (lane == 0 && g) {
                    if (mx) atomicMax((unsigned long long *)&sh.piv[i], (unsigned long long)b);
                    else atomicMin((unsigned long long *)&sh.piv[i], (unsigned long long)b);
                    has[i] = 1u;
                }
            }
            __syncthreads();
            // no sample in a trial: its minimum is +inf, which the initial
            // value ~0 already is (every active object lies at or below it);
            // its maximum is -inf: no object lies at or below it, so its
            // windows are emptied before the search
#pragma unroll
            for (int i = 0; i < D; ++i) none[i] = mx && has[i] == 0u;
        }
        // locate every pivot in every own row: lower bound (exact: the
        // objects below the pivot) or upper bound (flexible: at or below it)
        u32 L[QR * D], H[QR * D];
#pragma unroll
        for (int e = 0; e < QR * D; ++e) {
            L[e] = own[e / D] ? lo[e / D] : 0u;
            H[e] = (own[e / D] && !none[e % D]) ? hi[e / D] : L[e];
        }
        if (exact) ms_bounds<IS_F32, LARGEST, false, QR, D>(a.keys, base, L, H, sh.piv);
        else ms_bounds<IS_F32, LARGEST, true, QR, D>(a.keys, base, L, H, sh.piv);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            u32 c = 0;
#pragma unroll
            for (int q = 0; q < QR; ++q) c += own[q] ? L[q * D + i] - lo[q] : 0u;
            c = wave_sum_u32(c);
            if (lane == 0 && c) atomicAdd(&sh.cnt[i], c);
        }
        __syncthreads();
        if (tid == 0) {
            int hit = -1, ilo = -1, ihi = -1;
            u32 clo = 0, chi = 0;
            for (int i = 0; i < D; ++i) {
                const u32 c = sh.cnt[i];
                if (exact) {
                    // the pivot has rank c + 1 among the active objects
                    if ((u64)c + 1 == k_cur) { if (hit < 0) hit = i; }
                    else if ((u64)c + 1 < k_cur) { if (ilo < 0 || c > clo) { ilo = i; clo = c; } }
                    else if (ihi < 0 || c < chi) { ihi = i; chi = c; }
                } else {
                    if (c >= kmin && c <= kmax) { if (hit < 0) hit = i; }
                    else if (c < kmin) { if (ilo < 0 || c > clo) { ilo = i; clo = c; } }
                    else if (ihi < 0 || c < chi) { ihi = i; chi = c; }
                }
            }
            sh.hit = hit;
            sh.ilo = ilo;
            sh.ihi = ihi;
        }
        __syncthreads();
        const int hit = sh.hit, ilo = sh.ilo, ihi = sh.ihi;
        if (hit >= 0) {
            // done: the selected prefix of every row
            u32 s = 0;
#pragma unroll
            for (int q = 0; q < QR; ++q) {
                if (!own[q]) continue;
                const u32 r = tid + (u32)q * MS_THREADS;
                u32 sp = 0;
#pragma unroll
                for (int i = 0; i < D; ++i)
                    if (i == hit) sp = L[q * D + i] + ((exact && r == sh.prow[i]) ? 1u : 0u);
                a.split[r] = sp;
                s += sp;
            }
            if (tid == 0) {
                if (exact && a.kth_pos) {           // (the flexible call has no k-th object output)
                    const u32 pos = (u32)sh.piv[hit];
                    *a.kth_pos = pos;
                    *a.kth_key = a.keys[pos];
                }
                if (a.rounds) *a.rounds = round + 1;
            }
            if (FLEX) {
                u32 tot;
                (void)block_excl_scan<MS_THREADS>(s, sh.scan, &tot);
                if (tid == 0) *a.k_out = tot;
            }
            return;
        }
        // recurse between the best pivot below and the best above
        const u32 cl = ilo >= 0 ? sh.cnt[ilo] : 0u;
#pragma unroll
        for (int q = 0; q < QR; ++q) {
            if (!own[q]) continue;
            const u32 r = tid + (u32)q * MS_THREADS;
            u32 nlo = lo[q], nhi = hi[q];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (i == ilo) nlo = L[q * D + i] + ((exact && r == sh.prow[i]) ? 1u : 0u);
                if (i == ihi) nhi = L[q * D + i];
            }
            lo[q] = nlo;
            hi[q] = nhi;
        }
        if (ilo >= 0) {
            if (exact) {
                k_cur -= (u64)cl + 1;
            } else {
                kmin -= cl;
                kmax -= cl;
            }
        }
        if (FLEX && !exact && ++fl_round >= AMS_ROUNDS) {
            // flexible rounds spent: finish exactly at rank kmin
            exact = true;
            k_cur = kmin;
        }
        __syncthreads();
    }
}

template <bool F, bool LG, bool FLEX>
hipError_t ms_launch(const MsArgs &a, hipStream_t s)
{
    if (a.p <= (u32)MS_THREADS)
        hipLaunchKernelGGL((k_msselect<F, LG, 1, FLEX>), dim3(1), dim3(MS_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_msselect<F, LG, 8, FLEX>), dim3(1), dim3(MS_THREADS), 0, s, a);
    return hipGetLastError();
}

template <bool FLEX>
hipError_t ms_dispatch(const MsArgs &a, bool f32, bool largest, hipStream_t s)
{
    if (f32) return largest ? ms_launch<true, true, FLEX>(a, s) : ms_launch<true, false, FLEX>(a, s);
    return largest ? ms_launch<false, true, FLEX>(a, s) : ms_launch<false, false, FLEX>(a, s);
}

}  // namespace topk

using namespace topk;

namespace {

int ms_common(topk_ctx *c, const void *keys, const uint64_t *row_off, uint32_t p, uint64_t k,
              uint64_t kmin, uint64_t kmax, uint32_t flags, uint32_t *split, uint32_t *kth_pos,
              uint32_t *kth_key, uint64_t *k_out, uint32_t *rounds, uint32_t *status,
              hipStream_t stream, bool f32, bool flex)
{
    if (!c || !keys || !row_off || !split || !status) return TOPK_E_INVALID;
    if (flex ? !k_out : (!kth_pos || !kth_key)) return TOPK_E_INVALID;
    if (p == 0 || p > MS_ROWS_MAX) return TOPK_E_INVALID;
    if (flags & ~(uint32_t)TOPK_LARGEST) return TOPK_E_INVALID;
    if (flex ? (kmin == 0 || kmin > kmax) : k == 0) return TOPK_E_INVALID;
    if (((uintptr_t)keys & 3u) || ((uintptr_t)row_off & 7u)) return TOPK_E_INVALID;
    MsArgs a{};
    a.keys = (const u32 *)keys;
    a.row_off = (const u64 *)row_off;
    a.p = p;
    a.k = k;
    a.kmin = kmin;
    a.kmax = kmax;
    a.seed = c->seed;
    a.split = split;
    a.kth_pos = kth_pos;
    a.kth_key = kth_key;
    a.k_out = k_out;
    a.rounds = rounds;
    a.status = status;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    // the status word starts at OK; the kernel writes it only on an error
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, stream, status);
    const bool lg = (flags & TOPK_LARGEST) != 0;
    const hipError_t e = flex ? ms_dispatch<true>(a, f32, lg, stream) : ms_dispatch<false>(a, f32, lg, stream);
    return e == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}

}  // namespace

extern "C" {

int topk_msselect_u32(topk_ctx *c, const uint32_t *keys, const uint64_t *row_off, uint32_t p,
                      uint64_t k, uint32_t flags, uint32_t *split, uint32_t *kth_pos,
                      uint32_t *kth_key, uint32_t *rounds, uint32_t *status, hipStream_t stream)
{
    return ms_common(c, keys, row_off, p, k, 0, 0, flags, split, kth_pos, kth_key, nullptr, rounds,
                     status, stream, false, false);
}

int topk_msselect_f32(topk_ctx *c, const float *keys, const uint64_t *row_off, uint32_t p,
                      uint64_t k, uint32_t flags, uint32_t *split, uint32_t *kth_pos,
                      float *kth_key, uint32_t *rounds, uint32_t *status, hipStream_t stream)
{
    return ms_common(c, keys, row_off, p, k, 0, 0, flags, split, kth_pos, (uint32_t *)kth_key,
                     nullptr, rounds, status, stream, true, false);
}

int topk_amsselect_u32(topk_ctx *c, const uint32_t *keys, const uint64_t *row_off, uint32_t p,
                       uint64_t kmin, uint64_t kmax, uint32_t flags, uint32_t *split,
                       uint64_t *k_out, uint32_t *rounds, uint32_t *status, hipStream_t stream)
{
    return ms_common(c, keys, row_off, p, 0, kmin, kmax, flags, split, nullptr, nullptr, k_out,
                     rounds, status, stream, false, true);
}

int topk_amsselect_f32(topk_ctx *c, const float *keys, const uint64_t *row_off, uint32_t p,
                       uint64_t kmin, uint64_t kmax, uint32_t flags, uint32_t *split,
                       uint64_t *k_out, uint32_t *rounds, uint32_t *status, hipStream_t stream)
{
    return ms_common(c, keys, row_off, p, 0, kmin, kmax, flags, split, nullptr, nullptr, k_out,
                     rounds, status, stream, true, true);
}

}  // extern "C"
