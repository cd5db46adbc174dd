// Row-wise top-k of a score matrix (forward) and the scatter of its gradient
// (backward): the form of the selection a differentiable layer needs.
//
// Forward, one 1024-thread workgroup per row, the row in registers (at most
// 64 registers a thread, so that two rows share a CU and one row's loads
// overlap the other's selection).  In the
// selection order of the whole library (composite key (ord, position), §2:
// ties broken by the object), the row's k first elements are found as
// follows.  Every thread takes the first of its own keys; every wave
// contributes the j = ceil(k / 16) first of its 64 thread minima; T = the
// last of those 16 contributions.  At least 16 j >= k distinct elements come
// at or before T, so the k first elements of the row all come at or before T:
// the candidates {c <= T} contain the answer exactly (no retry).  This is the
// local-selection-then-merge the paper suggests for small k, with the
// threads of a workgroup as the PEs.  The candidates (about 2k on
// continuous data) are gathered into LDS and each one's rank among them is
// counted, which places the k first directly in sorted order: values
// descending (largest) with ties by ascending position, as torch.topk orders
// them.  When repeated keys make the candidate set larger than the LDS
// holds, the k-th element is found by radix select over the registers and
// the candidates become exactly the k first.
//
// Backward: grad_in[b, j] = grad_out[b, m] where indices[b, m] = j, else 0.
// A workgroup owns a 4096-column chunk of a row in LDS: zero it, scatter the
// gradients that fall in it, stream it out.  Every element of grad_in is
// written exactly once (no separate clearing pass).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "../../include/topk.h"

namespace topk {

constexpr int RW_THREADS = 1024;
constexpr u32 RW_CAND = 1024;            // candidates ranked in LDS
constexpr u32 RW_MAX_K = 1024;           // 16 waves x 64 lanes
constexpr u32 RB_CHUNK = 4096;           // backward: columns per workgroup
constexpr int RB_THREADS = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int RW_BITS = 10;              // radix digit of the repeated-keys path
constexpr u32 RW_BINS = 1u << RW_BITS;   // one bin per thread
static_assert(RW_BINS == RW_THREADS, "one histogram bin per thread");

struct RowShared {
    u32 hist[RW_BINS];                   // zero outside the radix select
    u64 cand[RW_CAND];
    u64 wthr[RW_THREADS / WAVE];
    u64 rcand[WAVE];
    u32 scan[RW_THREADS / WAVE];
    u32 ccount, rcount, sel_bin, sel_before, sel_count;
    u64 found;
};

// The thread index through an empty asm: each loop recomputes its columns
// (one add) instead of the compiler keeping every column of the row live
// across the kernel.
__device__ __forceinline__ u32 opaque(u32 x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// pack(ord, col) into LDS as two 32-bit stores (no 64-bit register pair)
__device__ __forceinline__ void store_pair(u64 *dst, u32 ord, u32 col)
{
    u32 *d = reinterpret_cast<u32 *>(dst);
    d[0] = col;
    d[1] = ord;
}

// Append the lanes with `take` to the LDS candidate list (one atomic per wave).
__device__ __forceinline__ void cand_append(RowShared &sh, bool take, u32 ord, u32 col)
{
    const u64 m = ballot(take);
    if (!m) return;
    const int first = __ffsll((unsigned long long)m) - 1;
    u32 base = 0;
    if ((int)lane_id() == first) base = atomicAdd(&sh.ccount, (u32)__popcll(m));
    base = __shfl(base, first, WAVE);
    if (take) {
        const u32 q = base + mbcnt(m);
        if (q < RW_CAND) store_pair(&sh.cand[q], ord, col);
    }
}

// Pair of rank `rank` (0-based) among the row's pairs (o[e], e RW_THREADS +
// tid), valid below column N: radix select over windows of RW_BITS bits of
// the 64-bit pair from the top, keeping the bucket that holds the rank, until
// it has at most 64 pairs, which one wave ranks.  The order words stay in
// the registers they were loaded into (no 64-bit copies).
template <int IPT>
__device__ __forceinline__ u64 rw_select(const u32 (&o)[IPT], u32 N, u32 rank, RowShared &sh)
{
    const u32 tid = threadIdx.x, lane = lane_id();
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    u32 ph = 0, pl = 0;                 // bits at and above lowb are fixed
    int lowb = 64;
    u32 rk = rank, cnt = N;
    auto match = [&](u32 oj, u32 col) -> bool {
        if (lowb >= 64) return true;
        if (lowb >= 32) return (oj >> (lowb - 32)) == (ph >> (lowb - 32));
        return oj == ph && (col >> lowb) == (pl >> lowb);
    };
    while (cnt > (u32)WAVE && lowb > 0) {
        const int sh_ = lowb > RW_BITS ? lowb - RW_BITS : 0;
        const u32 tb = opaque(tid);
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const u32 col = (u32)e * RW_THREADS + tb;
            if (col < N && match(o[e], col)) {
                // bits [sh_, sh_ + RW_BITS) of the pair (o, col), from the two
                // 32-bit halves (no 64-bit register pair)
                const u32 d = (sh_ >= 32 ? o[e] >> (sh_ - 32)
                                         : __builtin_amdgcn_alignbit(o[e], col, (u32)sh_)) & (RW_BINS - 1);
                atomicAdd(&sh.hist[d], 1u);
            }
        }
        __syncthreads();
        const u32 c = sh.hist[tid];
        sh.hist[tid] = 0u;
        u32 tot;
        const u32 before = block_excl_scan<RW_THREADS>(c, sh.scan, &tot);
        if (before <= rk && rk < before + c) {
            sh.sel_bin = tid;
            sh.sel_before = before;
            sh.sel_count = c;
        }
        __syncthreads();
        const u64 bsel = (u64)__builtin_amdgcn_readfirstlane(sh.sel_bin) << sh_;
        cnt = __builtin_amdgcn_readfirstlane(sh.sel_count);
        rk -= __builtin_amdgcn_readfirstlane(sh.sel_before);
        ph |= (u32)(bsel >> 32);
        pl |= (u32)bsel;
        lowb = sh_;
        __syncthreads();                // sel_* are rewritten by the next pass
    }
    if (lowb == 0) return ((u64)ph << 32) | pl;
    if (tid == 0) sh.rcount = 0u;
    __syncthreads();
    const u32 tb = opaque(tid);
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u32 col = (u32)e * RW_THREADS + tb;
        if (col < N && match(o[e], col)) store_pair(&sh.rcand[atomicAdd(&sh.rcount, 1u)], o[e], col);
    }
    __syncthreads();
    if (w == 0) {
        const u64 mine = lane < cnt ? sh.rcand[lane] : ~0ull;
        const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
        u32 lt = 0;
        for (u32 i = 0; i < cnt; ++i) {
            const u64 x = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                          (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
            lt += x < mine ? 1u : 0u;
        }
        if (lane < cnt && lt == rk) sh.found = mine;
    }
    __syncthreads();
    return sh.found;
}

template <int IPT, bool LARGEST>
__global__ __launch_bounds__(RW_THREADS) void k_rows_fwd(const u32 *__restrict__ scores, u32 N,
                                                         u32 k, float *__restrict__ values,
                                                         long long *__restrict__ indices)
{
    __shared__ RowShared sh;
    const u32 tid = threadIdx.x, lane = lane_id();
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const u64 row = blockIdx.x;
    const u32 *__restrict__ p = scores + row * N;

    // element e of thread t is column e * 1024 + t (coalesced loads); every
    // load is issued before the first is used (a column past the row reads
    // the row's last key)
    u32 o[IPT];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u32 col = (u32)e * RW_THREADS + tid;
        o[e] = __builtin_nontemporal_load(p + (col < N ? col : N - 1));
    }
    // (a column past the row holds the image of the row's last key; every
    // later step checks the column against N)
#pragma unroll
    for (int e = 0; e < IPT; ++e) o[e] = key_ord<true, LARGEST>(o[e]);
    // the thread's first pair: columns ascend with e, so the first of equal
    // order words is the one with the lowest column (32-bit compares; the
    // 64-bit pairs are formed only where a candidate is stored)
    u32 mo = 0xFFFFFFFFu, mcol = 0xFFFFFFFFu;
    const u32 tb0 = opaque(tid);
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u32 col = (u32)e * RW_THREADS + tb0;
        if (col < N && (mcol == 0xFFFFFFFFu || o[e] < mo)) {
            mo = o[e];
            mcol = col;
        }
    }
    const u64 m = mcol == 0xFFFFFFFFu ? ~0ull : pack(mo, mcol);
    // the j first thread minima of this wave; its contribution is the j-th
    const u32 j = (k + RW_THREADS / WAVE - 1) / (RW_THREADS / WAVE);
    u64 mine = m, last = 0;
    for (u32 r = 0; r < j; ++r) {
        last = wave_min_u64(mine);
        if (mine == last) mine = ~0ull;
    }
    if (lane == 0) sh.wthr[w] = last;
    if (tid == 0) sh.ccount = 0u;
    sh.hist[tid] = 0u;
    __syncthreads();
    u64 T = 0;
#pragma unroll
    for (int i = 0; i < RW_THREADS / WAVE; ++i) T = sh.wthr[i] > T ? sh.wthr[i] : T;

    // candidates: every element at or before T
    const u32 th = (u32)(T >> 32), tl = (u32)T;
    const u32 tb1 = opaque(tid);
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u32 col = (u32)e * RW_THREADS + tb1;
        const bool take = col < N && (o[e] < th || (o[e] == th && col <= tl));
        cand_append(sh, take, o[e], col);
    }
    __syncthreads();
    u32 mc = sh.ccount;
    if (mc > RW_CAND) {
        // too many equal keys: the k-th element exactly, then the k first
        const u64 tau = rw_select<IPT>(o, N, k - 1, sh);
        const u32 uh = (u32)(tau >> 32), ul = (u32)tau;
        if (tid == 0) sh.ccount = 0u;
        __syncthreads();
        const u32 tb2 = opaque(tid);
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const u32 col = (u32)e * RW_THREADS + tb2;
            const bool take = col < N && (o[e] < uh || (o[e] == uh && col <= ul));
            cand_append(sh, take, o[e], col);
        }
        __syncthreads();
        mc = sh.ccount;
    }
    // rank of each candidate among the candidates = its output slot
    for (u32 t = tid; t < mc; t += RW_THREADS) {
        const u64 me = sh.cand[t];
        u32 r = 0;
        u32 i = 0;
        for (; i + 4 <= mc; i += 4) {
            r += sh.cand[i] < me ? 1u : 0u;
            r += sh.cand[i + 1] < me ? 1u : 0u;
            r += sh.cand[i + 2] < me ? 1u : 0u;
            r += sh.cand[i + 3] < me ? 1u : 0u;
        }
        for (; i < mc; ++i) r += sh.cand[i] < me ? 1u : 0u;
        if (r < k) {
            const u32 col = (u32)me;
            values[row * k + r] = __uint_as_float(p[col]);
            indices[row * k + r] = (long long)col;
        }
    }
}

template <bool VEC>
__global__ __launch_bounds__(RB_THREADS) void k_scatter_bwd(const float *__restrict__ g,
                                                            const long long *__restrict__ idx,
                                                            u32 N, u32 k, u32 nchunk,
                                                            float *__restrict__ gin)
{
    __shared__ float buf[RB_CHUNK];
    const u32 tid = threadIdx.x;
    const u64 row = blockIdx.x / nchunk;
    const u32 lo = (blockIdx.x % nchunk) * RB_CHUNK;
    const u32 len = N - lo < RB_CHUNK ? N - lo : RB_CHUNK;
    f32x4 *b4 = (f32x4 *)buf;
    for (u32 i = tid; i < RB_CHUNK / 4; i += RB_THREADS) b4[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    for (u32 m = tid; m < k; m += RB_THREADS) {
        const long long jj = idx[row * k + m];
        if (jj >= (long long)lo && jj < (long long)lo + len) buf[(u32)jj - lo] = g[row * k + m];
    }
    __syncthreads();
    float *out = gin + row * N + lo;
    if (VEC) {
        f32x4 *o4 = (f32x4 *)out;
        for (u32 i = tid; i < len / 4; i += RB_THREADS) __builtin_nontemporal_store(b4[i], o4 + i);
    } else {
        for (u32 i = tid; i < len; i += RB_THREADS) __builtin_nontemporal_store(buf[i], out + i);
    }
}

}  // namespace topk

using namespace topk;

extern "C" int topk_rows_fwd_f32(topk_ctx *ctx, const float *scores, uint32_t B, uint32_t N,
                                 uint32_t k, uint32_t flags, float *values, int64_t *indices,
                                 hipStream_t stream)
{
    (void)ctx;
    if (!scores || !values || !indices) return TOPK_E_INVALID;
    if (B == 0 || N == 0 || k == 0 || k > N) return TOPK_E_INVALID;
    if (flags & ~(uint32_t)TOPK_LARGEST) return TOPK_E_INVALID;
    if (((uintptr_t)scores & 3u) || ((uintptr_t)values & 3u) || ((uintptr_t)indices & 7u))
        return TOPK_E_INVALID;
    if (N > 32u * RW_THREADS || k > RW_MAX_K) return TOPK_E_UNSUPPORTED;
    const bool lg = (flags & TOPK_LARGEST) != 0;
    const u32 *s = (const u32 *)scores;
    long long *ix = (long long *)indices;
    const dim3 grid(B), block(RW_THREADS);
    if (N <= 8u * RW_THREADS) {
        if (lg) hipLaunchKernelGGL((k_rows_fwd<8, true>), grid, block, 0, stream, s, N, k, values, ix);
        else    hipLaunchKernelGGL((k_rows_fwd<8, false>), grid, block, 0, stream, s, N, k, values, ix);
    } else {
        if (lg) hipLaunchKernelGGL((k_rows_fwd<32, true>), grid, block, 0, stream, s, N, k, values, ix);
        else    hipLaunchKernelGGL((k_rows_fwd<32, false>), grid, block, 0, stream, s, N, k, values, ix);
    }
    return hipGetLastError() == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}

extern "C" int topk_scatter_bwd_f32(const float *grad_out, const int64_t *indices, uint32_t B,
                                    uint32_t N, uint32_t k, float *grad_in, hipStream_t stream)
{
    if (!grad_out || !indices || !grad_in) return TOPK_E_INVALID;
    if (B == 0 || N == 0 || k == 0 || k > N) return TOPK_E_INVALID;
    if (((uintptr_t)grad_out & 3u) || ((uintptr_t)grad_in & 3u) || ((uintptr_t)indices & 7u))
        return TOPK_E_INVALID;
    const u32 nchunk = (N + RB_CHUNK - 1) / RB_CHUNK;
    if ((u64)B * nchunk > 0x7FFFFFFFull) return TOPK_E_UNSUPPORTED;
    const bool vec = (N % 4 == 0) && (((uintptr_t)grad_in & 15u) == 0);
    const dim3 grid(B * nchunk), block(RB_THREADS);
    const long long *ix = (const long long *)indices;
    if (vec) hipLaunchKernelGGL((k_scatter_bwd<true>), grid, block, 0, stream, grad_out, ix, N, k, nchunk, grad_in);
    else     hipLaunchKernelGGL((k_scatter_bwd<false>), grid, block, 0, stream, grad_out, ix, N, k, nchunk, grad_in);
    return hipGetLastError() == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}
