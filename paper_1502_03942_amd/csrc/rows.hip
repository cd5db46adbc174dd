// Row-wise top-k of a score matrix (forward) and the scatter of its gradient
// (backward): the form of the selection a differentiable layer needs.
//
// Forward, one 1024-thread workgroup per row, the row in registers.  In the
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
#include "radix.hpp"
#include "../../include/topk.h"

namespace topk {

constexpr int RW_THREADS = 1024;
constexpr u32 RW_CAND = 1024;            // candidates ranked in LDS
constexpr u32 RW_MAX_K = 1024;           // 16 waves x 64 lanes
constexpr u32 RB_CHUNK = 4096;           // backward: columns per workgroup
constexpr int RB_THREADS = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct RowShared {
    RadixShared rs;
    u64 cand[RW_CAND];
    u64 wthr[RW_THREADS / WAVE];
    u32 ccount;
};

// Append the lanes with `take` to the LDS candidate list (one atomic per wave).
__device__ __forceinline__ void cand_append(RowShared &sh, bool take, u64 c)
{
    const u64 m = ballot(take);
    if (!m) return;
    const int first = __ffsll((unsigned long long)m) - 1;
    u32 base = 0;
    if ((int)lane_id() == first) base = atomicAdd(&sh.ccount, (u32)__popcll(m));
    base = __shfl(base, first, WAVE);
    if (take) {
        const u32 q = base + mbcnt(m);
        if (q < RW_CAND) sh.cand[q] = c;
    }
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
    // the row's last key, then is marked empty)
    u32 o[IPT];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u32 col = (u32)e * RW_THREADS + tid;
        o[e] = __builtin_nontemporal_load(p + (col < N ? col : N - 1));
    }
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u32 col = (u32)e * RW_THREADS + tid;
        o[e] = col < N ? key_ord<true, LARGEST>(o[e]) : 0xFFFFFFFFu;
    }
    auto comp = [&](int e) -> u64 {
        const u32 col = (u32)e * RW_THREADS + tid;
        return col < N ? pack(o[e], col) : ~0ull;
    };
    u64 m = ~0ull;
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u64 c = comp(e);
        m = c < m ? c : m;
    }
    // the j first thread minima of this wave; its contribution is the j-th
    const u32 j = (k + RW_THREADS / WAVE - 1) / (RW_THREADS / WAVE);
    u64 mine = m, last = 0;
    for (u32 r = 0; r < j; ++r) {
        last = wave_min_u64(mine);
        if (mine == last) mine = ~0ull;
    }
    if (lane == 0) sh.wthr[w] = last;
    if (tid == 0) sh.ccount = 0u;
    __syncthreads();
    u64 T = 0;
#pragma unroll
    for (int i = 0; i < RW_THREADS / WAVE; ++i) T = sh.wthr[i] > T ? sh.wthr[i] : T;

    // candidates: every element at or before T
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const u64 c = comp(e);
        cand_append(sh, c <= T && c != ~0ull, c);
    }
    __syncthreads();
    u32 mc = sh.ccount;
    if (mc > RW_CAND) {
        // too many equal keys: the k-th element exactly, then the k first
        u64 v[IPT];
        int cnt = 0;                        // slots holding a column (a prefix)
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            v[e] = comp(e);
            cnt += (u32)e * RW_THREADS + tid < N ? 1 : 0;
        }
        const u64 ranks[2] = {(u64)k - 1, 0ull};
        const bool act[2] = {true, false};
        u64 tau2[2];
        radix_select<IPT>(v, cnt, ranks, act, tau2, sh.rs);
        __syncthreads();
        if (tid == 0) sh.ccount = 0u;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < IPT; ++e) cand_append(sh, e < cnt && v[e] <= tau2[0], v[e]);
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
