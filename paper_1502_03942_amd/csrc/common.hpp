// Device-side building blocks shared by the selection kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace topk {

typedef uint32_t u32;
typedef uint64_t u64;
typedef int64_t i64;

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Key order (§2: values made unique by the pair (value, object)).
// ord() maps a key to a u32 whose unsigned order is the selection order of the
// values; the pair (ord, position) packed as (ord << 32 | position) is then a
// u64 whose unsigned order is the unique total order.
//   f32: NaN (any sign/payload) -> 0xFFFFFFFF (above +inf, all NaNs tie);
//        -0.0 -> the image of +0.0; negatives -> ~bits; others -> bits | 2^31.
//   u32: identity.
//   largest: complement, which reverses the value order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 ord_f32_bits(u32 b)
{
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return 0xFFFFFFFFu;   // NaN
    if (b == 0x80000000u) b = 0u;                               // -0 -> +0
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

template <bool IS_F32, bool LARGEST>
__device__ __forceinline__ u32 key_ord(u32 bits)
{
    u32 o = IS_F32 ? ord_f32_bits(bits) : bits;
    return LARGEST ? ~o : o;
}

__device__ __forceinline__ u64 pack(u32 ord, u32 idx) { return ((u64)ord << 32) | idx; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies mixed with the other words and a key bumped by Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, u32 k0, u32 k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const u32 lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const u32 lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// ---------------------------------------------------------------------------
// Wave helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 lane_id() { return __lane_id(); }

// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ u32 mbcnt(u64 mask)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ u32 wave_sum_u32(u32 v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ u64 wave_max_u64(u64 v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u64 w = __shfl_xor(v, o, WAVE);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ u64 wave_min_u64(u64 v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u64 w = __shfl_xor(v, o, WAVE);
        v = w < v ? w : v;
    }
    return v;
}

// inclusive prefix sum across the wave
__device__ __forceinline__ u32 wave_incl_scan(u32 v)
{
    const u32 l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        u32 w = __shfl_up(v, o, WAVE);
        if (l >= (u32)o) v += w;
    }
    return v;
}

// Exclusive prefix sum over a workgroup of NT threads; returns this thread's
// exclusive prefix and writes the total to *total.  `scratch` holds NT/64 u32.
template <int NT>
__device__ __forceinline__ u32 block_excl_scan(u32 v, u32 *scratch, u32 *total)
{
    constexpr int NW = NT / WAVE;
    const u32 w = threadIdx.x / WAVE, l = lane_id();
    u32 inc = wave_incl_scan(v);
    if (l == WAVE - 1) scratch[w] = inc;
    __syncthreads();
    u32 before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        u32 s = scratch[i];
        before += (i < (int)w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Agent-scope relaxed atomics for the single-pass scan's status words (the
// payload travels in the same 64-bit word as its flag, so no fence is needed).
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 ld_status(const u64 *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(u64 *p, u64 v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace topk
