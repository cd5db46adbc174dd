// Device-side building blocks shared by the selection kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
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

// Cross-lane steps on the DPP network (row = 16 lanes): no LDS round trip.
// dpp<CTRL, ROWS>(v): v from the lane CTRL names, 0 where there is none or
// the destination row is not in ROWS.
enum : int {
    DPP_XOR1 = 0xB1,            // quad_perm [1,0,3,2]
    DPP_XOR2 = 0x4E,            // quad_perm [2,3,0,1]
    DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118,
    DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141,
    DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143,
};
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ u32 dpp(u32 v)
{
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, true);
}

// inclusive prefix sum across the wave
__device__ __forceinline__ u32 wave_incl_scan(u32 v)
{
    v += dpp<DPP_ROW_SHR1>(v);
    v += dpp<DPP_ROW_SHR2>(v);
    v += dpp<DPP_ROW_SHR4>(v);
    v += dpp<DPP_ROW_SHR8>(v);
    v += dpp<DPP_ROW_BCAST15, 0xA>(v);
    v += dpp<DPP_ROW_BCAST31, 0xC>(v);
    return v;
}

__device__ __forceinline__ u32 wave_sum_u32(u32 v)
{
    return (u32)__builtin_amdgcn_readlane((int)wave_incl_scan(v), WAVE - 1);
}

// min / max over the wave (wave-uniform result)
template <bool MAX>
__device__ __forceinline__ u64 wave_ext_u64(u64 v)
{
    auto step = [&](auto ctrl_tag, auto rows_tag) {
        constexpr int C = decltype(ctrl_tag)::value, R = decltype(rows_tag)::value;
        const u32 lo = (u32)__builtin_amdgcn_update_dpp((int)(u32)v, (int)(u32)v, C, R, 0xF, false);
        const u32 hi = (u32)__builtin_amdgcn_update_dpp((int)(u32)(v >> 32), (int)(u32)(v >> 32), C, R, 0xF, false);
        const u64 w = ((u64)hi << 32) | lo;
        v = MAX ? (w > v ? w : v) : (w < v ? w : v);
    };
    step(std::integral_constant<int, DPP_XOR1>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_XOR2>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_ROW_HALF_MIRROR>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_ROW_MIRROR>(), std::integral_constant<int, 0xF>());
    step(std::integral_constant<int, DPP_ROW_BCAST15>(), std::integral_constant<int, 0xA>());
    step(std::integral_constant<int, DPP_ROW_BCAST31>(), std::integral_constant<int, 0xC>());
    const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)v, WAVE - 1);
    const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)(v >> 32), WAVE - 1);
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ u64 wave_max_u64(u64 v) { return wave_ext_u64<true>(v); }
__device__ __forceinline__ u64 wave_min_u64(u64 v) { return wave_ext_u64<false>(v); }

// Exclusive prefix sum over a workgroup of NT threads; returns this thread's
// exclusive prefix and writes the total to *total.  `scratch` holds NT/64 u32.
// Barrier that orders only LDS: waits for the wave's LDS operations, not for
// its global loads and stores, which stay in flight across it.  For kernels
// whose waves exchange data only through LDS.
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int NT, bool LDS_ONLY = false>
__device__ __forceinline__ u32 block_excl_scan(u32 v, u32 *scratch, u32 *total)
{
    constexpr int NW = NT / WAVE;
    const u32 w = threadIdx.x / WAVE, l = lane_id();
    u32 inc = wave_incl_scan(v);
    if (l == WAVE - 1) scratch[w] = inc;
    if (LDS_ONLY) lds_sync(); else __syncthreads();
    u32 before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        u32 s = scratch[i];
        before += (i < (int)w) ? s : 0u;
        tot += s;
    }
    if (LDS_ONLY) lds_sync(); else __syncthreads();
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

// ---------------------------------------------------------------------------
// Pivot ranks (§2, FR-selection: sample ranks k|S|/n -/+ Delta).  Integer form
// of Delta = ceil(c sqrt(m_hi (s - m_lo) / s)) + 1 with c = c_num / 4:
// the least D with 16 s D^2 >= c_num^2 m_hi (s - m_lo).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pivot_ranks(u64 s, u64 k, u64 n, u32 c_num, i64 &lo, i64 &hi)
{
    if (s == 0) { lo = -1; hi = 0; return; }
    const u64 m_lo = k * s / n;
    const u64 m_hi = (k * s + n - 1) / n;
    const u64 X = (u64)c_num * c_num * m_hi * (s - m_lo);
    const u64 Y = 16 * s;
    const u64 t = (X + Y - 1) / Y;
    u64 d = (u64)sqrt((double)t);
    while (d * d < t) ++d;
    while (d > 0 && (d - 1) * (d - 1) >= t) --d;
    lo = (i64)m_lo - (i64)(d + 1);
    hi = (i64)m_hi + (i64)(d + 1);
}

}  // namespace topk
