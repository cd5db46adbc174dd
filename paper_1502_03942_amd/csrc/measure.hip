// Measurement helper, not part of the selection: one read of an array with
// the first sweep's access pattern, so that the stream-read bandwidth of the
// device can be measured next to the selection.  A wave reads wave-tiles of
// 4096 keys as 64 columns of 64 lanes (one 256-byte non-temporal load per
// column), two workgroups of 8 waves per CU walk the tiles grid-stride (the
// fastest arrangement of this pattern measured: 6.94 TB/s against 6.74 with
// one workgroup of 16 waves per CU), and the keys are summed into one word
// so that no load can be dropped.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "ctx.hpp"
#include "../../include/topk.h"

namespace topk {

constexpr int MR_THREADS = 512;
constexpr int MR_COLS = 64;
constexpr u32 MR_TILE = MR_COLS * WAVE;

__global__ __launch_bounds__(MR_THREADS) void k_stream_read(const u32 *__restrict__ keys, u32 ntile,
                                                            u32 *sink)
{
    const u32 lane = lane_id();
    const u32 w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const u32 waves = MR_THREADS / WAVE;
    u32 acc = 0;
    for (u32 t = blockIdx.x * waves + w; t < ntile; t += gridDim.x * waves) {
        const u32 *p = keys + (u64)t * MR_TILE;
        u32 x[MR_COLS];
#pragma unroll
        for (int j = 0; j < MR_COLS; ++j) x[j] = __builtin_nontemporal_load(p + j * WAVE + lane);
#pragma unroll
        for (int j = 0; j < MR_COLS; ++j) acc += x[j];
    }
    // one device atomic per workgroup (atomics on one word serialise: one per
    // wave would add tens of microseconds)
    __shared__ u32 red[MR_THREADS / WAVE];
    acc = wave_sum_u32(acc);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (u32 i = 0; i < waves; ++i) t += red[i];
        atomicAdd(sink, t);
    }
}

}  // namespace topk

using namespace topk;

extern "C" int topk_stream_read(topk_ctx *c, const uint32_t *keys, uint64_t n, uint32_t *sink,
                                hipStream_t stream)
{
    if (!c || !keys || !sink || n == 0 || n % MR_TILE != 0) return TOPK_E_INVALID;
    if (n / MR_TILE > 0xFFFFFFFFull) return TOPK_E_INVALID;
    if ((uintptr_t)keys & 255u || (uintptr_t)sink & 3u) return TOPK_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return TOPK_E_HIP;
    hipLaunchKernelGGL(k_stream_read, dim3(c->num_cu * 2), dim3(MR_THREADS), 0, stream, keys,
                       (u32)(n / MR_TILE), sink);
    return hipGetLastError() == hipSuccess ? TOPK_OK : TOPK_E_HIP;
}
