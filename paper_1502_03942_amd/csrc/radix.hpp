// Exact selection of one or two ranks among keys held in the registers of
// one workgroup (used by the pivot choice, the finisher and the row kernels).
#pragma once
#include "common.hpp"

namespace topk {

constexpr int RS_BITS = 12;                    // radix select digit
constexpr u32 RS_BINS = 1u << RS_BITS;
constexpr int RS_THREADS = 1024;              // workgroup size radix_select assumes (16 waves)

// LDS of radix_select
struct RadixShared {
    u32 rhist[2][RS_BINS];
    u64 rmin[2], rmax[2];
    u64 cand[2][WAVE];
    u32 ccount[2];
    u32 rscan[2][8];
    u32 sel_bin[2], sel_before[2], sel_count[2];
    u64 found[2];
};

// ---------------------------------------------------------------------------
// Radix select in one workgroup.  Every thread holds up to M keys in registers
// (the first `cnt` valid).  Finds the keys of 0-based ranks rank[0] and rank[1]
// (each only if act[t]) among all valid keys.  Keys must be distinct (they are
// (ord, position) pairs).
//
// The candidates of a target are the keys that share the bits fixed so far.
// A pass takes their minimum and maximum, histograms the RS_BITS bits just
// below the common prefix of the two (so bits every candidate shares cost no
// pass) and keeps the bucket that holds the rank.  Once that bucket holds at
// most 64 keys they are gathered and one wave ranks them directly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool rs_match(u64 x, u64 pref, int lowb)
{
    return lowb >= 64 || (x >> lowb) == (pref >> lowb);
}

template <int M>
__device__ __forceinline__ void radix_select(const u64 (&v)[M], int cnt, const u64 rank_in[2],
                                             const bool act[2], u64 out[2], RadixShared &sm)
{
    const u32 tid = threadIdx.x, lane = lane_id();
    const u32 w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    // slots at or past the wave's largest count hold nothing: skip them uniformly
    const int cw = (int)wave_max_u64((u64)(cnt > 0 ? cnt : 0));
    u64 pref[2] = {0ull, 0ull};
    int lowb[2] = {64, 64};               // bits [lowb, 64) of the candidates equal pref's
    u64 rank[2] = {rank_in[0], rank_in[1]};
    bool done[2] = {!act[0], !act[1]};
    u64 res[2] = {0ull, 0ull};
    for (u32 i = tid; i < 2u * RS_BINS; i += RS_THREADS) (&sm.rhist[0][0])[i] = 0u;
    if (tid < 2) {
        sm.rmin[tid] = ~0ull;
        sm.rmax[tid] = 0ull;
        sm.ccount[tid] = 0u;
    }
    __syncthreads();
    for (int pass = 0; pass < 8 && !(done[0] && done[1]); ++pass) {
        // (1) minimum and maximum of each target's candidates
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (done[t]) continue;
            u64 mn = ~0ull, mx = 0ull;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j < cw && j < cnt && rs_match(v[j], pref[t], lowb[t])) {
                    mn = v[j] < mn ? v[j] : mn;
                    mx = v[j] > mx ? v[j] : mx;
                }
            }
            mn = wave_min_u64(mn);
            mx = wave_max_u64(mx);
            if (lane == 0 && mn <= mx) {
                atomicMin((unsigned long long *)&sm.rmin[t], (unsigned long long)mn);
                atomicMax((unsigned long long *)&sm.rmax[t], (unsigned long long)mx);
            }
        }
        __syncthreads();
        // (2) histogram of the window below the common prefix
        int sh[2] = {0, 0};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (done[t]) continue;
            const u64 mn = sm.rmin[t], mx = sm.rmax[t];
            if (mn == mx) {
                res[t] = mn;
                done[t] = true;
                continue;
            }
            const int hb = 63 - __clzll((long long)(mn ^ mx));
            sh[t] = hb >= RS_BITS - 1 ? hb - (RS_BITS - 1) : 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j < cw && j < cnt && rs_match(v[j], pref[t], lowb[t]))
                    atomicAdd(&sm.rhist[t][(u32)(v[j] >> sh[t]) & (RS_BINS - 1)], 1u);
            }
        }
        __syncthreads();
        // (3) scan: waves 8t .. 8t+7 cover target t's bins, lane l eight of them
        const u32 t3 = w >> 3, sw = w & 7u;
        const u32 b0 = sw * (RS_BINS / 8) + lane * 8u;
        u32 c[8], csum = 0, cincl = 0;
        if (!done[t3]) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                c[i] = sm.rhist[t3][b0 + i];
                csum += c[i];
            }
            cincl = wave_incl_scan(csum);
            if (lane == WAVE - 1) sm.rscan[t3][sw] = cincl;
        }
        __syncthreads();
        if (!done[t3]) {
            u32 before = cincl - csum;
            for (u32 i = 0; i < sw; ++i) before += sm.rscan[t3][i];
            const u64 r = rank[t3];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if ((u64)before <= r && r < (u64)before + c[i]) {
                    sm.sel_bin[t3] = b0 + (u32)i;
                    sm.sel_before[t3] = before;
                    sm.sel_count[t3] = c[i];
                }
                before += c[i];
                sm.rhist[t3][b0 + i] = 0u;       // clean for the next pass
            }
        }
        __syncthreads();
        // (4) narrow to the bucket; gather it when small
        bool gather[2] = {false, false};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (done[t]) continue;
            const u64 mn = sm.rmin[t];
            const int top = sh[t] + RS_BITS;
            const u64 high = top >= 64 ? 0ull : (mn >> top) << top;
            pref[t] = high | ((u64)sm.sel_bin[t] << sh[t]);
            lowb[t] = sh[t];
            rank[t] -= sm.sel_before[t];
            gather[t] = sm.sel_count[t] <= (u32)WAVE;
        }
        __syncthreads();
        if (tid < 2) {
            sm.rmin[tid] = ~0ull;
            sm.rmax[tid] = 0ull;
        }
        if (gather[0] || gather[1]) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (!gather[t]) continue;
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    if (j < cw && j < cnt && rs_match(v[j], pref[t], lowb[t]))
                        sm.cand[t][atomicAdd(&sm.ccount[t], 1u)] = v[j];
                }
            }
            __syncthreads();
            if (w < 2 && gather[w]) {
                const u32 m = sm.ccount[w];
                const u64 mine = lane < m ? sm.cand[w][lane] : ~0ull;
                const u32 mlo = (u32)mine, mhi = (u32)(mine >> 32);
                u32 below = 0;
                for (u32 i = 0; i < m; ++i) {
                    const u64 o = ((u64)(u32)__builtin_amdgcn_readlane((int)mhi, (int)i) << 32) |
                                  (u32)__builtin_amdgcn_readlane((int)mlo, (int)i);
                    below += o < mine ? 1u : 0u;
                }
                if (lane < m && (u64)below == rank[w]) sm.found[w] = mine;
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (!gather[t]) continue;
                res[t] = sm.found[t];
                done[t] = true;
            }
        }
    }
    out[0] = res[0];
    out[1] = res[1];
    __syncthreads();
}


}  // namespace topk
