// Canonical output order of the single-instance selection (TOPK_SORTED):
// the k selected positions are rewritten in the unique order by (key,
// position) of §2.  A least-significant-digit radix sort of the 64-bit pairs
// (order word << 32 | position), 8-bit digits:
//   compose  gather each selected key, form its pair; each workgroup's OR
//            and AND of its pairs (no atomics: every workgroup its own slot)
//   plan     reduce the slots; a digit that is the same in every pair needs
//            no pass (the pass would be the identity); the plan records each
//            pass's source buffer and whether it runs
//   per pass histogram of the digit per tile of SS_TILE pairs (bin-major, so
//            one flat exclusive scan gives every (digit, tile) its first
//            output slot), the scan (chunk sums, one-workgroup scan of the
//            sums, chunk scans), and a stable scatter
//   out      positions (and keys) back to the caller's arrays
// Every kernel is enqueued for every pass; a pass the plan skips returns at
// once.  The scatter is stable: a tile is taken in rounds of SX_THREADS
// pairs in order; within a round the pairs of one digit are ranked by wave
// match masks (eight ballots) and the waves' counts of that digit, across
// rounds by a running count per digit.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "sort.hpp"

namespace topk {

typedef uint16_t u16;

constexpr int SS_THREADS = 256;
constexpr int SS_WAVES = SS_THREADS / WAVE;
constexpr int SS_ROUNDS = 16;
constexpr u32 SS_TILE = SS_THREADS * SS_ROUNDS;     // pairs per tile and pass
constexpr int SS_BITS = 8;
constexpr u32 SS_BINS = 1u << SS_BITS;
constexpr int SS_PASSES = 64 / SS_BITS;
constexpr int SX_THREADS = 1024;                    // scatter: a round of 1024 pairs
constexpr int SX_WAVES = SX_THREADS / WAVE;
constexpr int SX_ROUNDS = SS_TILE / SX_THREADS;
static_assert(SS_TILE % SX_THREADS == 0, "whole scatter rounds per tile");
static_assert(SS_TILE <= 65536, "16-bit local prefixes");
constexpr u32 SP_BLOCKS = 2048;                     // compose workgroups at most
constexpr int SP_THREADS = 1024;                    // plan: one workgroup reduces the slots
constexpr int SC_THREADS = 1024;
constexpr u32 SC_CHUNK = SC_THREADS * 4;            // scan entries per chunk
static_assert(SS_BINS == (u32)SS_THREADS, "one digit per thread");

struct SortWs {
    u64 *buf[2];        // ping-pong pairs
    u32 *hist;          // [SS_BINS][tiles], scanned in place
    u32 *hcount;        // [SS_BINS][tiles], the same counts unscanned
    u32 *chunk;         // chunk sums of the scan
    u64 *bits;          // [2 b], [2 b + 1]: OR and AND of compose workgroup b's pairs
    u32 *plan;          // [p]: source buffer of pass p, bit 31: the pass runs; [SS_PASSES]: result
};

namespace {

constexpr size_t SALIGN = 256;
inline size_t salign(size_t x) { return (x + SALIGN - 1) / SALIGN * SALIGN; }
inline u64 tiles_of(u64 k) { return (k + SS_TILE - 1) / SS_TILE; }
inline u64 chunks_of(u64 entries) { return (entries + SC_CHUNK - 1) / SC_CHUNK; }

SortWs carve(void *ws, u64 k)
{
    char *w = (char *)ws;
    SortWs s{};
    size_t off = 0;
    s.buf[0] = (u64 *)(w + off); off = salign(off + k * sizeof(u64));
    s.buf[1] = (u64 *)(w + off); off = salign(off + k * sizeof(u64));
    s.hist = (u32 *)(w + off);   off = salign(off + tiles_of(k) * SS_BINS * sizeof(u32));
    s.hcount = (u32 *)(w + off); off = salign(off + tiles_of(k) * SS_BINS * sizeof(u32));
    s.chunk = (u32 *)(w + off);  off = salign(off + chunks_of(tiles_of(k) * SS_BINS) * sizeof(u32));
    s.bits = (u64 *)(w + off);   off = salign(off + 2 * SP_BLOCKS * sizeof(u64));
    s.plan = (u32 *)(w + off);
    return s;
}

}  // namespace

size_t sort_ws_bytes(uint64_t n)
{
    size_t off = 0;
    off = salign(off + n * sizeof(u64));
    off = salign(off + n * sizeof(u64));
    off = salign(off + tiles_of(n) * SS_BINS * sizeof(u32));
    off = salign(off + tiles_of(n) * SS_BINS * sizeof(u32));
    off = salign(off + chunks_of(tiles_of(n) * SS_BINS) * sizeof(u32));
    off = salign(off + 2 * SP_BLOCKS * sizeof(u64));
    off = salign(off + (SS_PASSES + 1) * sizeof(u32));
    return off;
}

// Lanes of this wave holding a pair whose digit equals this lane's (valid
// lanes only): eight ballots, one per digit bit.
__device__ __forceinline__ u64 same_digit(bool valid, u32 d)
{
    u64 peer = ballot(valid);
#pragma unroll
    for (int b = 0; b < SS_BITS; ++b) {
        const bool bit = (d >> b) & 1u;
        const u64 m = ballot(bit);
        peer &= bit ? m : ~m;
    }
    return peer;
}

template <bool IS_F32, bool LARGEST>
__global__ __launch_bounds__(SS_THREADS) void k_ss_compose(const u32 *__restrict__ keys,
                                                          const u32 *__restrict__ idx, u64 k, SortWs w)
{
    __shared__ u64 red[2][SS_WAVES];
    u64 vo = 0ull, va = ~0ull;
    for (u64 i = (u64)blockIdx.x * SS_THREADS + threadIdx.x; i < k; i += (u64)gridDim.x * SS_THREADS) {
        const u32 p = idx[i];
        const u64 x = pack(key_ord<IS_F32, LARGEST>(keys[p]), p);
        w.buf[0][i] = x;
        vo |= x;
        va &= x;
    }
    // OR / AND over the wave by butterfly shuffles
    for (int d = 1; d < WAVE; d <<= 1) {
        vo |= __shfl_xor(vo, d, WAVE);
        va &= __shfl_xor(va, d, WAVE);
    }
    const u32 wv = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        red[0][wv] = vo;
        red[1][wv] = va;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < SS_WAVES; ++v) {
            vo |= red[0][v];
            va &= red[1][v];
        }
        w.bits[2 * blockIdx.x] = vo;
        w.bits[2 * blockIdx.x + 1] = va;
    }
}

__global__ __launch_bounds__(SP_THREADS) void k_ss_plan(SortWs w, u32 nblocks)
{
    __shared__ u64 red[2][SP_THREADS / WAVE];
    u64 vo = 0ull, va = ~0ull;
    for (u32 b = threadIdx.x; b < nblocks; b += SP_THREADS) {
        vo |= w.bits[2 * b];
        va &= w.bits[2 * b + 1];
    }
    for (int d = 1; d < WAVE; d <<= 1) {
        vo |= __shfl_xor(vo, d, WAVE);
        va &= __shfl_xor(va, d, WAVE);
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x / WAVE] = vo;
        red[1][threadIdx.x / WAVE] = va;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int v = 1; v < SP_THREADS / WAVE; ++v) {
        vo |= red[0][v];
        va &= red[1][v];
    }
    const u64 varies = vo ^ va;
    u32 src = 0;
    for (int p = 0; p < SS_PASSES; ++p) {
        const bool run = ((varies >> (SS_BITS * p)) & (SS_BINS - 1)) != 0;
        w.plan[p] = src | (run ? 0x80000000u : 0u);
        if (run) src ^= 1u;
    }
    w.plan[SS_PASSES] = src;
}

// histogram of digit p of tile blockIdx.x -> hist[d * tiles + tile]
__global__ __launch_bounds__(SS_THREADS) void k_ss_hist(SortWs w, u64 k, u32 tiles, int p)
{
    const u32 pl = w.plan[p];
    if (!(pl >> 31)) return;
    __shared__ u32 hw[SS_WAVES][SS_BINS];     // one histogram per wave
    const u32 t = threadIdx.x;
#pragma unroll
    for (int v = 0; v < SS_WAVES; ++v) hw[v][t] = 0u;
    __syncthreads();
    const u64 *__restrict__ src = w.buf[pl & 1u];
    const u64 base = (u64)blockIdx.x * SS_TILE;
    const int sh = SS_BITS * p;
    const u32 wv = t / WAVE;
    // every load of the tile is issued before the first add
    u64 xr[SS_ROUNDS];
#pragma unroll
    for (int r = 0; r < SS_ROUNDS; ++r) {
        const u64 i = base + (u64)r * SS_THREADS + t;
        xr[r] = i < k ? src[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < SS_ROUNDS; ++r)
        if (base + (u64)r * SS_THREADS + t < k) atomicAdd(&hw[wv][(u32)(xr[r] >> sh) & (SS_BINS - 1)], 1u);
    __syncthreads();
    u32 c = 0;
#pragma unroll
    for (int v = 0; v < SS_WAVES; ++v) c += hw[v][t];
    w.hist[(u64)t * tiles + blockIdx.x] = c;
    w.hcount[(u64)t * tiles + blockIdx.x] = c;
}

// scan, step 1: the sum of each chunk of SC_CHUNK entries
__global__ __launch_bounds__(SC_THREADS) void k_ss_scan1(SortWs w, u64 entries, int p)
{
    if (!(w.plan[p] >> 31)) return;
    __shared__ u32 red[SC_THREADS / WAVE];
    const u64 base = (u64)blockIdx.x * SC_CHUNK;
    u32 v = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const u64 i = base + (u64)q * SC_THREADS + threadIdx.x;
        if (i < entries) v += w.hist[i];
    }
    u32 tot;
    block_excl_scan<SC_THREADS>(v, red, &tot);
    if (threadIdx.x == 0) w.chunk[blockIdx.x] = tot;
}

// scan, step 2: exclusive scan of the chunk sums in one workgroup
__global__ __launch_bounds__(SC_THREADS) void k_ss_scan2(SortWs w, u32 nchunks, int p)
{
    if (!(w.plan[p] >> 31)) return;
    __shared__ u32 red[SC_THREADS / WAVE];
    u32 carry = 0;
    for (u32 c0 = 0; c0 < nchunks; c0 += SC_THREADS) {
        const u32 c = c0 + threadIdx.x;
        const u32 v = c < nchunks ? w.chunk[c] : 0u;
        u32 tot;
        const u32 ex = block_excl_scan<SC_THREADS>(v, red, &tot);
        if (c < nchunks) w.chunk[c] = carry + ex;
        carry += tot;
        __syncthreads();                 // red is reused
    }
}

// scan, step 3: exclusive scan inside each chunk plus the chunk's offset
__global__ __launch_bounds__(SC_THREADS) void k_ss_scan3(SortWs w, u64 entries, int p)
{
    if (!(w.plan[p] >> 31)) return;
    __shared__ u32 red[SC_THREADS / WAVE];
    // thread t takes entries base + 4 t .. + 3 (contiguous, so the scan over
    // threads keeps the entries in order)
    const u64 base = (u64)blockIdx.x * SC_CHUNK + 4ull * threadIdx.x;
    u32 v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = base + q < entries ? w.hist[base + q] : 0u;
        s += v[q];
    }
    u32 tot;
    u32 run = w.chunk[blockIdx.x] + block_excl_scan<SC_THREADS>(s, red, &tot);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < entries) w.hist[base + q] = run;
        run += v[q];
    }
}

// stable scatter of tile blockIdx.x by digit p.  The tile is first placed
// in LDS in digit order (SX_ROUNDS rounds of SX_THREADS pairs in order; per
// round the leader of each group of same-digit lanes stores the group's size
// for its wave, one thread per digit turns the waves' sizes into exclusive
// prefixes plus the digit's running count, and every pair goes to its local
// slot), then written out in that order, so each digit's pairs leave as one
// contiguous run.  The per-wave sizes alternate between two buffers by round
// parity: a round's buffer is cleared during the next round, after every
// reader has passed its first barrier, and written again two rounds later.
__global__ __launch_bounds__(SX_THREADS) void k_ss_scatter(SortWs w, u64 k, u32 tiles, int p)
{
    const u32 pl = w.plan[p];
    if (!(pl >> 31)) return;
    __shared__ u64 stage[SS_TILE];               // the tile in digit order
    __shared__ u32 off[SS_BINS];                 // first output slot of each digit in this tile
    __shared__ u32 loff[SS_BINS];                // first local slot of each digit
    __shared__ u32 run[SS_BINS];                 // pairs of each digit placed by earlier rounds
    __shared__ u16 wc[2][SX_WAVES][SS_BINS];     // per wave and digit: size, then exclusive prefix
    __shared__ u32 scan[SX_THREADS / WAVE];
    const u32 t = threadIdx.x;
    const u32 wv = t / WAVE;
    const u32 cnt_t = t < SS_BINS ? w.hcount[(u64)t * tiles + blockIdx.x] : 0u;
    if (t < SS_BINS) {
        off[t] = w.hist[(u64)t * tiles + blockIdx.x];
        run[t] = 0u;
    }
    for (u32 j = t; j < 2u * SX_WAVES * SS_BINS; j += SX_THREADS) (&wc[0][0][0])[j] = 0;
    u32 tot;
    const u32 lo = block_excl_scan<SX_THREADS>(cnt_t, scan, &tot);
    if (t < SS_BINS) loff[t] = lo;
    __syncthreads();
    const u64 *__restrict__ src = w.buf[pl & 1u];
    u64 *__restrict__ dst = w.buf[(pl & 1u) ^ 1u];
    const u64 base = (u64)blockIdx.x * SS_TILE;
    const int sh = SS_BITS * p;
    // the thread's pairs of every round, loaded together
    u64 xr[SX_ROUNDS];
#pragma unroll
    for (int r = 0; r < SX_ROUNDS; ++r) {
        const u64 i = base + (u64)r * SX_THREADS + t;
        xr[r] = i < k ? src[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < SX_ROUNDS; ++r) {
        const u32 par = (u32)r & 1u;
        const u64 i = base + (u64)r * SX_THREADS + t;
        const bool valid = i < k;
        const u64 x = xr[r];
        const u32 d = (u32)(x >> sh) & (SS_BINS - 1);
        const u64 peer = same_digit(valid, d);
        const u32 before = mbcnt(peer);          // same-digit lanes below this one
        if (valid && before == 0) wc[par][wv][d] = (u16)__popcll(peer);
        __syncthreads();
        if (t < SS_BINS) {
            u32 acc = run[t];
#pragma unroll
            for (int v = 0; v < SX_WAVES; ++v) {
                const u32 c = wc[par][v][t];
                wc[par][v][t] = (u16)acc;        // at most SS_TILE - 1
                acc += c;
                wc[par ^ 1u][v][t] = 0;          // the previous round's, read before this round's barrier
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            const u32 lpos = loff[d] + wc[par][wv][d] + before;
            if (lpos < SS_TILE) stage[lpos] = x;
        }
    }
    __syncthreads();
    const u32 nt = k - base < SS_TILE ? (u32)(k - base) : SS_TILE;
    for (u32 j = t; j < nt; j += SX_THREADS) {
        const u64 x = stage[j];
        const u32 d = (u32)(x >> sh) & (SS_BINS - 1);
        const u64 g = (u64)off[d] + (j - loff[d]);
        if (g < k) dst[g] = x;
    }
}

__global__ __launch_bounds__(SS_THREADS) void k_ss_out(const u32 *__restrict__ keys, u64 n,
                                                      u32 *__restrict__ out_idx, u32 *__restrict__ out_keys,
                                                      u64 k, SortWs w)
{
    const u64 *__restrict__ res = w.buf[w.plan[SS_PASSES] & 1u];
    for (u64 i = (u64)blockIdx.x * SS_THREADS + threadIdx.x; i < k; i += (u64)gridDim.x * SS_THREADS) {
        const u32 pos = (u32)res[i];
        out_idx[i] = pos;
        if (out_keys && pos < n) out_keys[i] = keys[pos];
    }
}

hipError_t sort_selected(const uint32_t *keys, uint64_t n, bool is_f32, bool largest, uint32_t *out_idx,
                         uint32_t *out_keys, uint64_t k, void *ws, hipStream_t stream)
{
    if (k == 0) return hipSuccess;
    const SortWs w = carve(ws, k);
    const u64 tiles = tiles_of(k);
    const u64 entries = tiles * SS_BINS;
    const u64 nch = chunks_of(entries);
    if (tiles > 0x7FFFFFFFull || nch > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const u64 gs = (k + SS_THREADS - 1) / SS_THREADS;
    const u32 ncomp = (u32)(gs < SP_BLOCKS ? gs : SP_BLOCKS);
    const dim3 gstream(ncomp);
    if (is_f32) {
        if (largest) hipLaunchKernelGGL((k_ss_compose<true, true>), gstream, dim3(SS_THREADS), 0, stream, keys, out_idx, k, w);
        else hipLaunchKernelGGL((k_ss_compose<true, false>), gstream, dim3(SS_THREADS), 0, stream, keys, out_idx, k, w);
    } else {
        if (largest) hipLaunchKernelGGL((k_ss_compose<false, true>), gstream, dim3(SS_THREADS), 0, stream, keys, out_idx, k, w);
        else hipLaunchKernelGGL((k_ss_compose<false, false>), gstream, dim3(SS_THREADS), 0, stream, keys, out_idx, k, w);
    }
    hipLaunchKernelGGL(k_ss_plan, dim3(1), dim3(SP_THREADS), 0, stream, w, ncomp);
    for (int p = 0; p < SS_PASSES; ++p) {
        hipLaunchKernelGGL(k_ss_hist, dim3((unsigned)tiles), dim3(SS_THREADS), 0, stream, w, k, (u32)tiles, p);
        hipLaunchKernelGGL(k_ss_scan1, dim3((unsigned)nch), dim3(SC_THREADS), 0, stream, w, entries, p);
        hipLaunchKernelGGL(k_ss_scan2, dim3(1), dim3(SC_THREADS), 0, stream, w, (u32)nch, p);
        hipLaunchKernelGGL(k_ss_scan3, dim3((unsigned)nch), dim3(SC_THREADS), 0, stream, w, entries, p);
        hipLaunchKernelGGL(k_ss_scatter, dim3((unsigned)tiles), dim3(SX_THREADS), 0, stream, w, k, (u32)tiles, p);
    }
    hipLaunchKernelGGL(k_ss_out, gstream, dim3(SS_THREADS), 0, stream, keys, n, out_idx, out_keys, k, w);
    return hipGetLastError();
}

}  // namespace topk
