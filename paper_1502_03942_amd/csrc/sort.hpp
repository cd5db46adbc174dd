// Canonical output order of the single-instance selection (TOPK_SORTED).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace topk {

// Device workspace bytes for sorting up to n selected pairs.
size_t sort_ws_bytes(uint64_t n);

// Enqueue on `stream`: rewrite out_idx[0..k) (positions below n) in the unique order by
// (key, position) of the selection (keys ascending, or descending with
// largest; ties by ascending position), and out_keys (if not null) to match.
// `ws` holds at least sort_ws_bytes(k) bytes, 256-byte aligned.
hipError_t sort_selected(const uint32_t *keys, uint64_t n, bool is_f32, bool largest, uint32_t *out_idx,
                         uint32_t *out_keys, uint64_t k, void *ws, hipStream_t stream);

}  // namespace topk
