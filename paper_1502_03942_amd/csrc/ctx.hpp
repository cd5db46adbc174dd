// Host state behind the opaque topk_ctx of the C-ABI (not part of the API).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <tuple>
#include <vector>

// Row-length classes of the batched form: class c holds the rows of length
// [2^(c-1), 2^c) (class 0: empty rows, the last class: everything longer).
constexpr int TOPK_BT_NCLS = 34;

struct topk_ctx {
    int device;
    uint64_t seed;
    int64_t s_target, c_num, t_fin, r_max, r_fast, band_div, tail_max, timing;
    // batched form: sample size of a long row, pivot spread, workgroups per CU,
    // sampling attempts before the exact fallback, fast sweep on/off, fast
    // sweep tile (keys per thread per step)
    int64_t bt_s_target, bt_c_num, bt_wg_per_cu, bt_attempts, bt_fast, bt_tile;
    // per row-length class overrides of bt_s_target / bt_c_num / bt_tile (-1: none)
    int64_t bt_s_cls[TOPK_BT_NCLS], bt_c_cls[TOPK_BT_NCLS], bt_t_cls[TOPK_BT_NCLS];
    // most frequent objects / sum aggregation: how objects are counted (0 by
    // the universe size, 1 LDS hash tables, 2 partitioned, 3 direct)
    int64_t fq_mode;
    int num_cu;
    // kernel timing: event pairs recorded by calls since the last read-out
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    int ev_used = 0;
    // batched form: instantiated graphs by call arguments
    hipStream_t capture_stream = nullptr;
    std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
};

// Device address of the scratch array of topk_select_batched_f32_noalloc on
// `device`, looked up once per device (batched.hip).
int topk_bt_scratch_setup(int device);
