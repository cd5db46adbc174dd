// Single-instance selection kernels: f32 keys, largest order.
#include "select_impl.hpp"

namespace topk {
TOPK_INSTANTIATE_SELECT(true, true)
}  // namespace topk
