// Single-instance selection kernels: f32 keys, smallest order.
#include "select_impl.hpp"

namespace topk {
TOPK_INSTANTIATE_SELECT(true, false)
}  // namespace topk
