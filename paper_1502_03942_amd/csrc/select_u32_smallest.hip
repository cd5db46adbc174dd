// Single-instance selection kernels: u32 keys, smallest order.
#include "select_impl.hpp"

namespace topk {
TOPK_INSTANTIATE_SELECT(false, false)
}  // namespace topk
