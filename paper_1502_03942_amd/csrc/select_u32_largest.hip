// Single-instance selection kernels: u32 keys, largest order.
#include "select_impl.hpp"

namespace topk {
TOPK_INSTANTIATE_SELECT(false, true)
}  // namespace topk
