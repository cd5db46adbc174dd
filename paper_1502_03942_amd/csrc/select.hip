// Dispatch of the single-instance selection to the instantiation for the key
// type and order (select_<type>_<order>.hip).
#include "select.hpp"

namespace topk {

template <bool F, bool LG>
hipError_t launch_impl(SelArgs a, const SelLaunch &L, hipStream_t s, KernelTimer *tm);
template <bool F, bool LG>
int sweep_blocks_per_cu();

int sweep_max_grid(bool is_f32, bool largest, int num_cu)
{
    int nb;
    if (is_f32) nb = largest ? sweep_blocks_per_cu<true, true>() : sweep_blocks_per_cu<true, false>();
    else nb = largest ? sweep_blocks_per_cu<false, true>() : sweep_blocks_per_cu<false, false>();
    return nb * num_cu;
}

hipError_t launch_select(const SelArgs &a, const SelLaunch &L, hipStream_t stream,
                         KernelTimer *tm)
{
    if (L.is_f32) {
        return L.largest ? launch_impl<true, true>(a, L, stream, tm)
                         : launch_impl<true, false>(a, L, stream, tm);
    }
    return L.largest ? launch_impl<false, true>(a, L, stream, tm)
                     : launch_impl<false, false>(a, L, stream, tm);
}

}  // namespace topk
