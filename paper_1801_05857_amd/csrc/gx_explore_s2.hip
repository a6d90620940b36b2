// Exploration level kernels (successor generation, find-or-put-and-append, small levels on one workgroup) with 2-word slots.
#include "gx_small_kernel.hpp"

namespace gx {
template hipError_t launch_gen<2>(const GenArgs& a, uint32_t grid, size_t lds, hipStream_t s);
template hipError_t append_b<2>(uint32_t B, uint32_t G, uint32_t U, const AppendArgs& a,
                                 uint32_t cus, hipStream_t s);
template hipError_t launch_small<2>(uint32_t B, const SmallArgs& a, hipStream_t s);
template hipError_t launch_lds_levels<2>(uint32_t B, SmallArgs a, size_t lds_limit,
                                         hipStream_t s);
}  // namespace gx
