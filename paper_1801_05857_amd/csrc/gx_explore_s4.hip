// Exploration level kernel specialisations with 4-word slots.
#include "gx_explore_kernel.hpp"

namespace gx {
template hipError_t level_b<4>(uint32_t B, uint32_t G, uint32_t U, const ExploreArgs& a,
                               uint32_t grid, size_t lds, hipStream_t s);
}  // namespace gx
