// Find-or-put specialisations with 4-word slots.
#include "gx_fop_kernel.hpp"

namespace gx {
template hipError_t dispatch_b<4>(uint32_t B, uint32_t G, uint32_t U, const FopArgs& a);
}  // namespace gx
