// Server step kernels with 2-word slots.
#include "gx_serve_kernel.hpp"

namespace gx {
template hipError_t serve_launch<2>(uint32_t, uint32_t, uint32_t, const ServeArgs&, uint32_t,
                                     size_t, hipStream_t);
}  // namespace gx
