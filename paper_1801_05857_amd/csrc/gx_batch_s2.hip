// Batched-exploration kernels with 2-word slots.
#include "gx_batch_kernel.hpp"

namespace gx {
template hipError_t batch_launch<2>(uint32_t, uint32_t, uint32_t, const BatchArgs&, uint32_t,
                                     size_t, hipStream_t);
template int batch_resident<2>(uint32_t, uint32_t, uint32_t, size_t);
template hipError_t batch_init<2>(uint32_t, uint32_t, uint32_t, const BatchArgs&, hipStream_t);
}  // namespace gx
