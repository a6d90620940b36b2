// Batched-exploration kernels with 1-word slots.
#include "gx_batch_kernel.hpp"

namespace gx {
template hipError_t batch_launch<1>(uint32_t, uint32_t, uint32_t, const BatchArgs&, uint32_t,
                                     size_t, hipStream_t);
template int batch_resident<1>(uint32_t, uint32_t, uint32_t, size_t);
template hipError_t batch_init<1>(uint32_t, uint32_t, uint32_t, const BatchArgs&, hipStream_t);
}  // namespace gx
