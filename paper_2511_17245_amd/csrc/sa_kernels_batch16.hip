// sa_kernels_batch16.hip -- the persistent batched kernel with 16-bit states (every variable's
// range inside the int16 range).
#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {

BatchKernelFn batch_kernel_z16(int maxe_class, bool narrow) {
    switch (maxe_class) {
        case 1: return narrow ? batch_kernel<1, uint32_t, int16_t> : batch_kernel<1, uint64_t, int16_t>;
        case 2: return narrow ? batch_kernel<2, uint32_t, int16_t> : batch_kernel<2, uint64_t, int16_t>;
        case 4: return batch_kernel<4, uint64_t, int16_t>;
        default: return batch_kernel<kMaxExpPoly, uint64_t, int16_t>;
    }
}

}  // namespace sa
