// sa_kernels_metropolis.hip -- Metropolis variants of the plain launch (Sec. 3.3.1).
#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {

// Metropolis kernels take each variable's exponents from its own mask, so one exponent class
// serves every problem.
AnnealKernelFn metropolis_kernel(bool in_lds, int reg_chunk, bool narrow, bool sixteen) {
    if (sixteen)
        return narrow ? anneal_kernel<SA_METROPOLIS, true, 0, 1, uint32_t, 1024>
                      : anneal_kernel<SA_METROPOLIS, true, 0, 1, uint64_t, 1024>;
    if (!in_lds) return anneal_kernel<SA_METROPOLIS, false, 0, 1, uint64_t, 512>;
    if (reg_chunk == 1)   // dense form: coupling rows prefetched one window ahead
        return narrow ? anneal_kernel<SA_METROPOLIS, true, 1, 1, uint32_t, 512>
                      : anneal_kernel<SA_METROPOLIS, true, 1, 1, uint64_t, 512>;
    return narrow ? anneal_kernel<SA_METROPOLIS, true, 0, 1, uint32_t, 512>
                  : anneal_kernel<SA_METROPOLIS, true, 0, 1, uint64_t, 512>;
}

}  // namespace sa
