// sa_kernels_otm.hip -- optimal-transition Metropolis variants of the plain launch (Sec. 3.3.3).
#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {

AnnealKernelFn otm_kernel(bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen) {
    if (sixteen) {
        if (maxe_class == 1)
            return narrow ? anneal_kernel<SA_OPT_METROPOLIS, true, 0, 1, uint32_t, 1024>
                          : anneal_kernel<SA_OPT_METROPOLIS, true, 0, 1, uint64_t, 1024>;
        return narrow ? anneal_kernel<SA_OPT_METROPOLIS, true, 0, 2, uint32_t, 1024>
                      : anneal_kernel<SA_OPT_METROPOLIS, true, 0, 2, uint64_t, 1024>;
    }
    if (!in_lds) return anneal_kernel<SA_OPT_METROPOLIS, false, 1, 4, uint64_t, 512>;
    if (reg_chunk == 1) {
        // ranges wider than the enumeration limit: the forward-difference argmin is built in
        switch (maxe_class) {
            case 1: return anneal_kernel<SA_OPT_METROPOLIS, true, 1, 1, uint64_t, 512>;
            case 2: return anneal_kernel<SA_OPT_METROPOLIS, true, 1, 2, uint64_t, 512>;
            default: return anneal_kernel<SA_OPT_METROPOLIS, true, 1, 4, uint64_t, 512>;
        }
    }
    switch (maxe_class) {
        case 1: return narrow ? anneal_kernel<SA_OPT_METROPOLIS, true, 0, 1, uint32_t, 512>
                              : anneal_kernel<SA_OPT_METROPOLIS, true, 0, 1, uint64_t, 512>;
        case 2: return narrow ? anneal_kernel<SA_OPT_METROPOLIS, true, 0, 2, uint32_t, 512>
                              : anneal_kernel<SA_OPT_METROPOLIS, true, 0, 2, uint64_t, 512>;
        default: return anneal_kernel<SA_OPT_METROPOLIS, true, 0, 4, uint64_t, 512>;
    }
}

}  // namespace sa
