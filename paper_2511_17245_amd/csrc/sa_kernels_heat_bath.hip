// sa_kernels_heat_bath.hip -- heat-bath variants of the plain launch (Sec. 3.3.2, enumeration).
#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {

AnnealKernelFn heat_bath_kernel(bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen) {
    if (sixteen) {
        if (maxe_class == 1)
            return narrow ? pick_heat_bath_lds_16<SA_HEAT_BATH, 1, uint32_t>(reg_chunk)
                          : pick_heat_bath_lds_16<SA_HEAT_BATH, 1, uint64_t>(reg_chunk);
        return narrow ? pick_heat_bath_lds_16<SA_HEAT_BATH, 2, uint32_t>(reg_chunk)
                      : pick_heat_bath_lds_16<SA_HEAT_BATH, 2, uint64_t>(reg_chunk);
    }
    if (!in_lds) return anneal_kernel<SA_HEAT_BATH, false, 0, kMaxExpPoly, uint64_t, 512>;
    switch (maxe_class) {
        case 1: return narrow ? pick_heat_bath_lds<SA_HEAT_BATH, 1, uint32_t>(reg_chunk)
                              : pick_heat_bath_lds<SA_HEAT_BATH, 1, uint64_t>(reg_chunk);
        case 2: return narrow ? pick_heat_bath_lds<SA_HEAT_BATH, 2, uint32_t>(reg_chunk)
                              : pick_heat_bath_lds<SA_HEAT_BATH, 2, uint64_t>(reg_chunk);
        case 4: return pick_heat_bath_lds<SA_HEAT_BATH, 4, uint64_t>(reg_chunk);
        default: return pick_heat_bath_lds<SA_HEAT_BATH, kMaxExpPoly, uint64_t>(reg_chunk);
    }
}

}  // namespace sa
