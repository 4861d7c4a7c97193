// sa_kernels_heat_bath_closed.hip -- heat-bath variants with the closed-form draw for linear
// variables (Sec. 3.3.2); variables with powers keep the enumeration.
#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {

AnnealKernelFn heat_bath_closed_kernel(bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen) {
    if (sixteen)
        return narrow ? anneal_kernel<SA_HEAT_BATH_CLOSED, true, 0, 1, uint32_t, 1024>
                      : anneal_kernel<SA_HEAT_BATH_CLOSED, true, 0, 1, uint64_t, 1024>;
    if (!in_lds) return anneal_kernel<SA_HEAT_BATH_CLOSED, false, 0, kMaxExpPoly, uint64_t, 512>;
    switch (maxe_class) {
        // every variable linear (class 1): no enumeration code at all
        case 1: return narrow ? anneal_kernel<SA_HEAT_BATH_CLOSED, true, 0, 1, uint32_t, 512>
                              : anneal_kernel<SA_HEAT_BATH_CLOSED, true, 0, 1, uint64_t, 512>;
        case 2: return narrow ? pick_heat_bath_lds<SA_HEAT_BATH_CLOSED, 2, uint32_t>(reg_chunk)
                              : pick_heat_bath_lds<SA_HEAT_BATH_CLOSED, 2, uint64_t>(reg_chunk);
        case 4: return pick_heat_bath_lds<SA_HEAT_BATH_CLOSED, 4, uint64_t>(reg_chunk);
        default: return pick_heat_bath_lds<SA_HEAT_BATH_CLOSED, kMaxExpPoly, uint64_t>(reg_chunk);
    }
}

}  // namespace sa
