// sa_kernel_table.h -- the kernel variants: one getter per rule for the plain launch, one per state
// width for the batched launch.  Each is compiled in a file of its own (sa_kernels_<rule>.hip,
// sa_kernels_batch*.hip) so that the files build in parallel; a getter returns nullptr for a
// combination that is not built.
#pragma once

#include "sa_internal.h"

namespace sa {

using AnnealKernelFn = void (*)(AnnealArgs);

// in_lds: states in LDS; reg_chunk: heat-bath weights per lane kept in registers (0: recomputed),
// for Metropolis and the optimal transition 1 selects the dense-form / wide-range argmin variant;
// maxe_class: 1, 2, 4 or kMaxExpPoly; narrow: 32-bit energy differences; sixteen: 1024-thread
// workgroups (16 cooperating waves).
AnnealKernelFn metropolis_kernel(bool in_lds, int reg_chunk, bool narrow, bool sixteen);
AnnealKernelFn heat_bath_kernel(bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen);
AnnealKernelFn heat_bath_closed_kernel(bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen);
AnnealKernelFn otm_kernel(bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen);

// The batched kernel for the batch's exponent class and integer width, with 16- or 32-bit states.
using BatchKernelFn = void (*)(BatchArgs);
BatchKernelFn batch_kernel_z16(int maxe_class, bool narrow);
BatchKernelFn batch_kernel_z32(int maxe_class, bool narrow);

}  // namespace sa
