// sa_kernels_quad_mo.hip -- variants and launch of the Metropolis / optimal-transition quad kernel
// (sa_quad_mo.h): one update per four lanes, one wavefront per replica, over the rounds of
// build_rounds.
#include "sa_quad_mo.h"

namespace sa {
namespace {

using QuadFn = void (*)(QuadArgs);

// values per lane of the optimal transition's enumeration: the smallest class holding ceil(W / 4)
template <int kMaxE, bool kNarrow, typename Acc>
QuadFn pick_otm(uint32_t c) {
    if (c <= 8) return quad_mo_kernel<SA_OPT_METROPOLIS, 8, kMaxE, kNarrow, Acc>;
    if (c <= 16) return quad_mo_kernel<SA_OPT_METROPOLIS, 16, kMaxE, kNarrow, Acc>;
    if (c <= 26) return quad_mo_kernel<SA_OPT_METROPOLIS, 26, kMaxE, kNarrow, Acc>;
    return quad_mo_kernel<SA_OPT_METROPOLIS, kQuadMaxR, kMaxE, kNarrow, Acc>;
}

template <bool kNarrow, typename Acc>
QuadFn pick(int rule, uint32_t c, int32_t max_exp) {
    if (rule == SA_METROPOLIS) {   // one proposal: no values per lane
        if (max_exp <= 1) return quad_mo_kernel<SA_METROPOLIS, 8, 1, kNarrow, Acc>;
        if (max_exp <= 2) return quad_mo_kernel<SA_METROPOLIS, 8, 2, kNarrow, Acc>;
        return quad_mo_kernel<SA_METROPOLIS, 8, 4, kNarrow, Acc>;
    }
    // linear energy differences: the optimal move is an end of the range, no enumeration
    if (max_exp <= 1) return quad_mo_kernel<SA_OPT_METROPOLIS, 8, 1, kNarrow, Acc>;
    if (max_exp <= 2) return pick_otm<2, kNarrow, Acc>(c);
    return pick_otm<4, kNarrow, Acc>(c);
}

}  // namespace

int launch_quad_mo(int rule, const QuadArgs &a, int32_t max_width, int32_t max_exp, bool narrow, void *stream,
                   std::string &err) {
    const uint32_t c = ((uint32_t)max_width + 3u) / 4u;
    if (c > (uint32_t)kQuadMaxR || max_exp > 4 || (rule != SA_METROPOLIS && rule != SA_OPT_METROPOLIS) ||
        a.n_rounds < 0 || a.n_rounds % kRoundBatch != 0) {
        err = "quad kernel: unsupported problem shape";
        return SA_EUNSUPPORTED;
    }
    // record products in 32 bits when every coefficient fits them; energy differences in 32 bits
    // where they fit and no exponent exceeds two (as the one-wavefront kernels)
    const bool rec32 = a.P.coef32 != 0;
    QuadFn fn = !rec32                          ? pick<false, uint64_t>(rule, c, max_exp)
                : narrow && max_exp <= 2        ? pick<true, uint32_t>(rule, c, max_exp)
                                                : pick<true, uint64_t>(rule, c, max_exp);
    if (a.n_rounds > 0 && (a.mrec == nullptr || a.mcoef == nullptr)) {
        err = "quad kernel: the rounds' records are missing";
        return SA_EINVAL;
    }
    // the state and, after it, the constant 1 that the records' unused places point at
    const int lds = (int)shared_state_bytes(a.P.n + 1, kQuadWavesMO);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
            return SA_EDEVICE;
        }
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)a.n_reads), dim3(kQuadWavesMO * kWave), (size_t)lds, (hipStream_t)stream,
                       a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

}  // namespace sa
