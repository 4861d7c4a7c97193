// sa_kernels_quad_mo.hip -- Metropolis and optimal-transition variants and launch of the quad
// kernel (sa_quad.h): one update per four lanes over dependency levels, kQuadWavesMO waves per
// replica (the levels of HUIO problems hold about as many variables as one wave has quads).
#include "sa_quad.h"

namespace sa {
namespace {

using QuadFn = void (*)(QuadArgs);

// values per lane of the optimal transition's enumeration: the smallest class holding ceil(W / 4)
template <int kMaxE, typename Acc>
QuadFn pick_otm(uint32_t c) {
    if (c <= 8) return quad_kernel<SA_OPT_METROPOLIS, 8, kMaxE, Acc, kQuadWavesMO>;
    if (c <= 16) return quad_kernel<SA_OPT_METROPOLIS, 16, kMaxE, Acc, kQuadWavesMO>;
    if (c <= 26) return quad_kernel<SA_OPT_METROPOLIS, 26, kMaxE, Acc, kQuadWavesMO>;
    return quad_kernel<SA_OPT_METROPOLIS, kQuadMaxR, kMaxE, Acc, kQuadWavesMO>;
}

template <typename Acc>
QuadFn pick(int rule, uint32_t c, int32_t max_exp) {
    if (rule == SA_METROPOLIS) {   // one proposal: no values per lane
        if (max_exp <= 1) return quad_kernel<SA_METROPOLIS, 8, 1, Acc, kQuadWavesMO>;
        if (max_exp <= 2) return quad_kernel<SA_METROPOLIS, 8, 2, Acc, kQuadWavesMO>;
        return quad_kernel<SA_METROPOLIS, 8, 4, Acc, kQuadWavesMO>;
    }
    if (max_exp <= 1) return pick_otm<1, Acc>(c);
    if (max_exp <= 2) return pick_otm<2, Acc>(c);
    return pick_otm<4, Acc>(c);
}

}  // namespace

int launch_quad_mo(int rule, const QuadArgs &a, int32_t max_width, int32_t max_exp, bool narrow, void *stream,
                   std::string &err) {
    const uint32_t c = ((uint32_t)max_width + 3u) / 4u;
    if (c > (uint32_t)kQuadMaxR || max_exp > 4 || (rule != SA_METROPOLIS && rule != SA_OPT_METROPOLIS)) {
        err = "quad kernel: unsupported problem shape";
        return SA_EUNSUPPORTED;
    }
    // 32-bit energy differences where they fit and no exponent exceeds two (as the one-wavefront kernels)
    QuadFn fn = narrow && max_exp <= 2 ? pick<uint32_t>(rule, c, max_exp) : pick<uint64_t>(rule, c, max_exp);
    const int lds = (int)shared_state_bytes(a.P.n, kQuadWavesMO);
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
