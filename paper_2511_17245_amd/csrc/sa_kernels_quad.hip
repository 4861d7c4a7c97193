// sa_kernels_quad.hip -- variants and launch of the quad heat-bath kernel (sa_quad.h).
#include "sa_quad.h"

namespace sa {
namespace {

using QuadFn = void (*)(QuadArgs);

// values per lane: the smallest class holding ceil(W / 4) (W = 101 takes 26: 104 slots)
template <int kRule, int kMaxE, typename Acc>
QuadFn pick_r(uint32_t c) {
    if (c <= 8) return quad_kernel<kRule, 8, kMaxE, Acc, kQuadWaves>;
    if (c <= 16) return quad_kernel<kRule, 16, kMaxE, Acc, kQuadWaves>;
    if (c <= 26) return quad_kernel<kRule, 26, kMaxE, Acc, kQuadWaves>;
    return quad_kernel<kRule, kQuadMaxR, kMaxE, Acc, kQuadWaves>;
}

template <int kRule>
QuadFn pick(uint32_t c, int32_t max_exp, bool narrow) {
    if (max_exp <= 1) return narrow ? pick_r<kRule, 1, uint32_t>(c) : pick_r<kRule, 1, uint64_t>(c);
    return narrow ? pick_r<kRule, 2, uint32_t>(c) : pick_r<kRule, 2, uint64_t>(c);
}

}  // namespace

int launch_quad(int rule, const QuadArgs &a, int32_t max_width, int32_t max_exp, bool narrow, void *stream,
                std::string &err) {
    const uint32_t c = ((uint32_t)max_width + 3u) / 4u;
    if (c > (uint32_t)kQuadMaxR || max_exp > 2 || (rule != SA_HEAT_BATH && rule != SA_HEAT_BATH_CLOSED)) {
        err = "quad kernel: unsupported problem shape";
        return SA_EUNSUPPORTED;
    }
    QuadFn fn = rule == SA_HEAT_BATH ? pick<SA_HEAT_BATH>(c, max_exp, narrow)
                                     : pick<SA_HEAT_BATH_CLOSED>(c, max_exp, narrow);
    const int lds = (int)shared_state_bytes(a.P.n, kQuadWaves);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
            return SA_EDEVICE;
        }
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)a.n_reads), dim3(kQuadWaves * kWave), (size_t)lds, (hipStream_t)stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

}  // namespace sa
