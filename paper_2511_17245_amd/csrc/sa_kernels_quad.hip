// sa_kernels_quad.hip -- variants and launch of the quad heat-bath kernel (sa_quad.h).
#include "sa_quad.h"

namespace sa {
namespace {

using QuadFn = void (*)(QuadArgs);

// the variant of class R: 16 waves where quad_high allows them, else 8
template <int kRule, int R, int kMaxE, typename Acc, bool kFact>
QuadFn variant() {
    constexpr int kW = quad_high(kRule, R, kMaxE, kFact) ? kQuadWavesHigh : kQuadWaves;
    return quad_kernel<kRule, R, kMaxE, Acc, kW, kFact>;
}

template <int kRule, int kMaxE, typename Acc, bool kFact>
QuadFn pick_r(int32_t r) {
    if (r == 8) return variant<kRule, 8, kMaxE, Acc, false>();   // no factored form below 16
    if (r == 16) return variant<kRule, 16, kMaxE, Acc, kFact>();
    if (r == 26) return variant<kRule, 26, kMaxE, Acc, kFact>();
    return variant<kRule, kQuadMaxR, kMaxE, Acc, kFact>();
}

template <int kRule, bool kFact>
QuadFn pick(int32_t r, int32_t max_exp, bool narrow) {
    if (max_exp <= 1) return narrow ? pick_r<kRule, 1, uint32_t, kFact>(r) : pick_r<kRule, 1, uint64_t, kFact>(r);
    return narrow ? pick_r<kRule, 2, uint32_t, kFact>(r) : pick_r<kRule, 2, uint64_t, kFact>(r);
}

}  // namespace

int launch_quad(int rule, const QuadArgs &a, int32_t max_width, int32_t max_exp, bool narrow, void *stream,
                std::string &err) {
    const uint32_t c = ((uint32_t)max_width + 3u) / 4u;
    if (c > (uint32_t)kQuadMaxR || max_exp > 2 || (rule != SA_HEAT_BATH && rule != SA_HEAT_BATH_CLOSED)) {
        err = "quad kernel: unsupported problem shape";
        return SA_EUNSUPPORTED;
    }
    const int32_t r = quad_r_class(max_width);
    // the factored weights of linear variables (the closed form draws them without weights); the
    // waves per replica follow from the same choice (quad_waves), as the levels were built for
    const bool fact = quad_factored(rule, r, a.uniform_width);
    const int waves = quad_waves(rule, max_width, max_exp, a.uniform_width);
    QuadFn fn = rule == SA_HEAT_BATH_CLOSED ? pick<SA_HEAT_BATH_CLOSED, false>(r, max_exp, narrow)
                : fact                      ? pick<SA_HEAT_BATH, true>(r, max_exp, narrow)
                                            : pick<SA_HEAT_BATH, false>(r, max_exp, narrow);
    const int lds = (int)shared_state_bytes(a.P.n, waves);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
            return SA_EDEVICE;
        }
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)a.n_reads), dim3(waves * kWave), (size_t)lds, (hipStream_t)stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

}  // namespace sa
