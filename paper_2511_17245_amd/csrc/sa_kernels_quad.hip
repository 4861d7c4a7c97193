// sa_kernels_quad.hip -- variants and launch of the quad heat-bath kernel (sa_quad.h).
#include "sa_quad.h"

namespace sa {
namespace {

using QuadFn = void (*)(QuadArgs);

// values per lane: the smallest class holding ceil(W / 4) (W = 101 takes 26: 104 slots)
constexpr uint32_t kClasses[] = {8, 16, 26, (uint32_t)kQuadMaxR};
uint32_t r_class(uint32_t c) {
    for (uint32_t r : kClasses)
        if (c <= r) return r;
    return (uint32_t)kQuadMaxR;
}

template <int kRule, int kMaxE, typename Acc, bool kFact>
QuadFn pick_r(uint32_t r) {
    if (r == 8) return quad_kernel<kRule, 8, kMaxE, Acc, kQuadWaves>;   // no factored form below 16
    if (r == 16) return quad_kernel<kRule, 16, kMaxE, Acc, kQuadWaves, kFact>;
    if (r == 26) return quad_kernel<kRule, 26, kMaxE, Acc, kQuadWaves, kFact>;
    return quad_kernel<kRule, kQuadMaxR, kMaxE, Acc, kQuadWaves, kFact>;
}

template <int kRule, bool kFact>
QuadFn pick(uint32_t r, int32_t max_exp, bool narrow) {
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
    const uint32_t r = r_class(c);
    // the factored weights of linear variables: one width for every variable, at most r / 4 of the
    // quad's 4 r places past the range (the closed form draws linear variables without weights)
    const bool fact = rule == SA_HEAT_BATH && r >= 16 && a.uniform_width > 0 &&
                      4u * r - (uint32_t)a.uniform_width <= r / 4u;
    QuadFn fn = rule == SA_HEAT_BATH_CLOSED ? pick<SA_HEAT_BATH_CLOSED, false>(r, max_exp, narrow)
                : fact                      ? pick<SA_HEAT_BATH, true>(r, max_exp, narrow)
                                            : pick<SA_HEAT_BATH, false>(r, max_exp, narrow);
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
