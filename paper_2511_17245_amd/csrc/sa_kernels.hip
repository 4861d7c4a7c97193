// sa_kernels.hip -- launch geometry and dispatch of the plain annealing kernels, and the energy
// kernel.  The annealing kernels themselves (sa_device.h) are compiled per rule in
// sa_kernels_<rule>.hip; the batched kernel in sa_kernels_batch.hip.
#include <algorithm>

#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {
namespace {

// Energies of stored states, one wavefront per state.
__global__ void __launch_bounds__(256) energy_kernel(DevProblem P, const int32_t *states,
                                                     int32_t n_states, int64_t *out) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int idx = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    if (idx >= n_states) return;
    const int64_t E = energy_part(P, states + (size_t)idx * P.n, lane, kWave);
    if (lane == 0) out[idx] = E;
}

__global__ void __launch_bounds__(256) zero_u64_kernel(uint64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// One thread per read: row r becomes its inclusive prefix sum (modulo 2^64).
__global__ void __launch_bounds__(256) trace_prefix_kernel(uint64_t *trace, int32_t n_reads, int32_t n_cols) {
    const int32_t r = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= n_reads) return;
    uint64_t *row = trace + (size_t)r * (size_t)n_cols;
    uint64_t acc = 0;
    for (int32_t c = 0; c < n_cols; ++c) {
        acc += row[c];
        row[c] = acc;
    }
}

using KernelFn = AnnealKernelFn;

// Variants built for 16 waves per replica (their register needs fit 128 VGPRs): states in LDS,
// every exponent <= 2, at most 8 heat-bath weights per lane, and the closed-form heat bath only
// when every variable takes the closed form.
bool sixteen_waves_ok(int rule, bool in_lds, int reg_chunk, int maxe_class) {
    if (!in_lds || maxe_class > 2) return false;
    if (rule == SA_HEAT_BATH) return reg_chunk >= 1 && reg_chunk <= 8;
    if (rule == SA_HEAT_BATH_CLOSED) return maxe_class == 1;
    if (rule == SA_OPT_METROPOLIS || rule == SA_METROPOLIS) return reg_chunk == 0;
    return true;
}

KernelFn pick_kernel(int rule, bool in_lds, int reg_chunk, int maxe_class, bool narrow, bool sixteen) {
    switch (rule) {
        case SA_METROPOLIS: return metropolis_kernel(in_lds, reg_chunk, narrow, sixteen);
        case SA_HEAT_BATH: return heat_bath_kernel(in_lds, reg_chunk, maxe_class, narrow, sixteen);
        case SA_HEAT_BATH_CLOSED: return heat_bath_closed_kernel(in_lds, reg_chunk, maxe_class, narrow, sixteen);
        case SA_OPT_METROPOLIS: return otm_kernel(in_lds, reg_chunk, maxe_class, narrow, sixteen);
        default: return nullptr;
    }
}

}  // namespace

int maxe_class_of(int32_t max_exp) {
    if (max_exp <= 1) return 1;
    if (max_exp <= 2) return 2;
    if (max_exp <= 4) return 4;
    return kMaxExpPoly;
}

int64_t shared_state_bytes(int32_t n, int G) {
    return (((int64_t)n + 1) & ~(int64_t)1) * (int64_t)sizeof(int32_t) + (int64_t)G * (int64_t)sizeof(int64_t);
}

LaunchChoice choose_launch(int rule, int32_t n, int32_t n_reads, int32_t max_width, int32_t max_exp,
                           int device, int win_waves, bool narrow_ok, int32_t otm_enum_max, bool dense) {
    LaunchChoice lc;
    int cus = 256, max_lds = 65536;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    const int64_t per_wave = (int64_t)n * (int64_t)sizeof(int32_t);
    const bool heat_bath = rule == SA_HEAT_BATH || rule == SA_HEAT_BATH_CLOSED;
    const int64_t chunk = ((int64_t)max_width + kWave - 1) / kWave;
    // heat bath: weights per lane kept in registers; optimal transition: 1 = wide-range argmin
    // from forward differences; Metropolis: 1 = dense form with prefetched coupling rows
    const bool otm_wide = rule == SA_OPT_METROPOLIS && max_width > otm_enum_max;
    const int reg_in_lds =
        heat_bath && !(rule == SA_HEAT_BATH_CLOSED && max_exp <= 1)
            ? (chunk <= 1 ? 1 : chunk <= 2 ? 2 : chunk <= 8 ? 8 : chunk <= kHeatBathRegChunk ? 32 : 0)
            : (otm_wide || (rule == SA_METROPOLIS && dense) ? 1 : 0);
    if (win_waves == 16 && !(shared_state_bytes(n, 16) <= max_lds &&
                             sixteen_waves_ok(rule, true, reg_in_lds, maxe_class_of(max_exp))))
        win_waves = 8;  // no 16-wave build of this variant: the next width gives the same result
    if (win_waves > 1 && shared_state_bytes(n, win_waves) <= max_lds) {
        // one replica per workgroup, its G waves share the state
        lc.win_waves = win_waves;
        lc.waves_per_group = win_waves;
        lc.groups = n_reads;
        lc.state_in_lds = true;
        lc.lds_bytes = (int)shared_state_bytes(n, win_waves);
    } else {
        // spread replicas over all compute units first, then stack them (up to 4 waves per group)
        int wpg = n_reads / (cus > 0 ? cus : 1);
        wpg = wpg < 1 ? 1 : (wpg > 4 ? 4 : wpg);
        while (wpg > 1 && per_wave * wpg > max_lds) --wpg;
        lc.win_waves = 1;
        lc.state_in_lds = per_wave * wpg <= max_lds;
        lc.waves_per_group = wpg;
        lc.groups = (n_reads + wpg - 1) / wpg;
        lc.lds_bytes = lc.state_in_lds ? (int)(per_wave * wpg) : 0;
        if (dense && lc.state_in_lds && n <= 1024) {
            // the dense form keeps the coefficient cache (8 bytes per variable) after the states,
            // with fewer replicas per workgroup if needed.  Each accepted move then updates N
            // cached sums; above N = 1024 (16 per lane) that costs more than the row product it
            // saves at every visit (measured on the N = 4096, W = 2001 heat bath: 677 against 400 ms)
            auto cache_bytes = [&](int w) { return ((((int64_t)w * n + 1) & ~(int64_t)1) * 4) + (int64_t)w * n * 8; };
            int w = wpg;
            while (w > 1 && cache_bytes(w) > max_lds) --w;
            if (cache_bytes(w) <= max_lds) {
                lc.dense_cache = true;
                lc.waves_per_group = w;
                lc.groups = (n_reads + w - 1) / w;
                lc.lds_bytes = (int)cache_bytes(w);
            }
        }
    }
    const int reg = lc.state_in_lds ? reg_in_lds : 0;
    lc.maxe_class = lc.state_in_lds ? maxe_class_of(max_exp)
                                    : (heat_bath ? kMaxExpPoly : rule == SA_OPT_METROPOLIS ? 4 : 1);
    lc.reg_chunk = reg;
    lc.narrow = narrow_ok && lc.state_in_lds && lc.maxe_class <= 2 && !otm_wide;
    lc.variant = (lc.win_waves == 16 ? 1000000 : 0) + rule * 100000 + (lc.narrow ? 10000 : 0) +
                 (lc.dense_cache ? 5000 : 0) + lc.maxe_class * 100 + reg * 2 + (lc.state_in_lds ? 1 : 0);
    return lc;
}

int launch_anneal(int rule, const AnnealArgs &a, const LaunchChoice &lc, void *stream,
                  std::string &err) {
    KernelFn fn = pick_kernel(rule, lc.state_in_lds, lc.reg_chunk, lc.maxe_class, lc.narrow, lc.win_waves == 16);
    if (!fn) {
        err = "unknown rule";
        return SA_EINVAL;
    }
    if (lc.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           lc.lds_bytes);
        if (e != hipSuccess) {
            err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
            return SA_EDEVICE;
        }
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)lc.groups), dim3((unsigned)(lc.waves_per_group * kWave)),
                       (size_t)lc.lds_bytes, (hipStream_t)stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

int launch_zero_u64(uint64_t *p, int64_t n, void *stream, std::string &err) {
    if (n <= 0) return SA_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

int launch_trace_prefix(uint64_t *trace, int32_t n_reads, int32_t n_cols, void *stream, std::string &err) {
    if (n_reads <= 0 || n_cols <= 0) return SA_OK;
    hipLaunchKernelGGL(trace_prefix_kernel, dim3((unsigned)((n_reads + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, trace, n_reads, n_cols);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

int launch_energy(const DevProblem &P, const int32_t *states, int32_t n_states, int64_t *out,
                  void *stream, std::string &err) {
    const int per_group = 4;
    const int groups = (n_states + per_group - 1) / per_group;
    hipLaunchKernelGGL(energy_kernel, dim3((unsigned)groups), dim3(per_group * kWave), 0,
                       (hipStream_t)stream, P, states, n_states, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("kernel launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

}  // namespace sa

