// sa_kernels_batch.hip -- the persistent batched kernel (many problems in one launch) with 32-bit
// states, and the batched launch.
#include "sa_device.h"
#include "sa_kernel_table.h"

namespace sa {
namespace {

// Sets the batch's task counter to zero (a kernel, so that graph replays stay plain kernel nodes).
__global__ void reset_counter_kernel(uint32_t *counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

}  // namespace

// 32-bit states; 16-bit states are built in sa_kernels_batch16.hip.
BatchKernelFn batch_kernel_z32(int maxe_class, bool narrow) {
    switch (maxe_class) {
        case 1: return narrow ? batch_kernel<1, uint32_t, int32_t> : batch_kernel<1, uint64_t, int32_t>;
        case 2: return narrow ? batch_kernel<2, uint32_t, int32_t> : batch_kernel<2, uint64_t, int32_t>;
        case 4: return batch_kernel<4, uint64_t, int32_t>;
        default: return batch_kernel<kMaxExpPoly, uint64_t, int32_t>;
    }
}

int launch_batch(const BatchArgs &b, const BatchLaunch &bl, void *stream, std::string &err) {
    BatchKernelFn fn = bl.z16 ? batch_kernel_z16(bl.maxe_class, bl.narrow) : batch_kernel_z32(bl.maxe_class, bl.narrow);
    const int lds = b.lds_words * (int)sizeof(int32_t);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
            return SA_EDEVICE;
        }
    }
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, b.counter);
    hipLaunchKernelGGL(fn, dim3((unsigned)bl.groups), dim3((unsigned)(kBatchWaves * kWave)), (size_t)lds,
                       (hipStream_t)stream, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("batch launch: ") + hipGetErrorString(e);
        return SA_EDEVICE;
    }
    return SA_OK;
}

}  // namespace sa
