// HBM bandwidth probe: the practical ceiling the step kernels are measured
// against, in the spirit of the STREAM calibration the paper uses for its
// roofline analysis (Sec. 4): a plain streaming copy b = a of 16-byte vectors,
// grid-stride, enough workgroups to fill every CU.
#include <hip/hip_runtime.h>

#include "lb.h"

namespace {

__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ a, float4* __restrict__ b,
                                                size_t n)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

}  // namespace

extern "C" lb_status lb_copy_probe(const void* src_dev, void* dst_dev, size_t bytes, void* hip_stream)
{
    if (!src_dev || !dst_dev || bytes % 16 != 0) return LB_EINVAL;
    if ((reinterpret_cast<uintptr_t>(src_dev) | reinterpret_cast<uintptr_t>(dst_dev)) % 256)
        return LB_EALIGN;
    const size_t n = bytes / 16;
    k_copy16<<<256 * 16, 256, 0, static_cast<hipStream_t>(hip_stream)>>>(
        static_cast<const float4*>(src_dev), static_cast<float4*>(dst_dev), n);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EHIP;
}
