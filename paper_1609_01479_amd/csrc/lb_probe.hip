// HBM bandwidth probe: the practical ceiling the step kernels are measured
// against, in the spirit of the STREAM calibration the paper uses for its
// roofline analysis (Sec. 4): a streaming copy b = a of 16-byte vectors.
// Each thread moves 4 vectors per trip (all loads issued before the stores),
// non-temporal, over a grid of 2 workgroups per CU -- the fastest of the copy
// shapes measured on MI355X (plain grid-stride copies at 256..16384
// workgroups were slower).  Over 1 GiB it moved 5.9-6.3 TB/s on the boxes
// used; its rate falls as the buffers grow (bench.py --footprint-sweep).
#include <hip/hip_runtime.h>

#include "lb.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;
constexpr int kProbeGrid = 512;

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeBlock) void k_copy16(const v4f* __restrict__ a, v4f* __restrict__ b,
                                                        size_t n)
{
    const size_t trip = size_t(gridDim.x) * kProbeBlock * kProbeUnroll;
    for (size_t base = size_t(blockIdx.x) * kProbeBlock * kProbeUnroll + threadIdx.x; base < n;
         base += trip) {
        v4f v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; u++) {
            const size_t i = base + size_t(u) * kProbeBlock;
            if (i < n) v[u] = __builtin_nontemporal_load(a + i);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; u++) {
            const size_t i = base + size_t(u) * kProbeBlock;
            if (i < n) __builtin_nontemporal_store(v[u], b + i);
        }
    }
}

}  // namespace

extern "C" lb_status lb_copy_probe(const void* src_dev, void* dst_dev, size_t bytes, void* hip_stream)
{
    if (!src_dev || !dst_dev || bytes % 16 != 0) return LB_EINVAL;
    if ((reinterpret_cast<uintptr_t>(src_dev) | reinterpret_cast<uintptr_t>(dst_dev)) % 256)
        return LB_EALIGN;
    const size_t n = bytes / 16;
    if (n == 0) return LB_OK;
    k_copy16<<<kProbeGrid, kProbeBlock, 0, static_cast<hipStream_t>(hip_stream)>>>(
        static_cast<const v4f*>(src_dev), static_cast<v4f*>(dst_dev), n);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_EHIP;
}
