// Site sweep of the persistent (one resident round of workgroups) adjoint
// kernels.  Workgroups are dispatched round-robin over the 8 XCDs, each with
// its own L2; here the workgroups of XCD k take the k-th contiguous eighth
// of the sites and sweep it together, one workgroup-width of sites each per
// round.  The x-neighbour planes that a site gathers (phi, u, lambda_phi,
// dL/dF) were then processed by the same XCD in the previous round or will
// be in the next one, except at the two ends of each eighth; with the
// plain interleaved order every second such plane belonged to another XCD
// and was fetched from memory again.  (A grid that is not a multiple of 8
// falls back to the interleaved order.)
#pragma once

#include <hip/hip_runtime.h>

namespace lbk {
namespace dev {

struct XcdSweep {
    int s;       // this thread's current site
    int end;     // one past the last site of its XCD's eighth
    int stride;  // sites per round of the XCD's workgroups
};

__device__ __forceinline__ XcdSweep xcd_sweep(int nsites, int block_threads)
{
    const int b = blockIdx.x, nb = gridDim.x;
    if (nb & 7) return XcdSweep{b * block_threads + int(threadIdx.x), nsites, nb * block_threads};
    const int k = b & 7, per_xcd = nb >> 3, local = b >> 3;
    const int per = (nsites + 7) / 8;
    const int begin = k * per;
    const int end = begin + per < nsites ? begin + per : nsites;
    return XcdSweep{begin + local * block_threads + int(threadIdx.x), end, per_xcd * block_threads};
}

}  // namespace dev
}  // namespace lbk
