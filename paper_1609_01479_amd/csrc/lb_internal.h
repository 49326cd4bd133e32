// Internal interface between the C-ABI host layer (lb_api.cpp) and the HIP
// kernels (lb_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lbk {

constexpr int NV = 19;

// Kernel-side view of the parameters, passed by value.
struct KParams {
    int nx, ny, nz;
    int nsites;            // nx*ny*nz
    long long stride;      // elements per distribution component
    double A, B, kappa, gamma;
    double omega_f, omega_g;  // 1/tau
    double rho0;
};

// All launchers enqueue on `s` and return hipGetLastError().
// `fp32` selects the FP32 deviation-storage instantiation; otherwise FP64.
hipError_t launch_init(const KParams& p, bool fp32, void* state, const double* phi0, hipStream_t s);
hipError_t launch_step(const KParams& p, bool fp32, const void* src, void* dst, void* phi,
                       hipStream_t s);
hipError_t launch_moments(const KParams& p, bool fp32, const void* state, double* rho, double* u,
                          double* phi, double* partials, int* nblocks_out, hipStream_t s);
hipError_t launch_sums_final(const double* partials, int nblocks, int ncomp, double* out,
                             bool accumulate, hipStream_t s);
hipError_t launch_export(const KParams& p, bool fp32, const void* state, double* f, double* g,
                         hipStream_t s);
hipError_t launch_import(const KParams& p, bool fp32, void* state, const double* f,
                         const double* g, hipStream_t s);

// Reverse mode.
hipError_t launch_adj_seed(const KParams& p, bool fp32, void* adj, const double* dphi,
                           hipStream_t s);
hipError_t launch_adj_step(const KParams& p, bool fp32, const void* state, void* phi,
                           const void* adj_next, void* adj_prev, void* adj_scratch,
                           double* partials, int* nblocks_out, hipStream_t s);
hipError_t launch_adj_phi0(const KParams& p, bool fp32, const void* adj, double* dphi0,
                           hipStream_t s);

// Upper bound on the block partials any reduction writes (per component).
constexpr int kMaxPartialBlocks = 2048;

}  // namespace lbk
