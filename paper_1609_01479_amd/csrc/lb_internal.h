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
    unsigned stride;       // elements per distribution component; every element
                           // offset in a kernel (component * stride + site, at
                           // most 39 components) fits in 32 bits
    // layout of the f and g regions: element (i, x, y, z) at
    //   x*plane_e + y*ry + (z >> vs)*zb + (z & vm) + i*cs
    unsigned plane_e, ry, zb, vs, vm, cs;
    double A, B, kappa, gamma;
    double omega_f, omega_g;  // 1/tau
    double rho0;
    int xh;     // x-slab shard: planes of halo on each side of the F and G
                // regions (2; the phi_c field has 1), x not periodic; 0: periodic
    int force;  // force coupling: -div Pi as a body force
    int fd;           // finite-difference order parameter (no g)
    double mobility;  // M = Gamma (tau_g - 1/2) of the finite-difference update
};

// Launch geometry of the single-pass step: (y, z) tiles times x segments.
struct TileCfg {
    int tz;                // tile width along z (128 or 64; kFused/tz rows)
    int nty, ntz, ntiles;  // tiles along y, along z, total
    int sx, nseg;          // planes per x segment, number of segments
    int seg_req;           // segment length asked for (<= 0: automatic)
};

// A time level's regions (LB order parameter): F and G of 19*stride
// elements of T each and, in FP32 mode, phi_c (stride 32-bit words: the high
// word of each site's reference order parameter, see lb_device.h).
template <typename T>
struct Lvl {
    T* F;
    T* G;
    unsigned* phic;  // FP32 mode only
};

template <typename T>
inline Lvl<T> level(void* state, const KParams& p, bool ref)
{
    T* base = static_cast<T*>(state);
    Lvl<T> l;
    l.F = base;
    l.G = base + size_t(NV) * p.stride;
    l.phic = ref ? reinterpret_cast<unsigned*>(base + size_t(2 * NV) * p.stride) : nullptr;
    return l;
}

// segment_x <= 0 picks the segment length automatically.
TileCfg tile_config(const KParams& p, int segment_x, bool fp32);

// Fills the layout fields of k (nx, ny, nz and stride set) for an lb_layout.
void set_layout(KParams& k, int layout, int aosoa_len);

// All launchers enqueue on `s` and return hipGetLastError().
// `fp32` selects the FP32 deviation-storage instantiation; otherwise FP64.
// A time level (`state`) is an F region and a G region of 19*stride elements
// each (laid out per KParams) and, in FP32 mode, phi_c[stride] (32-bit
// words, site order).  Order-parameter fields (`phi`) are FP64.
hipError_t launch_init(const KParams& p, bool fp32, void* state, const double* phi0, hipStream_t s);
// variant 0: single-pass fused step; 1: phi pass (phi into phi_work, and in
// FP32 mode the new level's phi_c) + collision pass.
// If sums_out is non-null, also writes the 5 FP64 conserved sums
// [rho, phi, jx, jy, jz] of the source level to sums_out, through block
// partials in `partials` (at least 5 * max(tc.ntiles * tc.nseg,
// kMaxPartialBlocks) doubles).
// phi_src_out (may be null): also store phi of src there (N FP64 values in
// site order, bit-identical to launch_phi's).
// The number of partial blocks the LB-scheme step of `variant` reduces over.
int step_sums_blocks(const KParams& p, const TileCfg& tc, int variant);
hipError_t launch_step(const KParams& p, const TileCfg& tc, bool fp32, int variant,
                       const void* src, void* dst, double* phi_work, double* partials,
                       double* sums_out, double* phi_src_out, hipStream_t s);
// Force coupling: the forcing collision from src to dst.  variant 0: the
// whole step in one pass over (y, z) tiles marching along x (its own 8 x 64
// tiling, segments as tc.seg_req asks), phi summed from the pulled g, Pi in
// LDS; phi of src goes to dst's phi_c field (FP32 mode) and to `phi` if not
// null; with `partials`, the pass also leaves block partials of
// [rho, phi, j + F/2] of src there (force_sums_blocks(p, tc.seg_req) blocks
// of 5).  variant 1: after the phi pass, which left phi (all sites, FP64) of
// src in `phi` and dst's phi_c, one site per thread, Pi formed at each face
// neighbour (`partials` unused).  Bit-identical levels.
hipError_t launch_force_collide(const KParams& p, const TileCfg& tc, bool fp32, int variant,
                                const void* src, void* dst, double* phi, double* partials,
                                hipStream_t s);
int force_sums_blocks(const KParams& p, int seg_req);
// phi(x) of the post-propagation state held in `state`.
hipError_t launch_phi(const KParams& p, bool fp32, const void* state, double* phi, hipStream_t s);
// work: the FP64 phi field the force coupling needs (`stride` long); unused
// otherwise.
hipError_t launch_moments(const KParams& p, bool fp32, const void* state, double* rho, double* u,
                          double* phi, double* work, double* partials, int* nblocks_out,
                          hipStream_t s);
hipError_t launch_sums_final(const double* partials, int nblocks, int ncomp, double* out,
                             bool accumulate, hipStream_t s);
hipError_t launch_export(const KParams& p, bool fp32, const void* state, double* f, double* g,
                         hipStream_t s);
hipError_t launch_import(const KParams& p, bool fp32, void* state, const double* f,
                         const double* g, hipStream_t s);

// Reverse mode.
// adj: the level seeded (lf = lg = 0, lp = dphi); other: the second level,
// whose lg is zeroed too when tau_g = 1 (the steps then never touch lg).
hipError_t launch_adj_seed(const KParams& p, bool fp32, void* adj, void* other, const double* dphi,
                           hipStream_t s);
// dtheta (may be null): FP64[3] incremented by the step's d/d(A, B, kappa),
// reduced from block partials in `partials` (3 * 1024 doubles; 6 * 1024
// with the force coupling).  The force coupling needs 8 components of
// adj_scratch (the stencil cotangents, then dL/dF).
// phi_given (may be null): phi of `state` (N FP64 values in site order), so
// that no phi pass is needed.
hipError_t launch_adj_step(const KParams& p, bool fp32, const void* state,
                           const double* phi_given, double* phi,
                           const void* adj_next, void* adj_prev, void* adj_scratch,
                           double* partials, double* dtheta, hipStream_t s);
// lp of adj_prev from the stencil cotangents in adj_scratch (a, b_x, b_y,
// b_z, c): lp = a - sum_a D_a b_a + lap c; with dtheta, also
// dtheta[k] += the sum of the nparts block partials of component k < 3 in
// `partials` and, if not null, in `partials2`.
hipError_t launch_adj_stencil(const KParams& p, bool fp32, const void* adj_scratch,
                              void* adj_prev, const double* partials, const double* partials2,
                              int nparts, double* dtheta, hipStream_t s);
// Force coupling: dL/dF (adj_scratch components 5..7) through Pi at the face
// neighbours into the stencil cotangents (components 0..4) of the FP64 phi
// field `phi`; nblocks workgroups, their partials of d/d(A, B, kappa) in
// partials2 (3 * nblocks).
hipError_t launch_adj_force_pi(const KParams& p, bool fp32, const double* phi, void* adj_scratch,
                               double* partials2, int nblocks, hipStream_t s);
// dL/dphi0 from the level in `adj` (LB scheme: lg_0 + lp; FD scheme: lp).
hipError_t launch_adj_phi0(const KParams& p, bool fp32, const void* adj, double* dphi0,
                           hipStream_t s);
// Dense FP64 (19, nx, ny, nz) copies of the level in `adj`: df = lf and
// (LB scheme; null for FD) dg = lg + lp.  Either pointer may be null.
hipError_t launch_adj_export(const KParams& p, bool fp32, const void* adj, double* df, double* dg,
                             hipStream_t s);

// Finite-difference order parameter (lb_fd.hip).  A time level is F
// (19*stride elements, laid out per KParams) then phi (stride FP64 values).
// variant 0: single-pass step with the tiling of tc; 1: collision pass, then
// update pass, with `work` holding mu, u_x, u_y, u_z (4 fields of `stride`:
// FP64, or FP32 with the force coupling in FP32 storage; 4 FP64 fields of
// space).  With sums_out, `partials` needs 5 * max(tc.ntiles * tc.nseg,
// fd_step_partial_blocks(p, segment_x)) doubles; fd_sums_blocks gives the
// exact number of partial blocks the step of `variant` reduces over.
int fd_step_partial_blocks(const KParams& p, int segment_x);
int fd_sums_blocks(const KParams& p, const TileCfg& tc, int variant);
hipError_t launch_fd_init(const KParams& p, bool fp32, void* state, const double* phi0,
                          hipStream_t s);
hipError_t launch_fd_step(const KParams& p, const TileCfg& tc, bool fp32, int variant,
                          const void* src, void* dst, double* work, double* partials,
                          double* sums_out, hipStream_t s);
// Reverse mode of one FD step (stress coupling): adj_prev = J(state)^T adj_next
// in the adjoint-level layout (lf[19], unused g components, lp), with
// `work` (4 FP64 fields of space) taking rho and u of `state`, adj_scratch
// the five stencil cotangents, and dtheta as for launch_adj_step.
hipError_t launch_fd_adj_step(const KParams& p, bool fp32, const void* state, double* work,
                              const void* adj_next, void* adj_prev, void* adj_scratch,
                              double* partials, double* dtheta, hipStream_t s);
hipError_t launch_fd_moments(const KParams& p, bool fp32, const void* state, double* rho,
                             double* u, double* phi, double* partials, int* nblocks_out,
                             hipStream_t s);
hipError_t launch_fd_export(const KParams& p, bool fp32, const void* state, double* f,
                            hipStream_t s);
hipError_t launch_fd_import(const KParams& p, bool fp32, void* state, const double* f,
                            hipStream_t s);

// x-slab shards (lb_halo.hip): bytes of one face buffer, and the copy of a
// face between `buf` and the level `state` -- pack: boundary plane xb and
// the plane behind it (xb - s) into buf; unpack: buf into the halo planes
// xb and xb - s.  s = +1: the face sent up (c_x = +1 populations), s = -1:
// the face sent down.
size_t face_bytes(const KParams& p, bool fp32);
hipError_t launch_face(const KParams& p, bool fp32, void* state, void* buf, int s, int xb,
                       bool pack, hipStream_t st);

// Upper bound on the block partials any reduction writes (per component).
constexpr int kMaxPartialBlocks = 2048;

}  // namespace lbk
