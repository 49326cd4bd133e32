// Finite-difference order parameter (LB_OP_FD): the state is the LB
// distribution f and a field phi, which follows a conservative Cahn-Hilliard
// update with upwind advection -- the binary-fluid counterpart of the paper's
// "Advection" (a stencil of fluxes) and order-parameter update (local)
// kernels, Sec. 2.1.1.  Two kernels per step:
//
//   k_fd_collide (one site per thread): pull of f, 7-point stencil of phi,
//     mu and Pi, collision of f with Pi in f^eq and its store; mu and
//     u = j/rho into work fields (FP64; FP32 with the force coupling in
//     FP32 storage); optionally the block partials of the source level's
//     conserved sums.
//   k_fd_update: marching along x, the fluxes through each site's six faces
//     from phi, mu and u of the site and its face neighbours,
//       J_a(x + e_a/2) = u_f (u_f > 0 ? phi(x) : phi(x + e_a)) - M (mu(x + e_a) - mu(x)),
//       u_f = (u_a(x) + u_a(x + e_a)) / 2,
//     and phi(t+1) = phi - sum_a [J_a(x + e_a/2) - J_a(x - e_a/2)].
//
// Each face flux is evaluated by both sites that share it, with the same
// instructions on the same operands, so the two values are identical and
// sum phi changes only by the rounding of each site's own update.
//
// With the force coupling (the paper's arrangement: the stress divergence
// acts on the fluid) the collision forms F = -div Pi from the phi field and
// collides f with it, and the fluxes use u = (j + F/2)/rho: one marching
// kernel, k_fd_force_fused, with Pi staged in LDS and mu, u and F also formed
// on the tile's face ring (LB_KERNEL_FUSED), or k_fd_collide one site per
// thread and then k_fd_update (LB_KERNEL_TWO_PASS), bit-identical.
//
// Time level: F (19*stride elements of T in the layout of didx(); FP32 mode
// stores f - w rho0) followed by phi (stride FP64 values in site order).
// Floating-point contraction within one source expression only (including
// the shared device functions this translation unit inlines): a multiply and
// an add written in one expression become one fused multiply-add in every
// kernel alike, so the single-pass and two-kernel paths round every
// expression the same way.  The compiler's default also fuses across
// statements, and did so differently in different kernels; with no
// contraction at all the force-coupled single pass ran 5% (FP32 storage) and
// 2.5% (FP64) slower.
#pragma clang fp contract(on)

#include <type_traits>

#include "lb_device.h"
#include "lb_sweep.h"

namespace lbk {

using namespace dev;

namespace {

template <typename T>
struct FdLvl {
    T* F;
    double* phi;
};

template <typename T>
FdLvl<T> fd_level(void* state, const KParams& p)
{
    T* base = static_cast<T*>(state);
    return FdLvl<T>{base, reinterpret_cast<double*>(base + size_t(NV) * p.stride)};
}

// rho = rho0, u = 0, phi = phi0.
template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_fd_init(KParams p, T* __restrict__ F,
                                                    double* __restrict__ phi,
                                                    const double* __restrict__ phi0)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
#pragma unroll
    for (int i = 0; i < NV; i++) F[dist_own(p, q, i)] = DEV ? T(0) : T(weight(i) * p.rho0);
    phi[s] = phi0[s];
}

// mu = A phi + B phi^3 - kappa lap phi (FP64), one expression for every kernel.
// The expression of chem_stress's mu, so that the force-coupled single pass
// can take mu from its Pi evaluation and stay bit-identical to the two-kernel
// path.
__device__ __forceinline__ double fd_mu(const KParams& p, double c, double lap)
{
    const double c2 = c * c;
    return p.A * c + p.B * c2 * c - p.kappa * lap;
}

// Element type of the collision pass's work fields (mu, u_x, u_y, u_z): FP64,
// except with the force coupling in FP32 storage, where u is an FP32 value
// already and mu is rounded to FP32 (the stress coupling's two passes stay
// bit-identical to its single-pass kernel, which keeps mu in FP64).
template <typename T, bool FORCE>
using FdWork = typename std::conditional<FORCE && std::is_same<T, float>::value, float, double>::type;

// Work fields (each `stride` FP64 values): mu, u_x, u_y, u_z.  FORCE: the
// force coupling, F = -div Pi from the phi field (force_from_phi), the
// forcing collision of f, u = (j + F/2)/rho, and momentum sums of j + F/2.
template <typename T, bool DEV, bool FORCE>
__global__ __launch_bounds__(kBlock) void k_fd_collide(KParams p, const T* __restrict__ sF,
                                                       const double* __restrict__ sphi,
                                                       T* __restrict__ dF,
                                                       FdWork<T, FORCE>* __restrict__ work,
                                                       double* __restrict__ partials)
{
    using W = FdWork<T, FORCE>;
    const int s = xcd_block() * kBlock + threadIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (s < p.nsites) {
        const Geo q = geo_of(p, s);
        T f[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) f[i] = sF[dist_pull(p, q, i)];
        const double c = sphi[s];
        const Stencil st = stencil(c, sphi[site_of(p, q.xp, q.y, q.z)], sphi[site_of(p, q.xm, q.y, q.z)],
                                   sphi[site_of(p, q.x, q.yp, q.z)], sphi[site_of(p, q.x, q.ym, q.z)],
                                   sphi[site_of(p, q.x, q.y, q.zp)], sphi[site_of(p, q.x, q.y, q.zm)]);
        double F[3] = {0.0, 0.0, 0.0};
        if (FORCE) force_from_phi(p, q, sphi, F);
        if (partials) {
            // FP64 moments of the source level, in index order
            double b = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const double v = double(f[i]);
                b += v;
                jx += CX[i] * v;
                jy += CY[i] * v;
                jz += CZ[i] * v;
            }
            acc[0] = DEV ? p.rho0 + b : b;
            acc[1] = c;
            acc[2] = FORCE ? jx + 0.5 * F[0] : jx;
            acc[3] = FORCE ? jy + 0.5 * F[1] : jy;
            acc[4] = FORCE ? jz + 0.5 * F[2] : jz;
        }
        const Vel<T> u = FORCE ? collide_force_f<T, DEV>(p, f, F) : collide_f<T, DEV>(p, f, st);
        // the new level is not read in this launch
#pragma unroll
        for (int i = 0; i < NV; i++) __builtin_nontemporal_store(f[i], &dF[dist_own(p, q, i)]);
        work[s] = W(fd_mu(p, c, st.lap));
        work[p.stride + s] = W(u.x);
        work[2 * p.stride + s] = W(u.y);
        work[3 * p.stride + s] = W(u.z);
    }
    if (partials) block_partials<5>(acc, partials);
}

// Flux through the face between L and L + e_a (R).  Explicit fma: both sites
// of the face evaluate exactly these instructions.
__device__ __forceinline__ double fd_flux(double phiL, double phiR, double uL, double uR,
                                          double muL, double muR, double M)
{
    const double uf = 0.5 * (uL + uR);
    const double up = uf > 0.0 ? phiL : phiR;
    const double dif = M * (muR - muL);
    return __builtin_fma(uf, up, -dif);
}

// Update pass, marching along x: a workgroup owns a kFdTY x kFdTZ tile of
// (y, z) columns and a segment of x planes; each thread keeps phi, mu and u_x
// of planes x-1, x, x+1 of its column in registers, so the x-neighbour
// fields are read from HBM once (one site per thread would need three
// planes of five fields, more than an XCD's L2, and read them twice).  The
// y and z neighbours are in the same plane, read by the neighbouring threads
// and tiles at about the same time (cache hits).  No LDS and no barriers:
// threads outside the lattice return at once.
constexpr int kFdTY = 4, kFdTZ = 64;
static_assert(kFdTY * kFdTZ == kBlock, "update tile must match the block");

// 8 waves per SIMD (at most 64 VGPRs): the ~2048 workgroups then run in one
// round on 256 CUs instead of 1.33.  W: the work fields' element type.
template <typename W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_fd_update(
    KParams p, int ntz, int ntiles, int sx, const double* __restrict__ sphi,
    const W* __restrict__ work, double* __restrict__ dphi)
{
    const int b = xcd_block();
    const int seg = b / ntiles, tile = b - seg * ntiles;
    const int y = (tile / ntz) * kFdTY + int(threadIdx.x) / kFdTZ;
    const int z = (tile % ntz) * kFdTZ + int(threadIdx.x) % kFdTZ;
    if (y >= p.ny || z >= p.nz) return;
    const int x0 = seg * sx, x1 = min(p.nx, x0 + sx);
    // (FP32 work fields widen exactly to FP64 on load)
    const W* __restrict__ mu = work;
    const W* __restrict__ ux = work + p.stride;
    const W* __restrict__ uy = work + 2 * size_t(p.stride);
    const W* __restrict__ uz = work + 3 * size_t(p.stride);
    const double M = p.mobility;
    const int plane = p.ny * p.nz;
    const int oc = y * p.nz + z;
    const int oym = wrapm(y, p.ny) * p.nz + z, oyp = wrapp(y, p.ny) * p.nz + z;
    const int ozm = y * p.nz + wrapm(z, p.nz), ozp = y * p.nz + wrapp(z, p.nz);
    const int sm = wrapm(x0, p.nx) * plane + oc;
    double pm = sphi[sm], mm = mu[sm], um = ux[sm];
    const int s0 = x0 * plane + oc;
    double pc = sphi[s0], mc = mu[s0], uc = ux[s0];
    for (int x = x0; x < x1; x++) {
        const int sc = x * plane;
        const int sp = wrapp(x, p.nx) * plane + oc;
        const double pp = sphi[sp], mp = mu[sp], up = ux[sp];
        double div = 0.0;
        div += fd_flux(pc, pp, uc, up, mc, mp, M) - fd_flux(pm, pc, um, uc, mm, mc, M);
        const double uyc = uy[sc + oc];
        div += fd_flux(pc, sphi[sc + oyp], uyc, uy[sc + oyp], mc, mu[sc + oyp], M)
             - fd_flux(sphi[sc + oym], pc, uy[sc + oym], uyc, mu[sc + oym], mc, M);
        const double uzc = uz[sc + oc];
        div += fd_flux(pc, sphi[sc + ozp], uzc, uz[sc + ozp], mc, mu[sc + ozp], M)
             - fd_flux(sphi[sc + ozm], pc, uz[sc + ozm], uzc, mu[sc + ozm], mc, M);
        dphi[sc + oc] = pc - div;
        pm = pc; mm = mc; um = uc;
        pc = pp; mc = mp; uc = up;
    }
}

// ---------------------------------------------------------------------------
// Single-pass step (LB_KERNEL_FUSED): both passes in one kernel, the
// collision one plane ahead of the flux update.  A workgroup of kFdFused
// threads owns a TY x TZ tile of (y, z) columns (the single-pass LB
// kernel's tiling) and marches over its x segment [x0, x1).  For plane P it
//   (a) stores phi(P+1) on the tile plus two cells around it into a 4-plane
//       LDS ring (loaded into registers one plane earlier, so the loads are
//       in flight across the previous plane's work), loads phi(P+2) and
//       issues the pulls of the own site of plane P, which then overlap the
//       barrier;
//   (c) collides f at the tile's sites of plane P (stencil from the ring),
//       keeps mu(P) and u(P) of the thread's own column in registers and
//       writes mu, u_y, u_z to a 2-plane LDS ring; the first 2(TY + TZ)
//       threads also form mu and the face-normal velocity on the tile's
//       face ring (rows y0-1, y0+TY; columns z0-1, z0+TZ) from their own
//       pulls, which hit in cache;
//   (e) updates phi at plane P-1 from the fluxes through its six faces.
// Planes x0-1 and x1 only supply mu and u_x of the own column (nothing is
// stored for them).  Tile cells beyond a ragged lattice edge stand for the
// periodic images of the sites there: they compute but store nothing.
// Every value is formed with the same arithmetic as the two-kernel path, so
// both paths give bit-identical levels.
constexpr int kFdFused = 512;

template <int TZ>
struct FdTile {
    static constexpr int TY = kFdFused / TZ;
    static constexpr int BY = TY + 4, BZ = TZ + 4;  // phi box: two cells around the tile
    static constexpr int RY = TY + 2, RZ = TZ + 2;  // tile and its face ring
    static constexpr int NBOX = BY * BZ;
    static constexpr int NRING = 2 * (TY + TZ);
    static constexpr int BOXPT = (NBOX + kFdFused - 1) / kFdFused;
};

__device__ __forceinline__ int wrap_any(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

template <typename T, bool DEV, int TZ>
__global__ __launch_bounds__(kFdFused) void k_fd_fused(KParams p, TileCfg tc,
                                                       const T* __restrict__ sF,
                                                       const double* __restrict__ sphi,
                                                       T* __restrict__ dF,
                                                       double* __restrict__ dphi,
                                                       double* __restrict__ partials)
{
    using G = FdTile<TZ>;
    constexpr int TY = G::TY, BZ = G::BZ, RZ = G::RZ;
    __shared__ double s_phi[4][G::NBOX];
    __shared__ double s_mu[2][G::RY * RZ];
    __shared__ double s_uy[2][G::RY * RZ];
    __shared__ double s_uz[2][G::RY * RZ];

    const int t = threadIdx.x;
    const int b = xcd_block();
    const int seg = b / tc.ntiles, tile = b - seg * tc.ntiles;
    const int y0 = (tile / tc.ntz) * TY, z0 = (tile % tc.ntz) * TZ;
    const int x0 = seg * tc.sx, x1 = min(p.nx, x0 + tc.sx);
    const int plane = p.ny * p.nz;

    // own tile cell
    const int ly = t / TZ, lz = t % TZ;
    const int yg = wrap_any(y0 + ly, p.ny), zg = wrap_any(z0 + lz, p.nz);
    const bool valid = y0 + ly < p.ny && z0 + lz < p.nz;
    const int bo = (ly + 2) * BZ + (lz + 2);
    const int ro = (ly + 1) * RZ + (lz + 1);
    // phi box cells loaded by this thread (in-plane offsets; -1: none)
    int boff[G::BOXPT];
#pragma unroll
    for (int k = 0; k < G::BOXPT; k++) {
        const int c = t + k * kFdFused;
        boff[k] = c < G::NBOX
                      ? wrap_any(y0 + c / BZ - 2, p.ny) * p.nz + wrap_any(z0 + c % BZ - 2, p.nz)
                      : -1;
    }
    // face-ring cell of this thread
    const bool ring = t < G::NRING;
    int rly, rlz;
    if (t < TZ) { rly = -1; rlz = t; }
    else if (t < 2 * TZ) { rly = TY; rlz = t - TZ; }
    else if (t < 2 * TZ + TY) { rly = t - 2 * TZ; rlz = -1; }
    else { rly = t - 2 * TZ - TY; rlz = TZ; }
    const bool ring_y = rly < 0 || rly >= TY;  // a row of the ring: u_y; else a column: u_z
    const int ryg = wrap_any(y0 + rly, p.ny), rzg = wrap_any(z0 + rlz, p.nz);
    const int rbo = (rly + 2) * BZ + (rlz + 2);
    const int rro = (rly + 1) * RZ + (rlz + 1);

    const double M = p.mobility;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    auto load_phi = [&](int xp) {
        const int xo = wrap_any(xp, p.nx) * plane;
        double* __restrict__ dst = s_phi[xp & 3];
#pragma unroll
        for (int k = 0; k < G::BOXPT; k++)
            if (boff[k] >= 0) dst[t + k * kFdFused] = sphi[xo + boff[k]];
    };
    load_phi(x0 - 2);
    load_phi(x0 - 1);
    double pre[G::BOXPT];
    {
        const int xo = wrap_any(x0, p.nx) * plane;
#pragma unroll
        for (int k = 0; k < G::BOXPT; k++) pre[k] = boff[k] >= 0 ? sphi[xo + boff[k]] : 0.0;
    }

    // own column: phi, mu, u_x at X-1 and X, u_y and u_z at X, X = P-1
    double phA = 0.0, phB = 0.0, muA = 0.0, muB = 0.0, uxA = 0.0, uxB = 0.0, uyB = 0.0, uzB = 0.0;
    for (int P = x0 - 1; P <= x1; P++) {
        // (a) phi(P+1) into the ring
        {
            double* __restrict__ dst = s_phi[(P + 1) & 3];
#pragma unroll
            for (int k = 0; k < G::BOXPT; k++)
                if (boff[k] >= 0) dst[t + k * kFdFused] = pre[k];
            const int xo = wrap_any(P + 2, p.nx) * plane;
#pragma unroll
            for (int k = 0; k < G::BOXPT; k++) pre[k] = boff[k] >= 0 ? sphi[xo + boff[k]] : 0.0;
        }
        const Geo q = geo_xyz(p, wrap_any(P, p.nx), yg, zg);
        T f[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) f[i] = sF[dist_pull(p, q, i)];
        lds_barrier();
        const double* __restrict__ fm = s_phi[(P - 1) & 3];
        const double* __restrict__ fc = s_phi[P & 3];
        const double* __restrict__ fp = s_phi[(P + 1) & 3];
        const bool interior = P >= x0 && P < x1;
        const int xg = wrap_any(P, p.nx);
        const int w = P & 1;

        // (c) collision of the own cell of plane P
        const double phc = fc[bo];
        const Stencil st = stencil(phc, fp[bo], fm[bo], fc[bo + BZ], fc[bo - BZ], fc[bo + 1], fc[bo - 1]);
        if (partials && interior && valid) {
            double bs = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const double v = double(f[i]);
                bs += v;
                jx += CX[i] * v;
                jy += CY[i] * v;
                jz += CZ[i] * v;
            }
            acc[0] += DEV ? p.rho0 + bs : bs;
            acc[1] += phc;
            acc[2] += jx;
            acc[3] += jy;
            acc[4] += jz;
        }
        const Vel<T> u = collide_f<T, DEV>(p, f, st);
        if (interior && valid)
#pragma unroll
            for (int i = 0; i < NV; i++) __builtin_nontemporal_store(f[i], &dF[dist_own(p, q, i)]);
        const double muP = fd_mu(p, phc, st.lap);
        const double uxP = double(u.x), uyP = double(u.y), uzP = double(u.z);
        s_mu[w][ro] = muP;
        s_uy[w][ro] = uyP;
        s_uz[w][ro] = uzP;
        // the face ring of plane P
        if (ring && interior) {
            const Geo qr = geo_xyz(p, xg, ryg, rzg);
            T fr[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) fr[i] = sF[dist_pull(p, qr, i)];
            const Moments<T> m = moments_of<T, DEV>(p, fr);
            const T ri = T(1) / m.rho;
            const double c = fc[rbo];
            const Stencil sr = stencil(c, fp[rbo], fm[rbo], fc[rbo + BZ], fc[rbo - BZ], fc[rbo + 1], fc[rbo - 1]);
            s_mu[w][rro] = fd_mu(p, c, sr.lap);
            if (ring_y)
                s_uy[w][rro] = double(m.jy * ri);
            else
                s_uz[w][rro] = double(m.jz * ri);
        }
        lds_barrier();

        // (e) phi(t+1) at plane X = P-1
        if (P - 1 >= x0 && valid) {
            const int v = (P - 1) & 1;
            const double* __restrict__ fx = s_phi[(P - 1) & 3];
            const double pc = phB, mc = muB, uc = uxB;
            double div = 0.0;
            div += fd_flux(pc, phc, uc, uxP, mc, muP, M) - fd_flux(phA, pc, uxA, uc, muA, mc, M);
            div += fd_flux(pc, fx[bo + BZ], uyB, s_uy[v][ro + RZ], mc, s_mu[v][ro + RZ], M)
                 - fd_flux(fx[bo - BZ], pc, s_uy[v][ro - RZ], uyB, s_mu[v][ro - RZ], mc, M);
            div += fd_flux(pc, fx[bo + 1], uzB, s_uz[v][ro + 1], mc, s_mu[v][ro + 1], M)
                 - fd_flux(fx[bo - 1], pc, s_uz[v][ro - 1], uzB, s_mu[v][ro - 1], mc, M);
            __builtin_nontemporal_store(pc - div, &dphi[(P - 1) * plane + yg * p.nz + zg]);
        }
        phA = phB; phB = phc;
        muA = muB; muB = muP;
        uxA = uxB; uxB = uxP;
        uyB = uyP; uzB = uzP;
    }
    if (partials) block_partials<5, kFdFused>(acc, partials);
}

template <typename T>
struct FdFused {
    using K = decltype(&k_fd_fused<T, std::is_same<T, float>::value, 128>);
    static K get(int tz)
    {
        constexpr bool DEV = std::is_same<T, float>::value;
        return tz == 64 ? k_fd_fused<T, DEV, 64> : k_fd_fused<T, DEV, 128>;
    }
};

// Single-pass step with the force coupling (LB_KERNEL_FUSED; the paper's
// arrangement: the divergence of the chemical stress acts on the fluid, the
// order parameter follows the finite-difference update).  A workgroup owns an
// 8 x 64 tile of (y, z) columns (the perimeter, and with it the halo work,
// is smaller than a 4 x 128 tile's) and marches over its x segment.  At
// iteration P it
//   (a) stores phi(P+1) of the tile plus three cells around it into a
//       4-plane LDS ring (loaded one iteration earlier) and issues the pulls
//       of f at the own cell of plane V = P-1;
//   (b) forms Pi of plane P on the tile plus two cells around it (the cells
//       that the forces of (c) need), keeping the x row Pi_xa of the own
//       cell and of the thread's face-ring cell in registers (planes P-2 ..
//       P) and the in-plane components in a 2-plane LDS ring;
//   (c) forms F = -div Pi at the own cell of plane V and collides f there
//       (stores it for V in the segment), and mu, u and phi of V for the
//       fluxes: the own column in registers, the tile and its face ring
//       (whose u needs the normal component of F and the ring cell's own
//       pulls, which hit in cache) in a 2-plane LDS ring;
//   (e) updates phi at plane U = P-2 from the fluxes through its six faces
//       (fields of plane U written an iteration earlier).  Two LDS-only
//       barriers per plane would suffice for the data (the collision's
//       x - 1 neighbour phi is carried in registers, so no one reads the ring
//       slot that the next iteration refills); a third after (c) keeps the
//       waves in step and measured 6% (FP32) and 1% (FP64) faster.
// Planes x0-1 and x1 only supply mu and u_x of the own column.  Every value
// is formed with the instructions of the two-kernel path (k_fd_collide with
// the force, then k_fd_update), with mu and u rounded to the work fields'
// type, so both paths give bit-identical levels.
struct FfTile {
    static constexpr int TY = 8, TZ = 64;
    static constexpr int BY = TY + 6, BZ = TZ + 6;   // phi box: three cells around the tile
    static constexpr int NBOX = BY * BZ;
    static constexpr int BOXPT = (NBOX + kFdFused - 1) / kFdFused;
    static constexpr int PY = TY + 4, PZ = TZ + 4;   // Pi box: two cells around the tile
    static constexpr int NPI = PY * PZ;
    static constexpr int RY = TY + 2, RZ = TZ + 2;   // tile and its face ring
    static constexpr int NR = RY * RZ;
    static constexpr int NRING = 2 * (TY + TZ);      // face-ring cells
    // Pi cells beyond the tile and its face ring that a face-ring force
    // needs: the rows y0-2, y0+TY+1 and columns z0-2, z0+TZ+1 next to the
    // ring, and the ring's four corners
    static constexpr int NPIX = 2 * (TY + TZ) + 4;
};
static_assert(FfTile::TY * FfTile::TZ == kFdFused, "one site per thread");
static_assert(FfTile::NPIX <= kFdFused && FfTile::NRING <= kFdFused, "halo cells per thread");

template <typename T, bool DEV>
__global__ __launch_bounds__(kFdFused) void k_fd_force_fused(KParams p, TileCfg tc,
                                                             const T* __restrict__ sF,
                                                             const double* __restrict__ sphi,
                                                             T* __restrict__ dF,
                                                             double* __restrict__ dphi,
                                                             double* __restrict__ partials)
{
    using G = FfTile;
    using W = FdWork<T, true>;
    constexpr int TY = G::TY, TZ = G::TZ, BZ = G::BZ, PZ = G::PZ, RZ = G::RZ;
    __shared__ double s_phi[4][G::NBOX];
    __shared__ double s_pi[2][5][G::NPI];  // Pi_xy, Pi_xz, Pi_yy, Pi_yz, Pi_zz
    __shared__ double s_ph[2][G::NR];
    __shared__ W s_mu[2][G::NR];
    __shared__ W s_uy[2][G::NR];
    __shared__ W s_uz[2][G::NR];

    const int t = threadIdx.x;
    const int b = xcd_block();
    const int seg = b / tc.ntiles, tile = b - seg * tc.ntiles;
    const int y0 = (tile / tc.ntz) * TY, z0 = (tile % tc.ntz) * TZ;
    const int x0 = seg * tc.sx, x1 = min(p.nx, x0 + tc.sx);
    const int plane = p.ny * p.nz;

    // own tile cell
    const int ly = t / TZ, lz = t % TZ;
    const int yg = wrap_any(y0 + ly, p.ny), zg = wrap_any(z0 + lz, p.nz);
    const bool valid = y0 + ly < p.ny && z0 + lz < p.nz;
    const int bo = (ly + 3) * BZ + (lz + 3);
    const int po = (ly + 2) * PZ + (lz + 2);
    const int ro = (ly + 1) * RZ + (lz + 1);
    // phi box cells loaded by this thread (in-plane offsets; -1: none)
    int boff[G::BOXPT];
#pragma unroll
    for (int k = 0; k < G::BOXPT; k++) {
        const int c = t + k * kFdFused;
        boff[k] = c < G::NBOX
                      ? wrap_any(y0 + c / BZ - 3, p.ny) * p.nz + wrap_any(z0 + c % BZ - 3, p.nz)
                      : -1;
    }
    // face-ring cell of this thread (rows y0-1, y0+TY: u_y; columns z0-1,
    // z0+TZ: u_z)
    const bool ring = t < G::NRING;
    int rly, rlz;
    if (t < TZ) { rly = -1; rlz = t; }
    else if (t < 2 * TZ) { rly = TY; rlz = t - TZ; }
    else if (t < 2 * TZ + TY) { rly = t - 2 * TZ; rlz = -1; }
    else { rly = t - 2 * TZ - TY; rlz = TZ; }
    const bool ring_y = rly < 0 || rly >= TY;
    const int ryg = wrap_any(y0 + rly, p.ny), rzg = wrap_any(z0 + rlz, p.nz);
    const int rbo = (rly + 3) * BZ + (rlz + 3);
    const int rpo = (rly + 2) * PZ + (rlz + 2);
    const int rro = (rly + 1) * RZ + (rlz + 1);
    // extra Pi cell of this thread, in Pi-box coordinates
    const bool extra = t < G::NPIX;
    int epy, epz;
    if (t < TZ) { epy = 0; epz = t + 2; }
    else if (t < 2 * TZ) { epy = G::PY - 1; epz = t - TZ + 2; }
    else if (t < 2 * TZ + TY) { epy = t - 2 * TZ + 2; epz = 0; }
    else if (t < 2 * (TY + TZ)) { epy = t - 2 * TZ - TY + 2; epz = PZ - 1; }
    else { const int c = t - 2 * (TY + TZ); epy = (c & 1) ? TY + 2 : 1; epz = (c & 2) ? TZ + 2 : 1; }
    const int ebo = (epy + 1) * BZ + (epz + 1);
    const int epo = epy * PZ + epz;

    const double M = p.mobility;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    auto load_box = [&](int xp, double (&v)[G::BOXPT]) {
        const int xo = wrap_any(xp, p.nx) * plane;
#pragma unroll
        for (int k = 0; k < G::BOXPT; k++) v[k] = boff[k] >= 0 ? sphi[xo + boff[k]] : 0.0;
    };
    auto store_box = [&](int xp, const double (&v)[G::BOXPT]) {
        double* __restrict__ dst = s_phi[xp & 3];
#pragma unroll
        for (int k = 0; k < G::BOXPT; k++)
            if (boff[k] >= 0) dst[t + k * kFdFused] = v[k];
    };
    // Pi at phi-box cell c of plane P (slots P-1, P, P+1)
    auto pi_at = [&](const double* __restrict__ fm, const double* __restrict__ fc,
                     const double* __restrict__ fp, int c, double (&tt)[6]) {
        const Stencil st = stencil(fc[c], fp[c], fm[c], fc[c + BZ], fc[c - BZ], fc[c + 1], fc[c - 1]);
        double mu;
        chem_stress(p, st, &mu, tt);
        return mu;
    };
    auto store_pi = [&](int w, int c, const double (&tt)[6]) {
        s_pi[w][0][c] = tt[1];
        s_pi[w][1][c] = tt[2];
        s_pi[w][2][c] = tt[3];
        s_pi[w][3][c] = tt[4];
        s_pi[w][4][c] = tt[5];
    };

    double pre[G::BOXPT];
    load_box(x0 - 3, pre);
    store_box(x0 - 3, pre);
    load_box(x0 - 2, pre);
    store_box(x0 - 2, pre);
    load_box(x0 - 1, pre);

    // own column: Pi_xa at planes P-2 (A), P-1 (B), P; phi, mu, u at the
    // planes U-1 (A), U (B) of the flux update; the ring cell's Pi_xn
    double pxA[3] = {0.0, 0.0, 0.0}, pxB[3] = {0.0, 0.0, 0.0};
    double rpA = 0.0, rpB = 0.0;
    double phA = 0.0, muA = 0.0, uxA = 0.0;
    double phB = 0.0, muB = 0.0, uxB = 0.0, uyB = 0.0, uzB = 0.0;
    // mu of plane P-1 at the own cell and at the ring cell, from the Pi
    // evaluation of the previous iteration (the stencil is the same)
    double mum = 0.0, rmum = 0.0;
    // flux through the x face below plane U, from the previous iteration
    double fxm = 0.0;
    for (int P = x0 - 2; P <= x1 + 1; P++) {
        const int V = P - 1;  // plane collided
        const bool coll = V >= x0 - 1 && V <= x1;
        const bool inner = V >= x0 && V < x1;
        // (a) phi(P+1) into the ring, phi(P+2) into registers, pulls of V
        store_box(P + 1, pre);
        if (P + 2 <= x1 + 2) load_box(P + 2, pre);
        const Geo q = geo_xyz(p, wrap_any(V, p.nx), yg, zg);
        T f[NV];
        if (coll)
#pragma unroll
            for (int i = 0; i < NV; i++) f[i] = sF[dist_pull(p, q, i)];
        lds_barrier();

        // (b) Pi of plane P
        const double* __restrict__ fm = s_phi[(P - 1) & 3];
        const double* __restrict__ fc = s_phi[P & 3];
        const double* __restrict__ fp = s_phi[(P + 1) & 3];
        const int wp = P & 1;
        double pxP[3], rpP = 0.0, muP, rmuP = 0.0;
        {
            double tt[6];
            muP = pi_at(fm, fc, fp, bo, tt);
            pxP[0] = tt[0];
            pxP[1] = tt[1];
            pxP[2] = tt[2];
            store_pi(wp, po, tt);
        }
        if (ring) {
            double tt[6];
            rmuP = pi_at(fm, fc, fp, rbo, tt);
            rpP = ring_y ? tt[1] : tt[2];  // Pi_xy (row) or Pi_xz (column)
            store_pi(wp, rpo, tt);
        }
        if (extra) {
            double tt[6];
            pi_at(fm, fc, fp, ebo, tt);
            store_pi(wp, epo, tt);
        }
        lds_barrier();

        // (c) force, collision and flux fields of plane V
        const int wv = V & 1;
        double phC = 0.0, muC = 0.0, uxC = 0.0, uyC = 0.0, uzC = 0.0;
        if (coll) {
            // F_a = -sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)] / 2, b = x, y, z in order
            const double* __restrict__ pv = &s_pi[wv][0][0];
            constexpr int KY[3] = {0, 2, 3};  // Pi_xy, Pi_yy, Pi_yz
            constexpr int KZ[3] = {1, 3, 4};  // Pi_xz, Pi_yz, Pi_zz
            double div[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 0; a < 3; a++) div[a] += 0.5 * (pxP[a] - pxA[a]);
#pragma unroll
            for (int a = 0; a < 3; a++)
                div[a] += 0.5 * (pv[KY[a] * G::NPI + po + PZ] - pv[KY[a] * G::NPI + po - PZ]);
#pragma unroll
            for (int a = 0; a < 3; a++)
                div[a] += 0.5 * (pv[KZ[a] * G::NPI + po + 1] - pv[KZ[a] * G::NPI + po - 1]);
            double F[3];
#pragma unroll
            for (int a = 0; a < 3; a++) F[a] = -div[a];
            const double c = fm[bo];
            if (partials && inner && valid) {
                double bs = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
                for (int i = 0; i < NV; i++) {
                    const double vv = double(f[i]);
                    bs += vv;
                    jx += CX[i] * vv;
                    jy += CY[i] * vv;
                    jz += CZ[i] * vv;
                }
                acc[0] += DEV ? p.rho0 + bs : bs;
                acc[1] += c;
                acc[2] += jx + 0.5 * F[0];
                acc[3] += jy + 0.5 * F[1];
                acc[4] += jz + 0.5 * F[2];
            }
            const Vel<T> u = collide_force_f<T, DEV>(p, f, F);
            if (inner && valid)
#pragma unroll
                for (int i = 0; i < NV; i++) __builtin_nontemporal_store(f[i], &dF[dist_own(p, q, i)]);
            const W muw = W(mum), uyw = W(u.y), uzw = W(u.z);
            phC = c;
            muC = double(muw);
            uxC = double(W(u.x));
            uyC = double(uyw);
            uzC = double(uzw);
            s_ph[wv][ro] = c;
            s_mu[wv][ro] = muw;
            s_uy[wv][ro] = uyw;
            s_uz[wv][ro] = uzw;
        }
        if (ring && inner) {
            // mu and the face-normal velocity u_n = (j_n + F_n/2)/rho of the
            // ring cell of plane V, F_n = -div Pi's n component
            const Geo qr = geo_xyz(p, wrap_any(V, p.nx), ryg, rzg);
            T fr[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) fr[i] = sF[dist_pull(p, qr, i)];
            const double* __restrict__ pv = &s_pi[wv][0][0];
            const int ky = ring_y ? 2 : 3, kz = ring_y ? 3 : 4;  // Pi_ny, Pi_nz
            double div = 0.0;
            div += 0.5 * (rpP - rpA);
            div += 0.5 * (pv[ky * G::NPI + rpo + PZ] - pv[ky * G::NPI + rpo - PZ]);
            div += 0.5 * (pv[kz * G::NPI + rpo + 1] - pv[kz * G::NPI + rpo - 1]);
            const double Fn = -div;
            const Moments<T> m = moments_of<T, DEV>(p, fr);
            const T ri = T(1) / m.rho;
            const T un = ((ring_y ? m.jy : m.jz) + T(0.5) * T(Fn)) * ri;
            s_ph[wv][rro] = fm[rbo];
            s_mu[wv][rro] = W(rmum);
            if (ring_y)
                s_uy[wv][rro] = W(un);
            else
                s_uz[wv][rro] = W(un);
        }
        mum = muP;
        rmum = rmuP;
        lds_barrier();  // not needed for the data (see above): keeps the waves in step

        // (e) phi(t+1) at plane U = P-2 (the fields of plane U were written
        // in the previous iteration)
        const int U = P - 2;
        if (U >= x0 && U < x1 && valid) {
            const int v = U & 1;
            const double pc = phB, mc = muB, uc = uxB;
            // the x face below U is the face above U - 1 of the same column
            const double fxp = fd_flux(pc, phC, uc, uxC, mc, muC, M);
            if (U == x0) fxm = fd_flux(phA, pc, uxA, uc, muA, mc, M);
            double dv = 0.0;
            dv += fxp - fxm;
            fxm = fxp;
            dv += fd_flux(pc, s_ph[v][ro + RZ], uyB, double(s_uy[v][ro + RZ]), mc,
                          double(s_mu[v][ro + RZ]), M)
                - fd_flux(s_ph[v][ro - RZ], pc, double(s_uy[v][ro - RZ]), uyB,
                          double(s_mu[v][ro - RZ]), mc, M);
            dv += fd_flux(pc, s_ph[v][ro + 1], uzB, double(s_uz[v][ro + 1]), mc,
                          double(s_mu[v][ro + 1]), M)
                - fd_flux(s_ph[v][ro - 1], pc, double(s_uz[v][ro - 1]), uzB,
                          double(s_mu[v][ro - 1]), mc, M);
            __builtin_nontemporal_store(pc - dv, &dphi[U * plane + yg * p.nz + zg]);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            pxA[a] = pxB[a];
            pxB[a] = pxP[a];
        }
        rpA = rpB;
        rpB = rpP;
        phA = phB; muA = muB; uxA = uxB;
        phB = phC; muB = muC; uxB = uxC; uyB = uyC; uzB = uzC;
    }
    if (partials) block_partials<5, kFdFused>(acc, partials);
}

// Dense FP64 moments and block partials of [rho, phi, jx, jy, jz]
// (grid-stride); u = j/rho, or with FORCE (j + F/2)/rho and sums of j + F/2.
template <typename T, bool DEV, bool FORCE>
__global__ __launch_bounds__(kBlock) void k_fd_moments(KParams p, const T* __restrict__ F,
                                                       const double* __restrict__ phi,
                                                       double* __restrict__ rho_out,
                                                       double* __restrict__ u_out,
                                                       double* __restrict__ phi_out,
                                                       double* __restrict__ partials)
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = xcd_block() * kBlock + threadIdx.x; s < p.nsites; s += gridDim.x * kBlock) {
        const Geo q = geo_of(p, s);
        double b = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const double v = double(F[dist_pull(p, q, i)]);
            b += v;
            jx += CX[i] * v;
            jy += CY[i] * v;
            jz += CZ[i] * v;
        }
        const double rho = DEV ? p.rho0 + b : b;
        const double ph = phi[s];
        if (FORCE) {
            double F[3];
            force_from_phi(p, q, phi, F);
            jx += 0.5 * F[0];
            jy += 0.5 * F[1];
            jz += 0.5 * F[2];
        }
        if (rho_out) rho_out[s] = rho;
        if (u_out) {
            u_out[s] = jx / rho;
            u_out[p.nsites + s] = jy / rho;
            u_out[2LL * p.nsites + s] = jz / rho;
        }
        if (phi_out) phi_out[s] = ph;
        acc[0] += rho;
        acc[1] += ph;
        acc[2] += jx;
        acc[3] += jy;
        acc[4] += jz;
    }
    block_partials<5>(acc, partials);
}

template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_fd_export(KParams p, const T* __restrict__ F,
                                                      double* __restrict__ f)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
#pragma unroll
    for (int i = 0; i < NV; i++)
        f[(long long)i * p.nsites + s] = double(F[dist_pull(p, q, i)]) + (DEV ? weight(i) * p.rho0 : 0.0);
}

// The stored value of direction i at y is the post-propagation value at y + c_i.
template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_fd_import(KParams p, T* __restrict__ F,
                                                      const double* __restrict__ f)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const long long n = push_site(p, q, i) + (long long)i * p.nsites;
        F[dist_own(p, q, i)] = T(f[n] - (DEV ? weight(i) * p.rho0 : 0.0));
    }
}

// ---------------------------------------------------------------------------
// Reverse mode of one step (stress coupling).  The adjoint level keeps the
// layout of the LB scheme's: lf[19] = dL/df_i(x) of the pulled populations,
// lp = dL/dphi(x) (component 2*19); the g components are not used.
//
// k_fd_adj_prep stores rho and u of level t (fields rho, u_x, u_y, u_z of
// the storage type: u is formed in that type, with the forward's own
// expressions, so the upwind choices below are the forward's): u = j/rho,
// or with the force coupling u = (j + F/2)/rho, F = -div Pi of phi; then F
// itself (in the storage type, as the forward uses it) goes to the three
// scratch fields that the local kernel reads at the same site and then
// overwrites with dL/dF.
template <typename T, bool DEV, bool FORCE>
__global__ __launch_bounds__(kBlock) void k_fd_adj_prep(KParams p, const T* __restrict__ F,
                                                        const double* __restrict__ phi,
                                                        T* __restrict__ work, T* __restrict__ sc)
{
    const int s = xcd_block() * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    T f[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) f[i] = F[dist_pull(p, q, i)];
    const Moments<T> m = moments_of<T, DEV>(p, f);
    const T ri = T(1) / m.rho;
    T jx = m.jx, jy = m.jy, jz = m.jz;
    if (FORCE) {
        double Fd[3];
        force_from_phi(p, q, phi, Fd);
        const T Ft[3] = {T(Fd[0]), T(Fd[1]), T(Fd[2])};
        jx = m.jx + T(0.5) * Ft[0];
        jy = m.jy + T(0.5) * Ft[1];
        jz = m.jz + T(0.5) * Ft[2];
        sc[5 * size_t(p.stride) + s] = Ft[0];
        sc[6 * size_t(p.stride) + s] = Ft[1];
        sc[7 * size_t(p.stride) + s] = Ft[2];
    }
    work[s] = m.rho;
    work[p.stride + s] = jx * ri;
    work[2 * p.stride + s] = jy * ri;
    work[3 * p.stride + s] = jz * ri;
}

// Transposed step at x.  With lambda' the later level:
//   flux update: dL/dJ_a(x + e_a/2) = lp'(x + e_a) - lp'(x) =: lJ_a(x), so
//     lambda_mu(x) = M sum_a [lJ_a(x) - lJ_a(x - e_a)],
//     lambda_u_a(x) = [lJ_a(x) phi_up(x + e_a/2) + lJ_a(x - e_a) phi_up(x - e_a/2)] / 2,
//     and phi at the upwind site of each face takes u_f lJ;
//   u = j/rho: lambda_f,i += (c_i - u) . lambda_u / rho;
//   mu = A phi + B phi^3 - kappa lap: lambda_mu feeds the direct phi
//     cotangent (A + 3B phi^2), the Laplacian's (-kappa) and d/d(A, B, kappa);
//   the f collision: the LB scheme's transposed Jacobian without its g part
//     (lambda* gathered from x + c_i, weighted moments S0, S1, S2).
// Writes lf of the earlier level, the stencil cotangents a, b_x, b_y, b_z, c
// (lp = a - sum_a D_a b_a + lap c follows in k_adj_stencil) and block
// partials of d/d(A, B, kappa).  One resident round of workgroups, each
// thread looping over its sites.
// FORCE: u = (j + F/2)/rho and the forcing collision of f (Pi is not in
// f^eq): the flux's lambda_u joins the collision's, the total goes to j,
// rho and F as in the LB scheme's force adjoint (lb_adjoint.hip), and dL/dF
// is written after the five cotangents for k_adj_force_pi.
template <typename T, bool FORCE>
__global__ __launch_bounds__(kBlock) void k_fd_adj_local(KParams p, const double* __restrict__ phi,
                                                         const T* __restrict__ work,
                                                         const T* __restrict__ an,
                                                         T* __restrict__ ap, T* __restrict__ sc,
                                                         double* __restrict__ partials)
{
    double dth[3] = {0.0, 0.0, 0.0};
    const unsigned S = p.stride;
    const T* __restrict__ lpn = an + size_t(2 * NV) * S;
    const T* __restrict__ rhof = work;
    const T* __restrict__ uf[3] = {work + S, work + 2 * size_t(S), work + 3 * size_t(S)};
    const T A = T(p.A), B = T(p.B), kap = T(p.kappa), M = T(p.mobility);
    const T omf = T(p.omega_f), cf = T(1) - omf;
    const T h = T(4.5), third = T(1.0 / 3.0);
    for (XcdSweep w = xcd_sweep(p.nsites, kBlock); w.s < w.end; w.s += w.stride) {
        const int s = w.s;
        const Geo q = geo_of(p, s);
        T lf[NV];
#pragma unroll
        for (int i = 0; i < NV; i++)
            lf[i] = __builtin_nontemporal_load(&an[i * S + push_site(p, q, i)]);
        const int nb[3][2] = {{site_of(p, q.xp, q.y, q.z), site_of(p, q.xm, q.y, q.z)},
                              {site_of(p, q.x, q.yp, q.z), site_of(p, q.x, q.ym, q.z)},
                              {site_of(p, q.x, q.y, q.zp), site_of(p, q.x, q.y, q.zm)}};
        const double pc = phi[s];
        double pn[3][2];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            pn[a][0] = phi[nb[a][0]];
            pn[a][1] = phi[nb[a][1]];
        }
        const Stencil st = stencil(pc, pn[0][0], pn[0][1], pn[1][0], pn[1][1], pn[2][0], pn[2][1]);

        // flux update, transposed (upwind choices in FP64, as the forward)
        const T lc = lpn[s];
        T lmu = T(0), adv = T(0), lu[3], u[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const double uc = double(uf[a][s]);
            const double ufp = 0.5 * (uc + double(uf[a][nb[a][0]]));  // face x + e_a/2
            const double ufm = 0.5 * (double(uf[a][nb[a][1]]) + uc);  // face x - e_a/2
            const T ljp = lpn[nb[a][0]] - lc, ljm = lc - lpn[nb[a][1]];
            const T upp = T(ufp > 0.0 ? pc : pn[a][0]);
            const T upm = T(ufm > 0.0 ? pn[a][1] : pc);
            lmu += ljp - ljm;
            lu[a] = T(0.5) * (ljp * upp + ljm * upm);
            if (ufp > 0.0) adv += T(ufp) * ljp;
            if (!(ufm > 0.0)) adv += T(ufm) * ljm;
            u[a] = T(uc);
        }
        lmu *= M;

        if (FORCE) {
            // forcing collision of f, transposed (full second moment M2);
            // F of this site from the pre-pass, in the slots dL/dF replaces
            const T Fx = sc[5 * S + s], Fy = sc[6 * S + s], Fz = sc[7 * S + s];
            const T ux = u[0], uy = u[1], uz = u[2];
            const T rho = rhof[s], ri = T(1) / rho;
            T m0 = 0, m1x = 0, m1y = 0, m1z = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0,
              myz = 0;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const T wl = T(weight(i)) * lf[i];
                m0 += wl;
                if (CX[i]) { m1x += CX[i] * wl; mxx += wl; }
                if (CY[i]) { m1y += CY[i] * wl; myy += wl; }
                if (CZ[i]) { m1z += CZ[i] * wl; mzz += wl; }
                if (CX[i] * CY[i]) mxy += CX[i] * CY[i] * wl;
                if (CX[i] * CZ[i]) mxz += CX[i] * CZ[i] * wl;
                if (CY[i] * CZ[i]) myz += CY[i] * CZ[i] * wl;
            }
            const T m2ux = mxx * ux + mxy * uy + mxz * uz;
            const T m2uy = mxy * ux + myy * uy + myz * uz;
            const T m2uz = mxz * ux + myz * uy + mzz * uz;
            const T m2Fx = mxx * Fx + mxy * Fy + mxz * Fz;
            const T m2Fy = mxy * Fx + myy * Fy + myz * Fz;
            const T m2Fz = mxz * Fx + myz * Fy + mzz * Fz;
            const T uu = ux * ux + uy * uy + uz * uz;
            const T pref = T(1) - T(0.5) * omf, orho = omf * rho;
            const T lux = lu[0] + orho * (T(3) * m1x + T(9) * m2ux - T(3) * ux * m0)
                        + pref * (T(9) * m2Fx - T(3) * Fx * m0);
            const T luy = lu[1] + orho * (T(3) * m1y + T(9) * m2uy - T(3) * uy * m0)
                        + pref * (T(9) * m2Fy - T(3) * Fy * m0);
            const T luz = lu[2] + orho * (T(3) * m1z + T(9) * m2uz - T(3) * uz * m0)
                        + pref * (T(9) * m2Fz - T(3) * Fz * m0);
            const T arho = omf * (m0 + T(3) * (m1x * ux + m1y * uy + m1z * uz)
                                  + h * (m2ux * ux + m2uy * uy + m2uz * uz) - T(1.5) * uu * m0)
                         - (lux * ux + luy * uy + luz * uz) * ri;
            const T ajx = lux * ri, ajy = luy * ri, ajz = luz * ri;
            const T hr = T(0.5) * ri;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                T v = cf * lf[i] + arho;
                if (CX[i]) v += CX[i] * ajx;
                if (CY[i]) v += CY[i] * ajy;
                if (CZ[i]) v += CZ[i] * ajz;
                __builtin_nontemporal_store(v, &ap[i * S + s]);
            }
            const T phc = T(pc);
            sc[0 * S + s] = lc + (A + T(3) * B * phc * phc) * lmu + adv;
            sc[1 * S + s] = T(0);
            sc[2 * S + s] = T(0);
            sc[3 * S + s] = T(0);
            sc[4 * S + s] = -kap * lmu;
            sc[5 * S + s] = pref * (T(3) * m1x - T(3) * ux * m0 + T(9) * m2ux) + hr * lux;
            sc[6 * S + s] = pref * (T(3) * m1y - T(3) * uy * m0 + T(9) * m2uy) + hr * luy;
            sc[7 * S + s] = pref * (T(3) * m1z - T(3) * uz * m0 + T(9) * m2uz) + hr * luz;
            const double dlm = double(lmu), dph = pc;
            dth[0] += dph * dlm;
            dth[1] += dph * dph * dph * dlm;
            dth[2] += -st.lap * dlm;
            continue;
        }

        // collision of f, transposed
        T s0 = 0, s1x = 0, s1y = 0, s1z = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const T wl = T(weight(i)) * omf * lf[i];
            s0 += wl;
            if (CX[i]) { s1x += CX[i] * wl; sxx += wl; }
            if (CY[i]) { s1y += CY[i] * wl; syy += wl; }
            if (CZ[i]) { s1z += CZ[i] * wl; szz += wl; }
            if (CX[i] * CY[i]) sxy += CX[i] * CY[i] * wl;
            if (CX[i] * CZ[i]) sxz += CX[i] * CZ[i] * wl;
            if (CY[i] * CZ[i]) syz += CY[i] * CZ[i] * wl;
        }
        sxx -= third * s0; syy -= third * s0; szz -= third * s0;
        const T ux = u[0], uy = u[1], uz = u[2];
        const T ri = T(1) / rhof[s];
        const T trs = sxx + syy + szz;
        const T s2ux = sxx * ux + sxy * uy + sxz * uz;
        const T s2uy = sxy * ux + syy * uy + syz * uz;
        const T s2uz = sxz * ux + syz * uy + szz * uz;
        const T s2uu = s2ux * ux + s2uy * uy + s2uz * uz;
        const T gx = T(st.gx), gy = T(st.gy), gz = T(st.gz), lap = T(st.lap), phc = T(pc);
        const T s2gx = sxx * gx + sxy * gy + sxz * gz;
        const T s2gy = sxy * gx + syy * gy + syz * gz;
        const T s2gz = sxz * gx + syz * gy + szz * gz;
        const T gsg = s2gx * gx + s2gy * gy + s2gz * gz;

        const T arho = s0 - h * s2uu - (lu[0] * ux + lu[1] * uy + lu[2] * uz) * ri;
        const T ajx = T(3) * s1x + T(9) * s2ux + lu[0] * ri;
        const T ajy = T(3) * s1y + T(9) * s2uy + lu[1] * ri;
        const T ajz = T(3) * s1z + T(9) * s2uz + lu[2] * ri;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            T v = cf * lf[i] + arho;
            if (CX[i]) v += CX[i] * ajx;
            if (CY[i]) v += CY[i] * ajy;
            if (CZ[i]) v += CZ[i] * ajz;
            __builtin_nontemporal_store(v, &ap[i * S + s]);
        }
        const T phi2 = phc * phc;
        const T a_dir = lc + (A + T(3) * B * phi2) * lmu + adv
                      + h * trs * (A * phc + T(3) * B * phi2 * phc - kap * lap);
        const T hk = h * kap;
        __builtin_nontemporal_store(a_dir, &sc[0 * S + s]);
        __builtin_nontemporal_store(hk * (T(2) * s2gx - trs * gx), &sc[1 * S + s]);
        __builtin_nontemporal_store(hk * (T(2) * s2gy - trs * gy), &sc[2 * S + s]);
        __builtin_nontemporal_store(hk * (T(2) * s2gz - trs * gz), &sc[3 * S + s]);
        __builtin_nontemporal_store(-kap * lmu - hk * phc * trs, &sc[4 * S + s]);
        const double g2 = st.gx * st.gx + st.gy * st.gy + st.gz * st.gz;
        const double dtrs = double(trs), dlm = double(lmu), dph = pc;
        dth[0] += dph * dlm + 4.5 * dtrs * 0.5 * dph * dph;
        dth[1] += dph * dph * dph * dlm + 4.5 * dtrs * 0.75 * dph * dph * dph * dph;
        dth[2] += -st.lap * dlm + 4.5 * (dtrs * (-dph * st.lap - 0.5 * g2) + double(gsg));
    }
    block_partials<3>(dth, partials);
}

int fd_grid(const KParams& p) { return (p.nsites + kBlock - 1) / kBlock; }

// Update-pass geometry: (y, z) tiles times x segments, about 2048
// workgroups (8 waves per SIMD on 256 CUs) when the lattice allows.
struct FdTiles {
    int ntz, ntiles, sx, nseg;
};

FdTiles fd_tiles(const KParams& p)
{
    FdTiles t;
    t.ntz = (p.nz + kFdTZ - 1) / kFdTZ;
    t.ntiles = ((p.ny + kFdTY - 1) / kFdTY) * t.ntz;
    int nseg = (2048 + t.ntiles - 1) / t.ntiles;
    nseg = nseg < 1 ? 1 : (nseg > p.nx ? p.nx : nseg);
    t.sx = (p.nx + nseg - 1) / nseg;
    t.nseg = (p.nx + t.sx - 1) / t.sx;
    return t;
}

// Geometry of k_fd_force_fused: 8 x 64 tiles times x segments; a workgroup
// holds a CU, so they run in rounds of 256, and a segment of s planes costs
// s + 4 iterations (the pipeline's fill and drain): the segment count
// minimises rounds * (s + 4) unless the caller fixed the segment length.
constexpr int kFfCUs = 256;

TileCfg ff_tiles(const KParams& p, int seg_req)
{
    TileCfg tc;
    tc.tz = FfTile::TZ;
    tc.nty = (p.ny + FfTile::TY - 1) / FfTile::TY;
    tc.ntz = (p.nz + FfTile::TZ - 1) / FfTile::TZ;
    tc.ntiles = tc.nty * tc.ntz;
    tc.seg_req = seg_req;
    int sx = seg_req;
    if (sx <= 0) {
        long long best = -1;
        for (int nseg = 1; nseg <= p.nx; nseg++) {
            const int sl = (p.nx + nseg - 1) / nseg;
            const long long nb = (long long)tc.ntiles * ((p.nx + sl - 1) / sl);
            const long long cost = ((nb + kFfCUs - 1) / kFfCUs) * (sl + 4);
            if (best < 0 || cost < best) {
                best = cost;
                sx = sl;
            }
        }
    }
    if (sx > p.nx) sx = p.nx;
    tc.sx = sx;
    tc.nseg = (p.nx + sx - 1) / sx;
    return tc;
}

int fd_reduction_grid(const KParams& p)
{
    const int g = fd_grid(p);
    return g < kMaxPartialBlocks ? g : kMaxPartialBlocks;
}

// FP64 mode <double, false>, FP32 mode <float, true>.
#define LB_FD_DISPATCH(fp32, CALL)      \
    do {                                \
        if (fp32) {                     \
            using T = float;            \
            constexpr bool DEV = true;  \
            (void)DEV;                  \
            CALL;                       \
        } else {                        \
            using T = double;           \
            constexpr bool DEV = false; \
            (void)DEV;                  \
            CALL;                       \
        }                               \
    } while (0)

}  // namespace

int fd_step_partial_blocks(const KParams& p, int segment_x)
{
    const TileCfg ft = ff_tiles(p, segment_x);
    const int g = fd_grid(p);
    return ft.ntiles * ft.nseg > g ? ft.ntiles * ft.nseg : g;
}

int fd_sums_blocks(const KParams& p, const TileCfg& tc, int variant)
{
    if (variant != 0) return fd_grid(p);
    if (p.force) {
        const TileCfg ft = ff_tiles(p, tc.seg_req);
        return ft.ntiles * ft.nseg;
    }
    return tc.ntiles * tc.nseg;
}

hipError_t launch_fd_init(const KParams& p, bool fp32, void* state, const double* phi0,
                          hipStream_t s)
{
#define CALL                                                                          \
    {                                                                                 \
        FdLvl<T> l = fd_level<T>(state, p);                                           \
        k_fd_init<T, DEV><<<fd_grid(p), kBlock, 0, s>>>(p, l.F, l.phi, phi0);         \
    }
    LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_fd_step(const KParams& p, const TileCfg& tc, bool fp32, int variant,
                          const void* src, void* dst, double* work, double* partials,
                          double* sums_out, hipStream_t s)
{
    int nparts;
    if (variant == 0 && p.force) {
        // one marching pass: force, collision and flux update
        const TileCfg ft = ff_tiles(p, tc.seg_req);
        nparts = ft.ntiles * ft.nseg;
#define CALL                                                                                  \
    {                                                                                         \
        FdLvl<T> a = fd_level<T>(const_cast<void*>(src), p);                                  \
        FdLvl<T> d = fd_level<T>(dst, p);                                                     \
        k_fd_force_fused<T, DEV><<<nparts, kFdFused, 0, s>>>(p, ft, a.F, a.phi, d.F, d.phi,    \
                                                             sums_out ? partials : nullptr);  \
    }
        LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    } else if (variant == 0) {
        nparts = tc.ntiles * tc.nseg;
#define CALL                                                                                  \
    {                                                                                         \
        FdLvl<T> a = fd_level<T>(const_cast<void*>(src), p);                                  \
        FdLvl<T> d = fd_level<T>(dst, p);                                                     \
        FdFused<T>::get(tc.tz)<<<nparts, kFdFused, 0, s>>>(p, tc, a.F, a.phi, d.F, d.phi,     \
                                                           sums_out ? partials : nullptr);    \
    }
        LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    } else {
        const FdTiles ft = fd_tiles(p);
        nparts = fd_grid(p);
#define CALL                                                                                  \
    {                                                                                         \
        FdLvl<T> a = fd_level<T>(const_cast<void*>(src), p);                                  \
        FdLvl<T> d = fd_level<T>(dst, p);                                                     \
        if (p.force) {                                                                        \
            using W = FdWork<T, true>;                                                        \
            W* w = reinterpret_cast<W*>(work);                                                \
            k_fd_collide<T, DEV, true><<<fd_grid(p), kBlock, 0, s>>>(p, a.F, a.phi, d.F, w,    \
                                                                     sums_out ? partials       \
                                                                              : nullptr);      \
            k_fd_update<W><<<ft.ntiles * ft.nseg, kBlock, 0, s>>>(p, ft.ntz, ft.ntiles, ft.sx, \
                                                                  a.phi, w, d.phi);           \
        } else {                                                                              \
            k_fd_collide<T, DEV, false><<<fd_grid(p), kBlock, 0, s>>>(p, a.F, a.phi, d.F, work,\
                                                                      sums_out ? partials      \
                                                                               : nullptr);     \
            k_fd_update<double><<<ft.ntiles * ft.nseg, kBlock, 0, s>>>(p, ft.ntz, ft.ntiles,   \
                                                                       ft.sx, a.phi, work,     \
                                                                       d.phi);                 \
        }                                                                                     \
    }
        LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    }
    if (sums_out) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_sums_final(partials, nparts, 5, sums_out, false, s);
    }
    return hipGetLastError();
}

hipError_t launch_fd_adj_step(const KParams& p, bool fp32, const void* state, double* work,
                              const void* adj_next, void* adj_prev, void* adj_scratch,
                              double* partials, double* dtheta, hipStream_t s)
{
    // rho and u go to `work` in the storage type (FP32 mode: half its
    // space); one resident round of workgroups (4 per CU), as the LB
    // scheme's local adjoint kernel
    constexpr int kAdjBlocks = 1024;
    const int nb = fd_reduction_grid(p) < kAdjBlocks ? fd_reduction_grid(p) : kAdjBlocks;
    // force coupling: dL/dF through Pi (launch_adj_force_pi), whose
    // partials follow the local kernel's
    double* partials2 = p.force ? partials + 3 * kAdjBlocks : nullptr;
    void* st = const_cast<void*>(state);
    const double* phi = fp32 ? fd_level<float>(st, p).phi : fd_level<double>(st, p).phi;
#define CALL                                                                                  \
    {                                                                                         \
        FdLvl<T> a = fd_level<T>(const_cast<void*>(state), p);                                \
        T* w = reinterpret_cast<T*>(work);                                                    \
        const T* an = static_cast<const T*>(adj_next);                                        \
        T* ap = static_cast<T*>(adj_prev);                                                    \
        T* sc = static_cast<T*>(adj_scratch);                                                 \
        if (p.force) {                                                                        \
            k_fd_adj_prep<T, DEV, true><<<fd_grid(p), kBlock, 0, s>>>(p, a.F, a.phi, w, sc);  \
            k_fd_adj_local<T, true><<<nb, kBlock, 0, s>>>(p, a.phi, w, an, ap, sc, partials); \
        } else {                                                                              \
            k_fd_adj_prep<T, DEV, false><<<fd_grid(p), kBlock, 0, s>>>(p, a.F, a.phi, w, sc); \
            k_fd_adj_local<T, false><<<nb, kBlock, 0, s>>>(p, a.phi, w, an, ap, sc, partials);\
        }                                                                                     \
    }
    LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p.force) {
        e = launch_adj_force_pi(p, fp32, phi, adj_scratch, partials2, nb, s);
        if (e != hipSuccess) return e;
    }
    return launch_adj_stencil(p, fp32, adj_scratch, adj_prev, partials, partials2, nb, dtheta, s);
}

hipError_t launch_fd_moments(const KParams& p, bool fp32, const void* state, double* rho,
                             double* u, double* phi, double* partials, int* nblocks_out,
                             hipStream_t s)
{
    const int nb = fd_reduction_grid(p);
    *nblocks_out = nb;
#define CALL                                                                                \
    {                                                                                       \
        FdLvl<T> a = fd_level<T>(const_cast<void*>(state), p);                              \
        if (p.force)                                                                        \
            k_fd_moments<T, DEV, true><<<nb, kBlock, 0, s>>>(p, a.F, a.phi, rho, u, phi,    \
                                                             partials);                     \
        else                                                                                \
            k_fd_moments<T, DEV, false><<<nb, kBlock, 0, s>>>(p, a.F, a.phi, rho, u, phi,   \
                                                              partials);                    \
    }
    LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_fd_export(const KParams& p, bool fp32, const void* state, double* f,
                            hipStream_t s)
{
#define CALL                                                                        \
    {                                                                               \
        FdLvl<T> a = fd_level<T>(const_cast<void*>(state), p);                      \
        k_fd_export<T, DEV><<<fd_grid(p), kBlock, 0, s>>>(p, a.F, f);               \
    }
    LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_fd_import(const KParams& p, bool fp32, void* state, const double* f,
                            hipStream_t s)
{
#define CALL                                                                        \
    {                                                                               \
        FdLvl<T> a = fd_level<T>(state, p);                                         \
        k_fd_import<T, DEV><<<fd_grid(p), kBlock, 0, s>>>(p, a.F, f);               \
    }
    LB_FD_DISPATCH(fp32, CALL);
#undef CALL
    return hipGetLastError();
}

}  // namespace lbk
