// Force coupling (LB_COUPLING_FORCE): F = -div Pi by central differences of
// the chemical stress at the six face neighbours (the paper's Ludwig model
// applies the stress's divergence as a body force, Sec. 2.1.1), with the
// half-force velocity and Guo's forcing term in collide_force().  Two forms
// with bit-identical results:
//
//   k_force_fused (LB_KERNEL_FUSED): the whole step in one pass, on the
//     single-pass LB kernel's tiling -- a TY x TZ tile of (y, z) columns
//     marching along x -- with phi of the tile plus two cells around it
//     summed from the pulled g into an LDS ring, Pi of plane P formed once
//     per site for the tile and its face ring and kept in LDS (the
//     components the y and z neighbours need) and in registers (the own
//     column's x row, for x +- 1), and the collision of plane P-1;
//   k_step_force (LB_KERNEL_TWO_PASS), after k_phi: one site per thread, Pi
//     formed at each face neighbour from the phi field (force_from_phi).
//
// No floating-point contraction in this translation unit (including the
// shared device functions it inlines): the compiler fuses multiply-adds
// differently in different kernels, and the two forms must round alike.
#pragma clang fp contract(off)

#include "lb_device.h"

namespace lbk {

using namespace dev;

namespace {

// The force-coupling collision and propagation, one site per thread; phi of
// the source level (all sites) comes from k_phi.
template <typename T, bool DEV, bool REF, bool G1>
__global__ __launch_bounds__(kBlock) void k_step_force(KParams p, const T* __restrict__ sF,
                                                       const T* __restrict__ sG,
                                                       const unsigned* __restrict__ sphic,
                                                       const double* __restrict__ phi,
                                                       T* __restrict__ dF, T* __restrict__ dG)
{
    const int s = xcd_block() * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    T f[NV], g[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        f[i] = sF[dist_pull(p, q, i)];
        g[i] = G1 ? T(0) : sG[dist_pull(p, q, i)];
    }
    const double c = phi[s];
    const double lap = (phi[site_of(p, q.xp, q.y, q.z)] + phi[site_of(p, q.xm, q.y, q.z)] - 2.0 * c)
                     + (phi[site_of(p, q.x, q.yp, q.z)] + phi[site_of(p, q.x, q.ym, q.z)] - 2.0 * c)
                     + (phi[site_of(p, q.x, q.y, q.zp)] + phi[site_of(p, q.x, q.y, q.zm)] - 2.0 * c);
    const double mu = p.A * c + p.B * c * c * c - p.kappa * lap;
    if (REF && !G1) {
        const double dphi = c - phic_value(sphic[phic_site(p, q.x, q.y, q.z)]);
#pragma unroll
        for (int i = 0; i < NV; i++) g[i] = pre_collision_dev(i, g[i], dphi);
    }
    double F[3];
    force_from_phi(p, q, phi, F);
    collide_force<T, DEV, REF, G1>(p, f, g, c, mu, F);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        dF[dist_own(p, q, i)] = f[i];
        dG[dist_own(p, q, i)] = REF ? to_dest_ref(i, g[i], c, phi[push_site(p, q, i)]) : g[i];
    }
}

constexpr int kForceFused = 512;
constexpr int kPhiSlots = 8;  // phi planes P-2 .. P+1 are read while P+2 is written

template <int TZ>
struct ForceTile {
    static constexpr int TY = kForceFused / TZ;
    static constexpr int BY = TY + 4, BZ = TZ + 4;  // phi box: two cells around the tile
    static constexpr int RY = TY + 2, RZ = TZ + 2;  // tile and its face ring
    static constexpr int NBOX = BY * BZ;
    static constexpr int NRING = 2 * (TY + TZ);
    static constexpr int BOXPT = (NBOX + kForceFused - 1) / kForceFused;
};

__device__ __forceinline__ int wrap_any(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// For plane P: (a) phi(P+1) into the LDS ring (its g pulled one plane
// earlier), the pulls of the own site of plane P-1 and of the box of plane
// P+2; (c) Pi of plane P at the own site and, for the first 2 (TY + TZ)
// threads, at a face-ring cell; (e) the forcing collision of plane P-1,
// whose F uses Pi of planes P-2 and P (own column, registers) and of plane
// P-1 at the four in-plane neighbours (LDS, written one plane earlier).
// Planes x0-1 and x1 only supply the own column's Pi.  Tile cells beyond a
// ragged lattice edge stand for the periodic images there: they form Pi but
// store nothing.  phi of the box is pulled and summed as k_phi sums it (so
// the values are bit-identical); the own cell's phi goes to the next
// level's phi_c (FP32 mode) and to the caller's phi field `phi_out` if that
// is not null.  Each population is read and written once per step.  G1
// (omega_g = 1): the collision takes g* = g^eq and loads no g.  SUMS: block partials
// of [rho, phi, j + F/2] of the state stepped from go to `partials`, as
// k_moments sums them with the force (a separate instantiation: the sums'
// registers would otherwise make the plain step spill).
template <typename T, bool DEV, bool REF, int TZ, bool G1, bool SUMS>
__global__ __launch_bounds__(kForceFused) void k_force_fused(KParams p, TileCfg tc,
                                                             const T* __restrict__ sF,
                                                             const T* __restrict__ sG,
                                                             const unsigned* __restrict__ sphic,
                                                             unsigned* __restrict__ dphic,
                                                             double* __restrict__ phi_out,
                                                             T* __restrict__ dF, T* __restrict__ dG,
                                                             double* __restrict__ partials)
{
    using G = ForceTile<TZ>;
    constexpr int TY = G::TY, BZ = G::BZ, RZ = G::RZ, NR = G::RY * G::RZ;
    __shared__ double s_phi[kPhiSlots][G::NBOX];
    __shared__ double s_piy[2][3][NR];  // Pi_xy, Pi_yy, Pi_yz: read by the y neighbours
    __shared__ double s_piz[2][3][NR];  // Pi_xz, Pi_yz, Pi_zz: read by the z neighbours

    const int t = threadIdx.x;
    const int b = xcd_block();
    const int seg = b / tc.ntiles, tile = b - seg * tc.ntiles;
    const int y0 = (tile / tc.ntz) * TY, z0 = (tile % tc.ntz) * TZ;
    const int x0 = seg * tc.sx, x1 = min(p.nx, x0 + tc.sx);
    const int plane = p.ny * p.nz;

    const int ly = t / TZ, lz = t % TZ;
    const int yg = wrap_any(y0 + ly, p.ny), zg = wrap_any(z0 + lz, p.nz);
    const bool valid = y0 + ly < p.ny && z0 + lz < p.nz;
    const int bo = (ly + 2) * BZ + (lz + 2);
    const int ro = (ly + 1) * RZ + (lz + 1);
    // box cells of this thread: the partly filled last slot goes to the last
    // threads, so that its extra work lands on the waves without face-ring
    // cells (the first 2 (TY + TZ) threads); 3% faster in FP64
    int boff[G::BOXPT], bcy[G::BOXPT], bcz[G::BOXPT], bcell[G::BOXPT];
#pragma unroll
    for (int k = 0; k < G::BOXPT; k++) {
        const int nk = G::NBOX - k * kForceFused < kForceFused ? G::NBOX - k * kForceFused : kForceFused;
        const int c = t >= kForceFused - nk ? k * kForceFused + t - (kForceFused - nk) : G::NBOX;
        bcell[k] = c;
        bcy[k] = c < G::NBOX ? wrap_any(y0 + c / BZ - 2, p.ny) : -1;
        bcz[k] = c < G::NBOX ? wrap_any(z0 + c % BZ - 2, p.nz) : -1;
        boff[k] = c < G::NBOX ? bcy[k] * p.nz + bcz[k] : -1;
    }
    const bool ring = t < G::NRING;
    int rly, rlz;
    if (t < TZ) { rly = -1; rlz = t; }
    else if (t < 2 * TZ) { rly = TY; rlz = t - TZ; }
    else if (t < 2 * TZ + TY) { rly = t - 2 * TZ; rlz = -1; }
    else { rly = t - 2 * TZ - TY; rlz = TZ; }
    const bool ring_y = rly < 0 || rly >= TY;  // a row of the ring, else a column
    const int rbo = (rly + 2) * BZ + (rlz + 2);
    const int rro = (rly + 1) * RZ + (rlz + 1);

    // the box of plane xp in flight: with FP32 storage the pulled g and phi_c
    // word of each box cell, summed when stored; FP64 storage sums its pulls
    // at once (carrying them would take 76 more VGPRs)
    constexpr bool CARRY = std::is_same<T, float>::value;
    struct BoxLoads {
        double v[CARRY ? 1 : G::BOXPT];
        unsigned w[CARRY ? G::BOXPT : 1];
        T g[CARRY ? G::BOXPT : 1][NV];
    };
    // phi_at's sum: the pulled values in index order, then phi_c
    auto sum_g = [&](const T (&g)[NV], double pc) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) acc += double(g[i]);
        return REF ? pc + acc : acc;
    };
    auto load_box = [&](int xp, BoxLoads& b) {
        const int xw = wrap_any(xp, p.nx);
#pragma unroll
        for (int k = 0; k < G::BOXPT; k++) {
            if (boff[k] < 0) continue;
            const Geo q = geo_xyz(p, xw, bcy[k], bcz[k]);
            T g[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) g[i] = sG[dist_pull(p, q, i)];
            if constexpr (CARRY) {
#pragma unroll
                for (int i = 0; i < NV; i++) b.g[k][i] = g[i];
                b.w[k] = sphic[xw * plane + boff[k]];
            } else {
                b.v[k] = sum_g(g, 0.0);
            }
        }
    };
    auto store_box = [&](int xp, const BoxLoads& b) {
        double* __restrict__ dst = s_phi[xp & (kPhiSlots - 1)];
#pragma unroll
        for (int k = 0; k < G::BOXPT; k++) {
            if (boff[k] < 0) continue;
            if constexpr (CARRY)
                dst[bcell[k]] = sum_g(b.g[k], phic_value(b.w[k]));
            else
                dst[bcell[k]] = b.v[k];
        }
    };
    BoxLoads pre;
    load_box(x0 - 2, pre);
    store_box(x0 - 2, pre);
    load_box(x0 - 1, pre);
    store_box(x0 - 1, pre);
    load_box(x0, pre);

    // own column's Pi x row (xx, xy, xz) at planes X-1 and X, X = P-1
    double pxA[3] = {0.0, 0.0, 0.0}, pxB[3] = {0.0, 0.0, 0.0};
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int P = x0 - 1; P <= x1; P++) {
        const int X = P - 1;
        const bool collide_x = X >= x0 && valid;
        // (a)
        store_box(P + 1, pre);
        T f[NV], g[NV];
        unsigned pc_src = 0;
        const Geo q = geo_xyz(p, wrap_any(X, p.nx), yg, zg);
        if (collide_x) {
#pragma unroll
            for (int i = 0; i < NV; i++) {
                f[i] = sF[dist_pull(p, q, i)];
                g[i] = G1 ? T(0) : sG[dist_pull(p, q, i)];
            }
            if (REF && !G1) pc_src = sphic[X * plane + yg * p.nz + zg];
        }
        load_box(P + 2, pre);
        lds_barrier();
        const double* __restrict__ fm = s_phi[(P - 1) & (kPhiSlots - 1)];
        const double* __restrict__ fc = s_phi[P & (kPhiSlots - 1)];
        const double* __restrict__ fp = s_phi[(P + 1) & (kPhiSlots - 1)];
        const int w = P & 1;

        // (c) Pi of plane P
        double pxP[3];
        {
            const Stencil st = stencil(fc[bo], fp[bo], fm[bo], fc[bo + BZ], fc[bo - BZ], fc[bo + 1],
                                       fc[bo - 1]);
            double mu, tt[6];
            chem_stress(p, st, &mu, tt);
            pxP[0] = tt[0];
            pxP[1] = tt[1];
            pxP[2] = tt[2];
            s_piy[w][0][ro] = tt[1];
            s_piy[w][1][ro] = tt[3];
            s_piy[w][2][ro] = tt[4];
            s_piz[w][0][ro] = tt[2];
            s_piz[w][1][ro] = tt[4];
            s_piz[w][2][ro] = tt[5];
        }
        if (ring && P >= x0 && P < x1) {
            const Stencil st = stencil(fc[rbo], fp[rbo], fm[rbo], fc[rbo + BZ], fc[rbo - BZ],
                                       fc[rbo + 1], fc[rbo - 1]);
            double mu, tt[6];
            chem_stress(p, st, &mu, tt);
            if (ring_y) {
                s_piy[w][0][rro] = tt[1];
                s_piy[w][1][rro] = tt[3];
                s_piy[w][2][rro] = tt[4];
            } else {
                s_piz[w][0][rro] = tt[2];
                s_piz[w][1][rro] = tt[4];
                s_piz[w][2][rro] = tt[5];
            }
        }

        // (e) the collision of plane X = P-1
        if (collide_x) {
            const int v = X & 1;
            const double* __restrict__ xm = s_phi[(X - 1) & (kPhiSlots - 1)];
            const double* __restrict__ xc = s_phi[X & (kPhiSlots - 1)];
            const double* __restrict__ xp = s_phi[(X + 1) & (kPhiSlots - 1)];
            const double c = xc[bo];
            const double lap = (xp[bo] + xm[bo] - 2.0 * c) + (xc[bo + BZ] + xc[bo - BZ] - 2.0 * c)
                             + (xc[bo + 1] + xc[bo - 1] - 2.0 * c);
            const double mu = p.A * c + p.B * c * c * c - p.kappa * lap;
            if (REF && !G1) {
                const double dphi = c - phic_value(pc_src);
#pragma unroll
                for (int i = 0; i < NV; i++) g[i] = pre_collision_dev(i, g[i], dphi);
            }
            // F_a = -sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)] / 2, b = x, y, z in order
            double div[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 0; a < 3; a++) div[a] += 0.5 * (pxP[a] - pxA[a]);
#pragma unroll
            for (int a = 0; a < 3; a++) div[a] += 0.5 * (s_piy[v][a][ro + RZ] - s_piy[v][a][ro - RZ]);
#pragma unroll
            for (int a = 0; a < 3; a++) div[a] += 0.5 * (s_piz[v][a][ro + 1] - s_piz[v][a][ro - 1]);
            double F[3];
#pragma unroll
            for (int a = 0; a < 3; a++) F[a] = -div[a];
            if (SUMS) {
                double b = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
                for (int i = 0; i < NV; i++) b += double(f[i]);
#pragma unroll
                for (int i = 0; i < NV; i++) {
                    jx += CX[i] * double(f[i]);
                    jy += CY[i] * double(f[i]);
                    jz += CZ[i] * double(f[i]);
                }
                acc[0] += DEV ? p.rho0 + b : b;
                acc[1] += c;
                acc[2] += jx + 0.5 * F[0];
                acc[3] += jy + 0.5 * F[1];
                acc[4] += jz + 0.5 * F[2];
            }
            collide_force<T, DEV, REF, G1>(p, f, g, c, mu, F);
            if (REF) dphic[X * plane + yg * p.nz + zg] = phic_word(c);
            if (phi_out) phi_out[X * plane + yg * p.nz + zg] = c;
#pragma unroll
            for (int i = 0; i < NV; i++) {
                __builtin_nontemporal_store(f[i], &dF[dist_own(p, q, i)]);
                T gv = g[i];
                if (REF) {
                    const double* __restrict__ pl = CX[i] > 0 ? xp : (CX[i] < 0 ? xm : xc);
                    gv = to_dest_ref(i, g[i], c, pl[bo + CY[i] * BZ + CZ[i]]);
                }
                __builtin_nontemporal_store(gv, &dG[dist_own(p, q, i)]);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            pxA[a] = pxB[a];
            pxB[a] = pxP[a];
        }
    }
    if (SUMS) block_partials<5, kForceFused>(acc, partials);
}

int force_grid(const KParams& p) { return (p.nsites + kBlock - 1) / kBlock; }

// Tiling of the single pass: 8 x 64 tiles, whose box of phi (two cells
// around the tile, 12 x 68) is 1.6 cells per thread, against 2.1 for
// 4 x 128 tiles (whose carried pulls spill unless tau_g = 1, and then ran
// only 0.4% faster); x segments as tile_config chooses them (fewest rounds
// of 256 workgroups times the segment length plus its two warm-up planes).
TileCfg force_tiles(const KParams& p, int seg_req)
{
    TileCfg tc;
    tc.tz = 64;
    tc.nty = (p.ny + kForceFused / 64 - 1) / (kForceFused / 64);
    tc.ntz = (p.nz + 63) / 64;
    tc.ntiles = tc.nty * tc.ntz;
    tc.seg_req = seg_req;
    int sx = seg_req;
    if (sx <= 0) {
        long long best = -1;
        for (int nseg = 1; nseg <= p.nx; nseg++) {
            const int sl = (p.nx + nseg - 1) / nseg;
            const long long nb = (long long)tc.ntiles * ((p.nx + sl - 1) / sl);
            const long long cost = ((nb + 255) / 256) * (sl + 2);
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

}  // namespace

int force_sums_blocks(const KParams& p, int seg_req)
{
    const TileCfg ft = force_tiles(p, seg_req);
    return ft.ntiles * ft.nseg;
}

hipError_t launch_force_collide(const KParams& p, const TileCfg& tc, bool fp32, int variant,
                                const void* src, void* dst, double* phi, double* partials,
                                hipStream_t s)
{
    const TileCfg ft = force_tiles(p, tc.seg_req);
    const int nft = ft.ntiles * ft.nseg;
    // omega_g = 1: g* = g^eq, so the collision loads no g (the single pass
    // still pulls g for phi)
    const bool g1 = p.omega_g == 1.0;
    if (fp32) {
        Lvl<float> a = level<float>(const_cast<void*>(src), p, true);
        Lvl<float> d = level<float>(dst, p, true);
        if (variant == 0) {
            auto k = g1 ? (partials ? k_force_fused<float, true, true, 64, true, true>
                                    : k_force_fused<float, true, true, 64, true, false>)
                        : (partials ? k_force_fused<float, true, true, 64, false, true>
                                    : k_force_fused<float, true, true, 64, false, false>);
            k<<<nft, kForceFused, 0, s>>>(p, ft, a.F, a.G, a.phic, d.phic, phi, d.F, d.G, partials);
        } else {
            auto k = g1 ? k_step_force<float, true, true, true> : k_step_force<float, true, true, false>;
            k<<<force_grid(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, phi, d.F, d.G);
        }
    } else {
        Lvl<double> a = level<double>(const_cast<void*>(src), p, false);
        Lvl<double> d = level<double>(dst, p, false);
        if (variant == 0) {
            auto k = g1 ? (partials ? k_force_fused<double, false, false, 64, true, true>
                                    : k_force_fused<double, false, false, 64, true, false>)
                        : (partials ? k_force_fused<double, false, false, 64, false, true>
                                    : k_force_fused<double, false, false, 64, false, false>);
            k<<<nft, kForceFused, 0, s>>>(p, ft, a.F, a.G, nullptr, nullptr, phi, d.F, d.G,
                                          partials);
        } else {
            auto k = g1 ? k_step_force<double, false, false, true>
                        : k_step_force<double, false, false, false>;
            k<<<force_grid(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, phi, d.F, d.G);
        }
    }
    return hipGetLastError();
}

}  // namespace lbk
