// Reverse-mode kernels: one adjoint timestep lambda_t = J(s_t)^T lambda_{t+1}
// of the D3Q19 binary-fluid step, hand-derived.
//
// One forward step is  s_{t+1} = P(C(s_t)), P the propagation (a permutation)
// and C the collision, which is local except through phi's stencil.  With
// Lambda = omega * lambda* (lambda* the cotangent of the post-collision
// populations) the collision's transposed Jacobian needs only the weighted
// moments of Lambda:
//   S0 = sum w L_f,  S1 = sum w L_f c,  S2 = sum w L_f (c c - I/3)   (f part)
//   T0, T1, T2 the same for L_g                                      (g part)
// because f_eq and g_eq are Hermite expansions in (rho, j, Pi) and
// (phi, u, mu).  Writing Phi = sum_i L_f,i f_eq,i + L_g,i g_eq,i:
//   dPhi/drho  = S0 - 9/2 S2:uu - 3 phi T1.u/rho - 9 phi T2:uu/rho
//   dPhi/dj    = 3 S1 + 9 S2.u + 3 phi T1/rho + 9 phi T2.u/rho
//   dPhi/dphi  = 9/2 trS2 (A phi + 3B phi^3 - kappa lap) + T0 + 3 T1.u
//                + 9/2 (Gamma (A + 3B phi^2) - 1/3) trT2 + 9/2 T2:uu
//   dPhi/d(d_a phi) = 9/2 kappa (2 (S2 grad)_a - trS2 d_a phi)
//   dPhi/d(lap)     = -9/2 kappa (phi trS2 + Gamma trT2)
//   dPhi/dA = 9/2 (trS2 phi^2/2 + Gamma phi trT2)
//   dPhi/dB = 9/2 (trS2 3 phi^4/4 + Gamma phi^3 trT2)
//   dPhi/dkappa = 9/2 (trS2 (-phi lap - |grad|^2/2) + grad.S2.grad - Gamma lap trT2)
// and then lambda_f,i = (1 - omega_f) lambda*_f,i + dPhi/drho + c_i . dPhi/dj,
// lambda_g,i = (1 - omega_g) lambda*_g,i + lambda_phi, where lambda_phi
// collects the phi cotangents through the transposed stencil
// (D_a^T = -D_a, lap^T = lap on the periodic lattice).
//
// An adjoint level stores 39 components of `stride` elements:
//   lf[19] = dL/df_i(x), lg[19] = the part of dL/dg_i(x) specific to i,
//   lp = dL/dphi(x), so that dL/dg_i(x) = lg_i(x) + lp(x).
// adj_scratch holds a (direct dPhi/dphi), b_x, b_y, b_z, c per site.
//
// With omega_g = 1 (tau_g = 1) the post-collision g is g^eq alone, so the
// previous level's lg = (1 - omega_g) lambda*_g is identically zero: the seed
// zeroes lg in both levels and the local kernels (G1) neither read nor write
// it, which takes 152 of the 412 bytes per site off the FP32 step (304 of
// 816 in FP64).
#include "lb_device.h"
#include "lb_sweep.h"

namespace lbk {

using namespace dev;

namespace {

// other (may be null): the other level, whose lg is zeroed too
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_seed(KParams p, T* __restrict__ adj,
                                                     T* __restrict__ other,
                                                     const double* __restrict__ dphi)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
#pragma unroll
    for (int i = 0; i < 2 * NV; i++) adj[i * p.stride + s] = T(0);
    adj[2 * NV * p.stride + s] = T(dphi[s]);
    if (other)
#pragma unroll
        for (int i = NV; i < 2 * NV; i++) other[i * p.stride + s] = T(0);
}

// A copy of v that the compiler cannot see through.  The FP32-storage
// kernels widen each lambda_f twice (for its moments and for its output)
// rather than keep the widened value live in two registers through the whole
// site; without the copy the two widenings merge into one.
template <typename T, typename AR>
__device__ __forceinline__ T opaque_copy(T v)
{
    if constexpr (!std::is_same<T, AR>::value) asm("" : "+v"(v));
    return v;
}

// Transposed propagation (gather lambda*_i(x) = lambda_i(x + c_i)), then the
// transposed local collision Jacobian at x with the forward locals recomputed
// from the saved state; writes lf, lg of the previous level, the stencil
// cotangents, and block partials of d/d(A, B, kappa).
template <typename T, typename AR, bool DEV, bool G1>
__device__ __forceinline__ void adj_local_body(const KParams& p, const T* __restrict__ F,
                                               const double* __restrict__ phi,
                                               const T* __restrict__ an, T* __restrict__ ap,
                                               T* __restrict__ sc, double* __restrict__ partials)
{
    double dth[3] = {0.0, 0.0, 0.0};
    const unsigned S = p.stride;
    for (XcdSweep w = xcd_sweep(p.nsites, kBlock); w.s < w.end; w.s += w.stride) {
        const int s = w.s;
        const Geo q = geo_of(p, s);
        T lfr[NV], lgr[NV], lpr[NV], f[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const int d = push_site(p, q, i);
            // lambda_f and lambda_g of the later level are read once (non-
            // temporal); lambda_phi at d is gathered by 19 sites (cached)
            lfr[i] = __builtin_nontemporal_load(&an[i * S + d]);
            lgr[i] = G1 ? T(0) : __builtin_nontemporal_load(&an[(NV + i) * S + d]);
            lpr[i] = an[2 * NV * S + d];
            f[i] = F[dist_pull(p, q, i)];
        }
        const Stencil st = stencil(phi[s], phi[site_of(p, q.xp, q.y, q.z)],
                                   phi[site_of(p, q.xm, q.y, q.z)],
                                   phi[site_of(p, q.x, q.yp, q.z)],
                                   phi[site_of(p, q.x, q.ym, q.z)],
                                   phi[site_of(p, q.x, q.y, q.zp)],
                                   phi[site_of(p, q.x, q.y, q.zm)]);
        const AR A = AR(p.A), B = AR(p.B), kap = AR(p.kappa), gam = AR(p.gamma);
        const AR omf = AR(p.omega_f), omg = AR(p.omega_g);
        const AR cf = AR(1) - omf, cg = AR(1) - omg;
        // g part first: its moments, and the previous level's lg, which no
        // later term needs
        AR t0 = 0, t1x = 0, t1y = 0, t1z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const AR lg = G1 ? AR(lpr[i]) : AR(lgr[i]) + AR(lpr[i]);
            const AR wg = AR(weight(i)) * omg * lg;
            t0 += wg;
            if (CX[i]) { t1x += CX[i] * wg; txx += wg; }
            if (CY[i]) { t1y += CY[i] * wg; tyy += wg; }
            if (CZ[i]) { t1z += CZ[i] * wg; tzz += wg; }
            if (CX[i] * CY[i]) txy += CX[i] * CY[i] * wg;
            if (CX[i] * CZ[i]) txz += CX[i] * CZ[i] * wg;
            if (CY[i] * CZ[i]) tyz += CY[i] * CZ[i] * wg;
            if (!G1) __builtin_nontemporal_store(T(cg * lg), &ap[(NV + i) * S + s]);
        }
        // the forward step's own rho and u (in the storage type's arithmetic)
        const Moments<T> mt = moments_of<T, DEV>(p, f);
        const T rit = T(1) / mt.rho;
        const AR ri = AR(rit);
        const AR ux = AR(mt.jx * rit), uy = AR(mt.jy * rit), uz = AR(mt.jz * rit);
        const AR phi_c = AR(st.phi), gx = AR(st.gx), gy = AR(st.gy), gz = AR(st.gz), lap = AR(st.lap);

        AR s0 = 0, s1x = 0, s1y = 0, s1z = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
        T lfc[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const AR wl = AR(weight(i)) * omf * AR(lfr[i]);
            s0 += wl;
            if (CX[i]) { s1x += CX[i] * wl; sxx += wl; }
            if (CY[i]) { s1y += CY[i] * wl; syy += wl; }
            if (CZ[i]) { s1z += CZ[i] * wl; szz += wl; }
            if (CX[i] * CY[i]) sxy += CX[i] * CY[i] * wl;
            if (CX[i] * CZ[i]) sxz += CX[i] * CZ[i] * wl;
            if (CY[i] * CZ[i]) syz += CY[i] * CZ[i] * wl;
            lfc[i] = opaque_copy<T, AR>(lfr[i]);
        }
        const AR third = AR(1.0 / 3.0);
        sxx -= third * s0; syy -= third * s0; szz -= third * s0;
        txx -= third * t0; tyy -= third * t0; tzz -= third * t0;
        const AR trs = sxx + syy + szz, trt = txx + tyy + tzz;
        const AR s2ux = sxx * ux + sxy * uy + sxz * uz;
        const AR s2uy = sxy * ux + syy * uy + syz * uz;
        const AR s2uz = sxz * ux + syz * uy + szz * uz;
        const AR t2ux = txx * ux + txy * uy + txz * uz;
        const AR t2uy = txy * ux + tyy * uy + tyz * uz;
        const AR t2uz = txz * ux + tyz * uy + tzz * uz;
        const AR s2uu = s2ux * ux + s2uy * uy + s2uz * uz;
        const AR t2uu = t2ux * ux + t2uy * uy + t2uz * uz;
        const AR t1u = t1x * ux + t1y * uy + t1z * uz;
        const AR s2gx = sxx * gx + sxy * gy + sxz * gz;
        const AR s2gy = sxy * gx + syy * gy + syz * gz;
        const AR s2gz = sxz * gx + syz * gy + szz * gz;
        const AR gsg = s2gx * gx + s2gy * gy + s2gz * gz;
        const AR h = AR(4.5);
        const AR pr = phi_c * ri;

        const AR arho = s0 - h * s2uu - AR(3) * pr * t1u - AR(9) * pr * t2uu;
        const AR ajx = AR(3) * s1x + AR(9) * s2ux + AR(3) * pr * t1x + AR(9) * pr * t2ux;
        const AR ajy = AR(3) * s1y + AR(9) * s2uy + AR(3) * pr * t1y + AR(9) * pr * t2uy;
        const AR ajz = AR(3) * s1z + AR(9) * s2uz + AR(3) * pr * t1z + AR(9) * pr * t2uz;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            AR v = cf * AR(lfc[i]) + arho;
            if (CX[i]) v += CX[i] * ajx;
            if (CY[i]) v += CY[i] * ajy;
            if (CZ[i]) v += CZ[i] * ajz;
            __builtin_nontemporal_store(T(v), &ap[i * S + s]);
        }
        const AR phi2 = phi_c * phi_c;
        const AR a_dir = h * trs * (A * phi_c + AR(3) * B * phi2 * phi_c - kap * lap) + t0
                      + AR(3) * t1u + h * (gam * (A + AR(3) * B * phi2) - third) * trt + h * t2uu;
        const AR hk = h * kap;
        __builtin_nontemporal_store(T(a_dir), &sc[0 * S + s]);
        __builtin_nontemporal_store(T(hk * (AR(2) * s2gx - trs * gx)), &sc[1 * S + s]);
        __builtin_nontemporal_store(T(hk * (AR(2) * s2gy - trs * gy)), &sc[2 * S + s]);
        __builtin_nontemporal_store(T(hk * (AR(2) * s2gz - trs * gz)), &sc[3 * S + s]);
        __builtin_nontemporal_store(T(-hk * (phi_c * trs + gam * trt)), &sc[4 * S + s]);
        const double g2 = st.gx * st.gx + st.gy * st.gy + st.gz * st.gz;
        const double dtrs = double(trs), dtrt = double(trt), dph = st.phi;
        dth[0] += 4.5 * (dtrs * 0.5 * dph * dph + p.gamma * dph * dtrt);
        dth[1] += 4.5 * (dtrs * 0.75 * dph * dph * dph * dph + p.gamma * dph * dph * dph * dtrt);
        dth[2] += 4.5 * (dtrs * (-dph * st.lap - 0.5 * g2) + double(gsg) - p.gamma * st.lap * dtrt);
    }
    block_partials<3>(dth, partials);
}

// FP32 storage with FP64 arithmetic: the transposed collision sums 19
// weighted cotangents into moments that nearly cancel, and in FP32 those
// roundings, repeated over a long rollout, dominated the gradient's error
// (1e-4 relative over 1000 steps at 128^3; 5e-6 in FP64, at no cost in
// time).  The forward's own rho and u are formed in FP32, as the step forms
// them, and then widened.  Register budgets: the g part goes first (its
// moments and its output need nothing of the f part) and lambda_f stays in
// FP32 until used, which fits 3 waves per SIMD (161 VGPRs, no spills; the
// plain order took 292 registers, one wave per SIMD, and capping that at 2
// waves made the compiler serialise the loads: 2.2x slower).  The FP32
// kernel runs 3-5% faster this way; the FP64 ones gain nothing but are kept
// at the budget that needs no AGPRs.
template <bool G1>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_adj_local_f32(
    KParams p, const float* __restrict__ F, const double* __restrict__ phi,
    const float* __restrict__ an, float* __restrict__ ap, float* __restrict__ sc,
    double* __restrict__ partials)
{
    adj_local_body<float, double, true, G1>(p, F, phi, an, ap, sc, partials);
}

template <bool G1>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adj_local_f64(
    KParams p, const double* __restrict__ F, const double* __restrict__ phi,
    const double* __restrict__ an, double* __restrict__ ap, double* __restrict__ sc,
    double* __restrict__ partials)
{
    adj_local_body<double, double, false, G1>(p, F, phi, an, ap, sc, partials);
}

// Force coupling (u = (j + F/2)/rho in both equilibria, f^eq = w rho (1 +
// 3 c.u + 9/2 (c.u)^2 - 3/2 u^2), Guo's source S = (1 - omega_f/2) w
// [3(c - u) + 9 (c.u) c].F, F = -div Pi).  With M0, M1, M2 the moments
// sum w L, sum w L c, sum w L c c of L = lambda*_f (full M2), and the g
// part's T moments as above:
//   dPhi/du   = omega_f rho (3 M1 + 9 M2 u - 3 u M0) + (1 - omega_f/2)
//               (9 M2 F - 3 F M0) + 3 phi T1 + 9 phi T2 u
//   dPhi/drho = omega_f (M0 + 3 M1.u + 9/2 u.M2.u - 3/2 u^2 M0) - dPhi/du . u / rho
//   dPhi/dj   = dPhi/du / rho
//   dPhi/dF   = (1 - omega_f/2) (3 M1 - 3 u M0 + 9 M2 u) + dPhi/du / (2 rho)
// and the g part's phi, mu terms as in the stress coupling without S2.
// dPhi/dF (three fields after the five stencil cotangents) reaches phi
// through Pi at the face neighbours: k_adj_force_pi.
// F_IN: F comes from k_adj_force_f in the dL/dF slots of sc (read at the own
// site before they are overwritten), instead of being formed here.
template <typename T, typename AR, bool DEV, bool F_IN, bool G1>
__device__ __forceinline__ void adj_local_force_body(const KParams& p, const T* __restrict__ F,
                                                     const double* __restrict__ phi,
                                                     const T* __restrict__ an, T* __restrict__ ap,
                                                     T* __restrict__ sc,
                                                     double* __restrict__ partials)
{
    double dth[3] = {0.0, 0.0, 0.0};
    const unsigned S = p.stride;
    const AR A = AR(p.A), B = AR(p.B), kap = AR(p.kappa), gam = AR(p.gamma);
    const AR omf = AR(p.omega_f), omg = AR(p.omega_g), pref = AR(1) - AR(0.5) * omf;
    const AR h = AR(4.5), third = AR(1.0 / 3.0);
    for (XcdSweep w = xcd_sweep(p.nsites, kBlock); w.s < w.end; w.s += w.stride) {
        const int s = w.s;
        const Geo q = geo_of(p, s);
        T lfr[NV], lgr[NV], lpr[NV], f[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const int d = push_site(p, q, i);
            lfr[i] = __builtin_nontemporal_load(&an[i * S + d]);
            lgr[i] = G1 ? T(0) : __builtin_nontemporal_load(&an[(NV + i) * S + d]);
            lpr[i] = an[2 * NV * S + d];
            f[i] = F[dist_pull(p, q, i)];
        }
        const Stencil st = stencil(phi[s], phi[site_of(p, q.xp, q.y, q.z)],
                                   phi[site_of(p, q.xm, q.y, q.z)],
                                   phi[site_of(p, q.x, q.yp, q.z)],
                                   phi[site_of(p, q.x, q.ym, q.z)],
                                   phi[site_of(p, q.x, q.y, q.zp)],
                                   phi[site_of(p, q.x, q.y, q.zm)]);
        // the forward step's own F, rho and u (the storage type's arithmetic)
        T Ft[3];
        if (F_IN) {
            Ft[0] = sc[5 * S + s];
            Ft[1] = sc[6 * S + s];
            Ft[2] = sc[7 * S + s];
        } else {
            double Fd[3];
            force_from_phi(p, q, phi, Fd);
            Ft[0] = T(Fd[0]);
            Ft[1] = T(Fd[1]);
            Ft[2] = T(Fd[2]);
        }
        const Moments<T> mt = moments_of<T, DEV>(p, f);
        const T rit = T(1) / mt.rho;
        const AR Fx = AR(Ft[0]), Fy = AR(Ft[1]), Fz = AR(Ft[2]);
        const AR rho = AR(mt.rho), ri = AR(rit);
        const AR ux = AR((mt.jx + T(0.5) * Ft[0]) * rit), uy = AR((mt.jy + T(0.5) * Ft[1]) * rit),
                 uz = AR((mt.jz + T(0.5) * Ft[2]) * rit);
        const AR phi_c = AR(st.phi);

        const AR cf = AR(1) - omf, cg = AR(1) - omg;
        AR t0 = 0, t1x = 0, t1y = 0, t1z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const AR lg = G1 ? AR(lpr[i]) : AR(lgr[i]) + AR(lpr[i]);
            const AR wg = AR(weight(i)) * omg * lg;
            t0 += wg;
            if (CX[i]) { t1x += CX[i] * wg; txx += wg; }
            if (CY[i]) { t1y += CY[i] * wg; tyy += wg; }
            if (CZ[i]) { t1z += CZ[i] * wg; tzz += wg; }
            if (CX[i] * CY[i]) txy += CX[i] * CY[i] * wg;
            if (CX[i] * CZ[i]) txz += CX[i] * CZ[i] * wg;
            if (CY[i] * CZ[i]) tyz += CY[i] * CZ[i] * wg;
            if (!G1) __builtin_nontemporal_store(T(cg * lg), &ap[(NV + i) * S + s]);
        }
        AR m0 = 0, m1x = 0, m1y = 0, m1z = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0;
        T lfc[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const AR wl = AR(weight(i)) * AR(lfr[i]);
            m0 += wl;
            if (CX[i]) { m1x += CX[i] * wl; mxx += wl; }
            if (CY[i]) { m1y += CY[i] * wl; myy += wl; }
            if (CZ[i]) { m1z += CZ[i] * wl; mzz += wl; }
            if (CX[i] * CY[i]) mxy += CX[i] * CY[i] * wl;
            if (CX[i] * CZ[i]) mxz += CX[i] * CZ[i] * wl;
            if (CY[i] * CZ[i]) myz += CY[i] * CZ[i] * wl;
            lfc[i] = opaque_copy<T, AR>(lfr[i]);
        }
        txx -= third * t0; tyy -= third * t0; tzz -= third * t0;
        const AR trt = txx + tyy + tzz;
        const AR t2ux = txx * ux + txy * uy + txz * uz;
        const AR t2uy = txy * ux + tyy * uy + tyz * uz;
        const AR t2uz = txz * ux + tyz * uy + tzz * uz;
        const AR t2uu = t2ux * ux + t2uy * uy + t2uz * uz;
        const AR t1u = t1x * ux + t1y * uy + t1z * uz;
        const AR m2ux = mxx * ux + mxy * uy + mxz * uz;
        const AR m2uy = mxy * ux + myy * uy + myz * uz;
        const AR m2uz = mxz * ux + myz * uy + mzz * uz;
        const AR m2Fx = mxx * Fx + mxy * Fy + mxz * Fz;
        const AR m2Fy = mxy * Fx + myy * Fy + myz * Fz;
        const AR m2Fz = mxz * Fx + myz * Fy + mzz * Fz;
        const AR uu = ux * ux + uy * uy + uz * uz;
        const AR orho = omf * rho;
        const AR lux = orho * (AR(3) * m1x + AR(9) * m2ux - AR(3) * ux * m0)
                    + pref * (AR(9) * m2Fx - AR(3) * Fx * m0) + phi_c * (AR(3) * t1x + AR(9) * t2ux);
        const AR luy = orho * (AR(3) * m1y + AR(9) * m2uy - AR(3) * uy * m0)
                    + pref * (AR(9) * m2Fy - AR(3) * Fy * m0) + phi_c * (AR(3) * t1y + AR(9) * t2uy);
        const AR luz = orho * (AR(3) * m1z + AR(9) * m2uz - AR(3) * uz * m0)
                    + pref * (AR(9) * m2Fz - AR(3) * Fz * m0) + phi_c * (AR(3) * t1z + AR(9) * t2uz);
        const AR arho = omf * (m0 + AR(3) * (m1x * ux + m1y * uy + m1z * uz)
                              + h * (m2ux * ux + m2uy * uy + m2uz * uz) - AR(1.5) * uu * m0)
                     - (lux * ux + luy * uy + luz * uz) * ri;
        const AR ajx = lux * ri, ajy = luy * ri, ajz = luz * ri;
        const AR hr = AR(0.5) * ri;
        const AR lFx = pref * (AR(3) * m1x - AR(3) * ux * m0 + AR(9) * m2ux) + hr * lux;
        const AR lFy = pref * (AR(3) * m1y - AR(3) * uy * m0 + AR(9) * m2uy) + hr * luy;
        const AR lFz = pref * (AR(3) * m1z - AR(3) * uz * m0 + AR(9) * m2uz) + hr * luz;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            AR v = cf * AR(lfc[i]) + arho;
            if (CX[i]) v += CX[i] * ajx;
            if (CY[i]) v += CY[i] * ajy;
            if (CZ[i]) v += CZ[i] * ajz;
            __builtin_nontemporal_store(T(v), &ap[i * S + s]);
        }
        const AR phi2 = phi_c * phi_c;
        const AR a_dir = t0 + AR(3) * t1u + h * (gam * (A + AR(3) * B * phi2) - third) * trt + h * t2uu;
        sc[0 * S + s] = T(a_dir);
        sc[1 * S + s] = T(0);
        sc[2 * S + s] = T(0);
        sc[3 * S + s] = T(0);
        sc[4 * S + s] = T(-h * kap * gam * trt);
        sc[5 * S + s] = T(lFx);
        sc[6 * S + s] = T(lFy);
        sc[7 * S + s] = T(lFz);
        const double dtrt = double(trt), dph = st.phi;
        dth[0] += 4.5 * p.gamma * dph * dtrt;
        dth[1] += 4.5 * p.gamma * dph * dph * dph * dtrt;
        dth[2] += -4.5 * p.gamma * st.lap * dtrt;
    }
    block_partials<3>(dth, partials);
}

template <bool G1>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adj_local_force_f32(
    KParams p, const float* __restrict__ F, const double* __restrict__ phi,
    const float* __restrict__ an, float* __restrict__ ap, float* __restrict__ sc,
    double* __restrict__ partials)
{
    adj_local_force_body<float, double, true, false, G1>(p, F, phi, an, ap, sc, partials);
}

template <bool G1>
__global__ __launch_bounds__(kBlock) void k_adj_local_force_f64(
    KParams p, const double* __restrict__ F, const double* __restrict__ phi,
    const double* __restrict__ an, double* __restrict__ ap, double* __restrict__ sc,
    double* __restrict__ partials)
{
    adj_local_force_body<double, double, false, true, G1>(p, F, phi, an, ap, sc, partials);
}

// F = -div Pi of the phi field (T-rounded, as the forward uses it) into the
// dL/dF slots of sc, one site per thread.  FP64 runs it before its local
// kernel: formed there, F's six neighbour stencils made that kernel (which
// holds 256 VGPRs) half again as slow; in FP32 forming it inline costs
// nothing measurable, and this pass would.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_force_f(KParams p, const double* __restrict__ phi,
                                                        T* __restrict__ sc)
{
    const int s = xcd_block() * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    double Fd[3];
    force_from_phi(p, geo_of(p, s), phi, Fd);
    sc[5 * size_t(p.stride) + s] = T(Fd[0]);
    sc[6 * size_t(p.stride) + s] = T(Fd[1]);
    sc[7 * size_t(p.stride) + s] = T(Fd[2]);
}

// F_a(x) = -sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)]/2 transposed: Pi(y) takes
// L = (K + K^T)/2, K_ab(y) = [lambda_F,a(y + e_b) - lambda_F,a(y - e_b)]/2,
// and Pi_ab = iso delta_ab + kappa d_a phi d_b phi (iso = A/2 phi^2 +
// 3B/4 phi^4 - kappa phi lap - kappa/2 |grad|^2) passes it on to the
// stencil cotangents at y:
//   a += trL (A phi + 3B phi^3 - kappa lap),  b += kappa (2 L grad - trL grad),
//   c += -kappa phi trL,
// and d/d(A, B, kappa) += trL (phi^2/2, 3 phi^4/4, -phi lap - |grad|^2/2)
// + (0, 0, grad.L.grad).  Each site updates only its own cotangents.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_force_pi(KParams p, const double* __restrict__ phi,
                                                         T* __restrict__ sc,
                                                         double* __restrict__ partials)
{
    double dth[3] = {0.0, 0.0, 0.0};
    const unsigned S = p.stride;
    const T* __restrict__ lF[3] = {sc + 5 * size_t(S), sc + 6 * size_t(S), sc + 7 * size_t(S)};
    const T A = T(p.A), B = T(p.B), kap = T(p.kappa);
    for (XcdSweep w = xcd_sweep(p.nsites, kBlock); w.s < w.end; w.s += w.stride) {
        const int s = w.s;
        const Geo q = geo_of(p, s);
        const int nb[3][2] = {{site_of(p, q.xp, q.y, q.z), site_of(p, q.xm, q.y, q.z)},
                              {site_of(p, q.x, q.yp, q.z), site_of(p, q.x, q.ym, q.z)},
                              {site_of(p, q.x, q.y, q.zp), site_of(p, q.x, q.y, q.zm)}};
        T K[3][3];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) K[a][b] = T(0.5) * (lF[a][nb[b][0]] - lF[a][nb[b][1]]);
        const T Lxx = K[0][0], Lyy = K[1][1], Lzz = K[2][2];
        const T Lxy = T(0.5) * (K[0][1] + K[1][0]);
        const T Lxz = T(0.5) * (K[0][2] + K[2][0]);
        const T Lyz = T(0.5) * (K[1][2] + K[2][1]);
        const Stencil st = stencil(phi[s], phi[nb[0][0]], phi[nb[0][1]], phi[nb[1][0]],
                                   phi[nb[1][1]], phi[nb[2][0]], phi[nb[2][1]]);
        const T ph = T(st.phi), gx = T(st.gx), gy = T(st.gy), gz = T(st.gz), lap = T(st.lap);
        const T trL = Lxx + Lyy + Lzz;
        const T Lgx = Lxx * gx + Lxy * gy + Lxz * gz;
        const T Lgy = Lxy * gx + Lyy * gy + Lyz * gz;
        const T Lgz = Lxz * gx + Lyz * gy + Lzz * gz;
        const T ph2 = ph * ph;
        sc[0 * S + s] += trL * (A * ph + T(3) * B * ph2 * ph - kap * lap);
        sc[1 * S + s] += kap * (T(2) * Lgx - trL * gx);
        sc[2 * S + s] += kap * (T(2) * Lgy - trL * gy);
        sc[3 * S + s] += kap * (T(2) * Lgz - trL * gz);
        sc[4 * S + s] += -kap * ph * trL;
        const double dtr = double(trL), dph = st.phi;
        const double g2 = st.gx * st.gx + st.gy * st.gy + st.gz * st.gz;
        const double gLg = double(Lgx) * st.gx + double(Lgy) * st.gy + double(Lgz) * st.gz;
        dth[0] += dtr * 0.5 * dph * dph;
        dth[1] += dtr * 0.75 * dph * dph * dph * dph;
        dth[2] += dtr * (-dph * st.lap - 0.5 * g2) + gLg;
    }
    block_partials<3>(dth, partials);
}

// lp(x) = a(x) - sum_a D_a b_a (x) + lap c (x).  With dtheta, workgroups
// 0-2 also add the step's d/d(A, B, kappa) from the local kernel's nparts
// block partials, and from k_adj_force_pi's in partials2 if given (instead
// of a launch of its own).
template <typename T>
__device__ __forceinline__ void adj_stencil_site(const KParams& p, int s, const T* __restrict__ sc,
                                                 T* __restrict__ ap)
{
    const Geo q = geo_of(p, s);
    const unsigned S = p.stride;
    const int xp = site_of(p, q.xp, q.y, q.z), xm = site_of(p, q.xm, q.y, q.z);
    const int yp = site_of(p, q.x, q.yp, q.z), ym = site_of(p, q.x, q.ym, q.z);
    const int zp = site_of(p, q.x, q.y, q.zp), zm = site_of(p, q.x, q.y, q.zm);
    const T* a = sc;
    const T* bx = sc + S;
    const T* by = sc + 2 * S;
    const T* bz = sc + 3 * S;
    const T* c = sc + 4 * S;
    const T cc = c[s];
    const T divb = T(0.5) * (bx[xp] - bx[xm]) + T(0.5) * (by[yp] - by[ym]) + T(0.5) * (bz[zp] - bz[zm]);
    const T lapc = (c[xp] + c[xm] - T(2) * cc) + (c[yp] + c[ym] - T(2) * cc) + (c[zp] + c[zm] - T(2) * cc);
    ap[2 * NV * S + s] = a[s] - divb + lapc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_stencil(KParams p, const T* __restrict__ sc,
                                                        T* __restrict__ ap,
                                                        const double* __restrict__ partials,
                                                        const double* __restrict__ partials2,
                                                        int nparts, double* __restrict__ dtheta)
{
    const int s = xcd_block() * kBlock + threadIdx.x;
    if (s < p.nsites) adj_stencil_site<T>(p, s, sc, ap);
    if (!dtheta) return;
    // workgroup k < 3 adds component k (one workgroup does all three on a
    // grid smaller than that), so no workgroup carries the whole reduction
    const int k0 = gridDim.x >= 3 ? int(blockIdx.x) : 0;
    const int nk = gridDim.x >= 3 ? 1 : 3;
    if (int(blockIdx.x) != k0 || k0 >= 3) return;
    reduce_partials_block(partials + size_t(k0) * nparts, nparts, nk, dtheta + k0, true);
    if (partials2) {
        __syncthreads();
        reduce_partials_block(partials2 + size_t(k0) * nparts, nparts, nk, dtheta + k0, true);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_phi0(KParams p, const T* __restrict__ adj,
                                                     double* __restrict__ out)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    // LB scheme: dL/dphi0 = dL/dg_0 = lg_0 + lp (the rest state holds phi0
    // in g_0); FD scheme: the phi field itself
    const double lp = double(adj[2 * NV * p.stride + s]);
    out[s] = p.fd ? lp : double(adj[NV * p.stride + s]) + lp;
}

// Dense FP64 copy of an adjoint level: df[i][s] = lf_i(s) and, LB scheme,
// dg[i][s] = lg_i(s) + lp(s) = dL/dg_i(s), each (19, nx, ny, nz); the FD
// scheme has no g (dg is null there).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_export(KParams p, const T* __restrict__ adj,
                                                       double* __restrict__ df,
                                                       double* __restrict__ dg)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const long long n = p.nsites;
    if (df)
#pragma unroll
        for (int i = 0; i < NV; i++) df[i * n + s] = double(adj[size_t(i) * p.stride + s]);
    if (dg) {
        const double lp = double(adj[size_t(2 * NV) * p.stride + s]);
#pragma unroll
        for (int i = 0; i < NV; i++)
            dg[i * n + s] = double(adj[size_t(NV + i) * p.stride + s]) + lp;
    }
}

int grid_for(const KParams& p) { return (p.nsites + kBlock - 1) / kBlock; }

// tau_g = 1: the levels' lg is identically zero (see the top of this file)
bool g_free(const KParams& p) { return p.omega_g == 1.0; }

int reduction_grid(const KParams& p)
{
    const int g = grid_for(p);
    return g < kMaxPartialBlocks ? g : kMaxPartialBlocks;
}

}  // namespace

hipError_t launch_adj_seed(const KParams& p, bool fp32, void* adj, void* other, const double* dphi,
                           hipStream_t s)
{
    if (!g_free(p)) other = nullptr;
    if (fp32)
        k_adj_seed<float><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<float*>(adj),
                                                         static_cast<float*>(other), dphi);
    else
        k_adj_seed<double><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<double*>(adj),
                                                          static_cast<double*>(other), dphi);
    return hipGetLastError();
}

hipError_t launch_adj_step(const KParams& p, bool fp32, const void* state,
                           const double* phi_given, double* phi,
                           const void* adj_next, void* adj_prev, void* adj_scratch,
                           double* partials, double* dtheta, hipStream_t s)
{
    if (phi_given) {
        // phi of state stored by the step that made its successor
        phi = const_cast<double*>(phi_given);
    } else {
        hipError_t e = launch_phi(p, fp32, state, phi, s);
        if (e != hipSuccess) return e;
    }
    // 1024 workgroups of 256 threads, each thread looping over its sites (a
    // few resident rounds at the local kernels' 1-3 waves per SIMD; a grid
    // of exactly one round measured no faster); the parameter reduction (in
    // the stencil kernel's first workgroups) then reads half the partials of
    // 2048 workgroups (measured as a launch of its own at 128^3: 9.9 -> 5.5
    // us, k_adj_local unchanged)
    constexpr int kAdjBlocks = 1024;
    const int nb = reduction_grid(p) < kAdjBlocks ? reduction_grid(p) : kAdjBlocks;
    // force coupling: the second pass's partials follow the first's
    double* partials2 = p.force ? partials + 3 * kAdjBlocks : nullptr;
    if (fp32) {
        const float* F = static_cast<const float*>(state);
        const float* an = static_cast<const float*>(adj_next);
        float* ap = static_cast<float*>(adj_prev);
        float* sc = static_cast<float*>(adj_scratch);
        if (p.force) {
            if (g_free(p))
                k_adj_local_force_f32<true><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
            else
                k_adj_local_force_f32<false><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
            k_adj_force_pi<float><<<nb, kBlock, 0, s>>>(p, phi, sc, partials2);
        } else if (g_free(p)) {
            k_adj_local_f32<true><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
        } else {
            k_adj_local_f32<false><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
        }
    } else {
        const double* F = static_cast<const double*>(state);
        const double* an = static_cast<const double*>(adj_next);
        double* ap = static_cast<double*>(adj_prev);
        double* sc = static_cast<double*>(adj_scratch);
        if (p.force) {
            k_adj_force_f<double><<<grid_for(p), kBlock, 0, s>>>(p, phi, sc);
            if (g_free(p))
                k_adj_local_force_f64<true><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
            else
                k_adj_local_force_f64<false><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
            k_adj_force_pi<double><<<nb, kBlock, 0, s>>>(p, phi, sc, partials2);
        } else if (g_free(p)) {
            k_adj_local_f64<true><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
        } else {
            k_adj_local_f64<false><<<nb, kBlock, 0, s>>>(p, F, phi, an, ap, sc, partials);
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_adj_stencil(p, fp32, adj_scratch, adj_prev, partials, partials2, nb, dtheta, s);
}

hipError_t launch_adj_force_pi(const KParams& p, bool fp32, const double* phi, void* adj_scratch,
                               double* partials2, int nblocks, hipStream_t s)
{
    if (fp32)
        k_adj_force_pi<float><<<nblocks, kBlock, 0, s>>>(p, phi, static_cast<float*>(adj_scratch),
                                                         partials2);
    else
        k_adj_force_pi<double><<<nblocks, kBlock, 0, s>>>(p, phi, static_cast<double*>(adj_scratch),
                                                          partials2);
    return hipGetLastError();
}

hipError_t launch_adj_stencil(const KParams& p, bool fp32, const void* adj_scratch,
                              void* adj_prev, const double* partials, const double* partials2,
                              int nparts, double* dtheta, hipStream_t s)
{
    if (fp32)
        k_adj_stencil<float><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const float*>(adj_scratch),
                                                            static_cast<float*>(adj_prev), partials,
                                                            partials2, nparts, dtheta);
    else
        k_adj_stencil<double><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const double*>(adj_scratch),
                                                             static_cast<double*>(adj_prev), partials,
                                                             partials2, nparts, dtheta);
    return hipGetLastError();
}

hipError_t launch_adj_phi0(const KParams& p, bool fp32, const void* adj, double* dphi0, hipStream_t s)
{
    if (fp32)
        k_adj_phi0<float><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const float*>(adj), dphi0);
    else
        k_adj_phi0<double><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const double*>(adj), dphi0);
    return hipGetLastError();
}

hipError_t launch_adj_export(const KParams& p, bool fp32, const void* adj, double* df, double* dg,
                             hipStream_t s)
{
    if (fp32)
        k_adj_export<float><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const float*>(adj), df, dg);
    else
        k_adj_export<double><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const double*>(adj), df,
                                                            dg);
    return hipGetLastError();
}

}  // namespace lbk
