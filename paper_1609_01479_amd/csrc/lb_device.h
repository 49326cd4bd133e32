// Device-side building blocks shared by the forward and adjoint kernels:
// the D3Q19 lattice, periodic site geometry, the pull of a stored time level,
// and the local physics (order-parameter stencil, chemical potential and
// stress, equilibria, BGK).
//
// Stored time level (pre-propagation, post-collision values at site y):
//   FP64 mode  (T = double, DEV = REF = false):
//       F_i(y) = f*_i(y),  G_i(y) = g*_i(y)
//   FP32 mode  (T = float,  DEV = REF = true):
//       F_i(y) = f*_i(y) - w_i rho0                          (FP32)
//       G_i(y) = g*_i(y) - r_i phi_c(y + c_i)                (FP32)
//       phi_c(x) = the order parameter of x's last collision with the low
//                  32 bits of its binary64 encoding cleared      (32 bits)
//   with r_i = w_i (1 - 3/2 (|c_i|^2 - 1)) = (5/6, 1/18, -1/72): r_i phi is
//   the order-parameter equilibrium of a fluid at rest with mu = 0 and
//   sum_i r_i = 1.  Each stored g deviation is referenced to the order
//   parameter of the site it propagates TO, so the pull at x needs only x's
//   own phi_c:  g_i(x) = G_i(x - c_i) + r_i phi_c(x),
//   phi(x) = phi_c(x) + sum_i G_i(x - c_i).  Both stored deviations are small
//   in the bulk phases, so FP32 rounding does not accumulate into the O(1)
//   order parameter.  The reference need not be phi itself, only a value
//   writer and reader share exactly: phi truncated to its high word (20
//   mantissa bits, stored as that word) leaves at most 2^-20 |phi| in the
//   deviations, whose FP32 rounding then stays ~2^-44 |phi|, and halves the
//   reference's traffic against an FP64 phi_c.
// Post-propagation values at x are the pull  f_i(x) = f*_i(x - c_i).
// Memory layout of F and G: didx() below; phi_c is one 32-bit word per site
// in site order (x*ny + y)*nz + z.
#pragma once

#include "lb_internal.h"

namespace lbk {
namespace dev {

constexpr int kBlock = 256;

// D3Q19 velocities: rest, +-x, +-y, +-z, 12 edges (ABI order).
constexpr int CX[NV] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[NV] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[NV] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr double weight(int i)
{
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// rest-state order-parameter equilibrium weights r_i
__host__ __device__ constexpr double rweight(int i)
{
    return i == 0 ? 5.0 / 6.0 : (i < 7 ? 1.0 / 18.0 : -1.0 / 72.0);
}

// ---------------------------------------------------------------------------
// Periodic geometry.

struct Geo {
    int x, y, z, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ int wrapm(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrapp(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// In an x-slab shard (p.xh > 0) x is not periodic: x - 1 and x + 1 of the
// boundary planes are the halo planes -1 and nx.
__device__ __forceinline__ Geo geo_xyz(const KParams& p, int x, int y, int z)
{
    Geo q;
    q.x = x; q.y = y; q.z = z;
    q.xm = p.xh ? x - 1 : wrapm(x, p.nx); q.xp = p.xh ? x + 1 : wrapp(x, p.nx);
    q.ym = wrapm(y, p.ny); q.yp = wrapp(y, p.ny);
    q.zm = wrapm(z, p.nz); q.zp = wrapp(z, p.nz);
    return q;
}

__device__ __forceinline__ Geo geo_of(const KParams& p, int s)
{
    const int z = s % p.nz;
    const int t = s / p.nz;
    return geo_xyz(p, t / p.ny, t % p.ny, z);
}

__device__ __forceinline__ int site_of(const KParams& p, int x, int y, int z)
{
    return (x * p.ny + y) * p.nz + z;
}

// Index of site (x, y, z) in a level's phi_c field: site order, after one
// halo plane in an x-slab shard (x from -1 to nx there).
__device__ __forceinline__ int phic_site(const KParams& p, int x, int y, int z)
{
    return site_of(p, x + (p.xh >> 1), y, z);
}

// phi_c as stored (the high word of phi's binary64 encoding) and as used
// (that word with a zero low word); phic_round(phi) is the reference the
// store of phi_c(x) = phic_word(phi(x)) stands for.
__device__ __forceinline__ unsigned phic_word(double phi) { return unsigned(__double2hiint(phi)); }
__device__ __forceinline__ double phic_value(unsigned w) { return __hiloint2double(int(w), 0); }
__device__ __forceinline__ double phic_round(double phi) { return phic_value(phic_word(phi)); }

__device__ __forceinline__ int minus_c(int c, int v, int vm, int vp) { return c > 0 ? vm : (c < 0 ? vp : v); }
__device__ __forceinline__ int plus_c(int c, int v, int vm, int vp) { return c > 0 ? vp : (c < 0 ? vm : v); }

// x - c_i and x + c_i
__device__ __forceinline__ int pull_site(const KParams& p, const Geo& q, int i)
{
    return site_of(p, minus_c(CX[i], q.x, q.xm, q.xp), minus_c(CY[i], q.y, q.ym, q.yp),
                   minus_c(CZ[i], q.z, q.zm, q.zp));
}
__device__ __forceinline__ int push_site(const KParams& p, const Geo& q, int i)
{
    return site_of(p, plus_c(CX[i], q.x, q.xm, q.xp), plus_c(CY[i], q.y, q.ym, q.yp),
                   plus_c(CZ[i], q.z, q.zm, q.zp));
}

// Workgroup ids are dispatched round-robin over the 8 XCDs, each with its own
// L2.  This remaps them so that each XCD receives a contiguous run of ids
// (when the grid is a multiple of 8): neighbouring sites, whose pulls share
// cache lines, are then fetched into one L2.
__device__ __forceinline__ int xcd_block()
{
    const int b = blockIdx.x, nb = gridDim.x;
    return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

// Distribution layout of a time level (KParams layout fields, set by
// set_layout): element (i, x, y, z) of the F or G region at
//   x*plane_e + y*ry + (z >> vs)*zb + (z & vm) + i*cs,
// which covers the row-blocked default ((x*ny + y)*19 + i)*nz + z, one array
// per component, a site's components together, and blocks of 2^vs z-sites.
// Indices fit 32 bits (39*stride < 2^32 is checked at creation).  In an
// x-slab shard the regions start with p.xh halo planes, so plane x (from -2
// to nx + 1) is at (x + p.xh)*plane_e.
__device__ __forceinline__ unsigned row_off(const KParams& p, int y, int z)
{
    return unsigned(y) * p.ry + (unsigned(z) >> p.vs) * p.zb + (unsigned(z) & p.vm);
}
__device__ __forceinline__ unsigned didx(const KParams& p, int i, int x, int y, int z)
{
    return unsigned(x + p.xh) * p.plane_e + row_off(p, y, z) + unsigned(i) * p.cs;
}
// component i at x - c_i, at x itself, at x + c_i
__device__ __forceinline__ unsigned dist_pull(const KParams& p, const Geo& q, int i)
{
    return didx(p, i, minus_c(CX[i], q.x, q.xm, q.xp), minus_c(CY[i], q.y, q.ym, q.yp),
                minus_c(CZ[i], q.z, q.zm, q.zp));
}
__device__ __forceinline__ unsigned dist_own(const KParams& p, const Geo& q, int i)
{
    return didx(p, i, q.x, q.y, q.z);
}

// ---------------------------------------------------------------------------
// Pull of the order-parameter populations.  d[i] = g_i(x) in FP64:
//   FP64 mode: G_i(x - c_i);  FP32 mode: G_i(x - c_i) + r_i phi_c(x).
// Returns phi(x): the index-order FP64 sum of the pulled values (FP64 mode),
// or phi_c(x) plus the index-order FP64 sum of the pulled deviations (FP32
// mode).  Every kernel forms phi this way, so a site's phi is bit-identical
// everywhere.
template <typename T, bool REF>
__device__ __forceinline__ double pull_g(const KParams& p, const Geo& q, const T* __restrict__ G,
                                         const unsigned* __restrict__ phic, double* d)
{
    double acc = 0.0;
    const double pc = REF ? phic_value(phic[phic_site(p, q.x, q.y, q.z)]) : 0.0;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const double gv = double(G[dist_pull(p, q, i)]);
        if (d) d[i] = REF ? __builtin_fma(rweight(i), pc, gv) : gv;
        acc += gv;
    }
    return REF ? pc + acc : acc;
}

template <typename T, bool REF>
__device__ __forceinline__ double phi_at(const KParams& p, const Geo& q, const T* __restrict__ G,
                                         const unsigned* __restrict__ phic)
{
    return pull_g<T, REF>(p, q, G, phic, nullptr);
}

// FP32 mode: pre-collision deviation g_i(x) - r_i phi(x) of the pulled
// stored value G = G_i(x - c_i), with dphi = phi(x) - phi_c(x).
template <typename T>
__device__ __forceinline__ T pre_collision_dev(int i, T G, double dphi)
{
    return T(double(G) - rweight(i) * dphi);
}

// FP32 mode: the stored value of direction i at y from the collided
// deviation h* = g* - r_i phi(y), the order parameter at y and that at the
// destination y + c_i, whose reference the store at y + c_i forms alike:
// G_i(y) = h* + r_i (phi(y) - phi_c(y + c_i)).
template <typename T>
__device__ __forceinline__ T to_dest_ref(int i, T hstar, double phi_here, double phi_dest)
{
    return T(__builtin_fma(rweight(i), phi_here - phic_round(phi_dest), double(hstar)));
}

// ---------------------------------------------------------------------------
// Local physics.

// Order-parameter derivatives from the 7 stencil values (FP64 differences).
struct Stencil {
    double phi, gx, gy, gz, lap;
};

__device__ __forceinline__ Stencil stencil(double c, double xp, double xm, double yp, double ym,
                                           double zp, double zm)
{
    Stencil s;
    s.phi = c;
    s.gx = 0.5 * (xp - xm);
    s.gy = 0.5 * (yp - ym);
    s.gz = 0.5 * (zp - zm);
    s.lap = (xp + xm - 2.0 * c) + (yp + ym - 2.0 * c) + (zp + zm - 2.0 * c);
    return s;
}

template <typename T>
struct Moments {
    T b;  // sum of the stored f (rho, or rho - rho0 in DEV)
    T rho, jx, jy, jz;
};

template <typename T, bool DEV>
__device__ __forceinline__ Moments<T> moments_of(const KParams& p, const T* f)
{
    Moments<T> m;
    T b = f[0];
#pragma unroll
    for (int i = 1; i < NV; i++) b += f[i];
    m.b = b;
    m.rho = DEV ? T(p.rho0) + b : b;
    m.jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    m.jy = (f[3] - f[4]) + (f[7] - f[8]) - (f[9] - f[10]) + (f[15] - f[16]) + (f[17] - f[18]);
    m.jz = (f[5] - f[6]) + (f[11] - f[12]) - (f[13] - f[14]) + (f[15] - f[16]) - (f[17] - f[18]);
    return m;
}

// BGK collision of one site, in place on f[] (stored convention: raw or
// deviation) and g[] (FP64 mode: g_i; FP32 mode: g_i - r_i phi).
//   mu = A phi + B phi^3 - kappa lap,  Pi = iso I + kappa grad grad,
//   f_eq = w [b + 3 c.j + 9/2 Q:(Pi + j j / rho)]           (b = sum f stored)
//   g_eq = w [phi + 3 phi c.u + 9/2 (Gamma mu - phi/3)(|c|^2 - 1)
//             + 9/2 phi ((c.u)^2 - |u|^2/3)]
//   g_eq - r phi = w [3 phi c.u + 9/2 Gamma mu (|c|^2 - 1) + 9/2 phi ((c.u)^2 - |u|^2/3)]
// collide_f does f and returns u = j/rho; collide_g does g.
template <typename T>
struct Vel {
    T x, y, z;
};

template <typename T, bool DEV>
__device__ __forceinline__ Vel<T> collide_f(const KParams& p, T* f, const Stencil& st)
{
    const T A = T(p.A), B = T(p.B), kap = T(p.kappa);
    const T omf = T(p.omega_f);
    const T phi = T(st.phi), gx = T(st.gx), gy = T(st.gy), gz = T(st.gz), lap = T(st.lap);
    const T phi2 = phi * phi;
    const T iso = T(0.5) * A * phi2 + T(0.75) * B * phi2 * phi2 - kap * phi * lap
                - T(0.5) * kap * (gx * gx + gy * gy + gz * gz);

    const Moments<T> m = moments_of<T, DEV>(p, f);
    const T b = m.b, jx = m.jx, jy = m.jy, jz = m.jz;
    const T ri = T(1) / m.rho;
    const T ux = jx * ri, uy = jy * ri, uz = jz * ri;

    // M = Pi + rho u u
    const T mxx = iso + kap * gx * gx + jx * ux;
    const T myy = iso + kap * gy * gy + jy * uy;
    const T mzz = iso + kap * gz * gz + jz * uz;
    const T mxy = kap * gx * gy + jx * uy;
    const T mxz = kap * gx * gz + jx * uz;
    const T myz = kap * gy * gz + jy * uz;
    const T tm = (mxx + myy + mzz) * T(1.0 / 3.0);

    const T h = T(4.5);
    const T w0 = T(weight(0)), wf = T(weight(1)), we = T(weight(7));
    const T wf3 = T(3.0 * weight(1)), we3 = T(3.0 * weight(7));

    T eq[NV];
    eq[0] = w0 * (b - h * tm);
    {
        const T sx = wf * (b + h * (mxx - tm)), ax = wf3 * jx;
        const T sy = wf * (b + h * (myy - tm)), ay = wf3 * jy;
        const T sz = wf * (b + h * (mzz - tm)), az = wf3 * jz;
        eq[1] = sx + ax; eq[2] = sx - ax;
        eq[3] = sy + ay; eq[4] = sy - ay;
        eq[5] = sz + az; eq[6] = sz - az;
    }
    {
        const T dxy = mxx + myy - tm, dxz = mxx + mzz - tm, dyz = myy + mzz - tm;
        const T s7 = we * (b + h * (dxy + T(2) * mxy)), a7 = we3 * (jx + jy);
        const T s9 = we * (b + h * (dxy - T(2) * mxy)), a9 = we3 * (jx - jy);
        const T s11 = we * (b + h * (dxz + T(2) * mxz)), a11 = we3 * (jx + jz);
        const T s13 = we * (b + h * (dxz - T(2) * mxz)), a13 = we3 * (jx - jz);
        const T s15 = we * (b + h * (dyz + T(2) * myz)), a15 = we3 * (jy + jz);
        const T s17 = we * (b + h * (dyz - T(2) * myz)), a17 = we3 * (jy - jz);
        eq[7] = s7 + a7;     eq[8] = s7 - a7;
        eq[9] = s9 + a9;     eq[10] = s9 - a9;
        eq[11] = s11 + a11;  eq[12] = s11 - a11;
        eq[13] = s13 + a13;  eq[14] = s13 - a13;
        eq[15] = s15 + a15;  eq[16] = s15 - a15;
        eq[17] = s17 + a17;  eq[18] = s17 - a17;
    }
#pragma unroll
    for (int i = 0; i < NV; i++) f[i] += omf * (eq[i] - f[i]);
    return Vel<T>{ux, uy, uz};
}

template <typename T, bool REF>
__device__ __forceinline__ void collide_g(const KParams& p, T* g, T phi, T mu, Vel<T> u)
{
    const T gam = T(p.gamma), omg = T(p.omega_g);
    const T ux = u.x, uy = u.y, uz = u.z;
    const T h = T(4.5);
    const T w0 = T(weight(0)), wf = T(weight(1)), we = T(weight(7));
    const T wf3 = T(3.0 * weight(1)), we3 = T(3.0 * weight(7));
    T eq[NV];

    const T uu3 = (ux * ux + uy * uy + uz * uz) * T(1.0 / 3.0);
    const T hp = h * phi;
    // rest, face and edge parts of (g_eq or g_eq - r phi) without the c.u terms
    T e0, ef, ee;
    if (REF) {
        const T hgm = h * gam * mu;
        e0 = w0 * (-hgm - hp * uu3);
        ef = -hp * uu3;          // times wf below, plus hp (c.u)^2
        ee = hgm - hp * uu3;     // times we below, plus hp (c.u)^2
    } else {
        const T sg = gam * mu - phi * T(1.0 / 3.0);
        e0 = w0 * (phi - h * sg - hp * uu3);
        ef = phi - hp * uu3;
        ee = phi + h * sg - hp * uu3;
    }
    eq[0] = e0;
    {
        const T p3f = wf3 * phi;
        const T sx = wf * (ef + hp * ux * ux);
        const T sy = wf * (ef + hp * uy * uy);
        const T sz = wf * (ef + hp * uz * uz);
        eq[1] = sx + p3f * ux; eq[2] = sx - p3f * ux;
        eq[3] = sy + p3f * uy; eq[4] = sy - p3f * uy;
        eq[5] = sz + p3f * uz; eq[6] = sz - p3f * uz;
    }
    {
        const T p3e = we3 * phi;
        const T c7 = ux + uy, c9 = ux - uy, c11 = ux + uz, c13 = ux - uz, c15 = uy + uz,
                c17 = uy - uz;
        const T s7 = we * (ee + hp * c7 * c7), s9 = we * (ee + hp * c9 * c9);
        const T s11 = we * (ee + hp * c11 * c11), s13 = we * (ee + hp * c13 * c13);
        const T s15 = we * (ee + hp * c15 * c15), s17 = we * (ee + hp * c17 * c17);
        eq[7] = s7 + p3e * c7;     eq[8] = s7 - p3e * c7;
        eq[9] = s9 + p3e * c9;     eq[10] = s9 - p3e * c9;
        eq[11] = s11 + p3e * c11;  eq[12] = s11 - p3e * c11;
        eq[13] = s13 + p3e * c13;  eq[14] = s13 - p3e * c13;
        eq[15] = s15 + p3e * c15;  eq[16] = s15 - p3e * c15;
        eq[17] = s17 + p3e * c17;  eq[18] = s17 - p3e * c17;
    }
#pragma unroll
    for (int i = 0; i < NV; i++) g[i] += omg * (eq[i] - g[i]);
}

template <typename T, bool DEV, bool REF>
__device__ __forceinline__ void collide(const KParams& p, T* f, T* g, const Stencil& st)
{
    const Vel<T> u = collide_f<T, DEV>(p, f, st);
    const T A = T(p.A), B = T(p.B), kap = T(p.kappa);
    const T phi = T(st.phi), lap = T(st.lap);
    const T phi2 = phi * phi;
    const T mu = A * phi + B * phi2 * phi - kap * lap;
    collide_g<T, REF>(p, g, phi, mu, u);
}

// ---------------------------------------------------------------------------
// Force coupling (FP64): the chemical stress leaves f^eq and its central
// divergence F = -div Pi acts as a body force, with the half-force velocity
// u = (j + F/2)/rho and the forcing source (1 - omega/2) w [3(c - u) + 9(c.u) c].F
// (Guo, Zheng and Shi), so one collision adds exactly F to the momentum.

// mu and the chemical stress Pi (xx, xy, xz, yy, yz, zz) of one site.
__device__ __forceinline__ void chem_stress(const KParams& p, const Stencil& st, double* mu,
                                            double pi[6])
{
    const double phi = st.phi, phi2 = phi * phi, k = p.kappa;
    *mu = p.A * phi + p.B * phi2 * phi - k * st.lap;
    const double iso = 0.5 * p.A * phi2 + 0.75 * p.B * phi2 * phi2 - k * phi * st.lap
                     - 0.5 * k * (st.gx * st.gx + st.gy * st.gy + st.gz * st.gz);
    pi[0] = iso + k * st.gx * st.gx;
    pi[1] = k * st.gx * st.gy;
    pi[2] = k * st.gx * st.gz;
    pi[3] = iso + k * st.gy * st.gy;
    pi[4] = k * st.gy * st.gz;
    pi[5] = iso + k * st.gz * st.gz;
}

// In place on f[] and g[] in the stored convention (as collide()), in T:
//   f^eq_i = w rho [1 + 3 c.u + 9/2 ((c.u)^2 - |u|^2/3)],
//   g^eq_i = w [phi + 3 phi c.u + 9/2 ((Gamma mu - phi/3)(|c|^2 - 1) + phi ((c.u)^2 - |u|^2/3))],
//   g^eq_i - r_i phi = w [3 phi c.u + 9/2 (Gamma mu (|c|^2 - 1) + phi ((c.u)^2 - |u|^2/3))],
//   f*_i = f_i + omega_f (f^eq_i - f_i) + (1 - omega_f/2) w [3 (c - u).F + 9 (c.u)(c.F)].
// The f half of collide_force (returns u = (j + F/2)/rho) and the g half.
// collide_force_f forms omega f^eq_i + S_i from its Hermite moments, as
// collide_f forms f^eq_i: one value per direction pair from the even part and
// one from the odd, then f*_i = (1 - omega_f) f_i + that (about half the
// arithmetic of evaluating the two sums direction by direction).
template <typename T, bool DEV>
__device__ __forceinline__ Vel<T> collide_force_f(const KParams& p, T* f, const double Fd[3])
{
    const Moments<T> m = moments_of<T, DEV>(p, f);
    const T F[3] = {T(Fd[0]), T(Fd[1]), T(Fd[2])};
    const T ri = T(1) / m.rho;
    const T ux = (m.jx + T(0.5) * F[0]) * ri, uy = (m.jy + T(0.5) * F[1]) * ri,
            uz = (m.jz + T(0.5) * F[2]) * ri;
    const T omf = T(p.omega_f);
    const T pref = T(1) - T(0.5) * omf;
    // omega f^eq_i + S_i = w_i [omega b + 3 c.a + 9/2 (c c - I/3):M] with
    //   a = omega rho u + pref F,  M = omega rho u u + pref (u F + F u)
    const T orho = omf * m.rho;
    const T ob = omf * m.b;
    const T ax = orho * ux + pref * F[0], ay = orho * uy + pref * F[1], az = orho * uz + pref * F[2];
    const T pux = pref * ux, puy = pref * uy, puz = pref * uz;
    const T mxx = orho * ux * ux + T(2) * pux * F[0];
    const T myy = orho * uy * uy + T(2) * puy * F[1];
    const T mzz = orho * uz * uz + T(2) * puz * F[2];
    const T mxy = orho * ux * uy + (pux * F[1] + puy * F[0]);
    const T mxz = orho * ux * uz + (pux * F[2] + puz * F[0]);
    const T myz = orho * uy * uz + (puy * F[2] + puz * F[1]);
    const T tm = (mxx + myy + mzz) * T(1.0 / 3.0);
    const T h = T(4.5);
    const T w0 = T(weight(0)), wf = T(weight(1)), we = T(weight(7));
    const T wf3 = T(3.0 * weight(1)), we3 = T(3.0 * weight(7));
    T x[NV];
    x[0] = w0 * (ob - h * tm);
    {
        const T sx = wf * (ob + h * (mxx - tm)), vx = wf3 * ax;
        const T sy = wf * (ob + h * (myy - tm)), vy = wf3 * ay;
        const T sz = wf * (ob + h * (mzz - tm)), vz = wf3 * az;
        x[1] = sx + vx; x[2] = sx - vx;
        x[3] = sy + vy; x[4] = sy - vy;
        x[5] = sz + vz; x[6] = sz - vz;
    }
    {
        const T dxy = mxx + myy - tm, dxz = mxx + mzz - tm, dyz = myy + mzz - tm;
        const T s7 = we * (ob + h * (dxy + T(2) * mxy)), v7 = we3 * (ax + ay);
        const T s9 = we * (ob + h * (dxy - T(2) * mxy)), v9 = we3 * (ax - ay);
        const T s11 = we * (ob + h * (dxz + T(2) * mxz)), v11 = we3 * (ax + az);
        const T s13 = we * (ob + h * (dxz - T(2) * mxz)), v13 = we3 * (ax - az);
        const T s15 = we * (ob + h * (dyz + T(2) * myz)), v15 = we3 * (ay + az);
        const T s17 = we * (ob + h * (dyz - T(2) * myz)), v17 = we3 * (ay - az);
        x[7] = s7 + v7;     x[8] = s7 - v7;
        x[9] = s9 + v9;     x[10] = s9 - v9;
        x[11] = s11 + v11;  x[12] = s11 - v11;
        x[13] = s13 + v13;  x[14] = s13 - v13;
        x[15] = s15 + v15;  x[16] = s15 - v15;
        x[17] = s17 + v17;  x[18] = s17 - v17;
    }
    const T cf = T(1) - omf;
#pragma unroll
    for (int i = 0; i < NV; i++) f[i] = cf * f[i] + x[i];
    return Vel<T>{ux, uy, uz};
}

// G1 (omega_g = 1): g* = g^eq, with no term in the pre-collision g, which
// the caller then need not load.
template <typename T, bool REF, bool G1>
__device__ __forceinline__ void collide_force_g(const KParams& p, T* g, double phi_d, double mu_d,
                                                Vel<T> u)
{
    const T phi = T(phi_d), mu = T(mu_d);
    const T ux = u.x, uy = u.y, uz = u.z;
    const T uu3 = (ux * ux + uy * uy + uz * uz) * T(1.0 / 3.0);
    const T gm = T(p.gamma) * mu, sg = REF ? gm : gm - phi * T(1.0 / 3.0);
    const T omg = T(p.omega_g);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const T w = T(weight(i));
        const T cu = T(CX[i]) * ux + T(CY[i]) * uy + T(CZ[i]) * uz;
        const T q = cu * cu - uu3;
        const T c2m1 = T(CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i] - 1);
        const T geq = w * ((REF ? T(0) : phi) + T(3) * phi * cu + T(4.5) * (sg * c2m1 + phi * q));
        if (G1)
            g[i] = geq;
        else
            g[i] += omg * (geq - g[i]);
    }
}

template <typename T, bool DEV, bool REF, bool G1>
__device__ __forceinline__ void collide_force(const KParams& p, T* f, T* g, double phi_d, double mu_d,
                                              const double Fd[3])
{
    const Vel<T> u = collide_force_f<T, DEV>(p, f, Fd);
    collide_force_g<T, REF, G1>(p, g, phi_d, mu_d, u);
}

// Force coupling: F = -div Pi by central differences of Pi at the six face
// neighbours.  Each neighbour's Pi is formed from its own 7-point stencil of
// the phi field (phi within distance 2 of the site; neighbouring threads read
// the same values, so they come from cache) instead of being stored by a
// separate pass and read back.

// Pi (xx, xy, xz, yy, yz, zz) at site n from the phi field.
__device__ __forceinline__ void pi_of(const KParams& p, const Geo& n, const double* __restrict__ phi,
                                      double t[6])
{
    const Stencil st = stencil(phi[site_of(p, n.x, n.y, n.z)], phi[site_of(p, n.xp, n.y, n.z)],
                               phi[site_of(p, n.xm, n.y, n.z)], phi[site_of(p, n.x, n.yp, n.z)],
                               phi[site_of(p, n.x, n.ym, n.z)], phi[site_of(p, n.x, n.y, n.zp)],
                               phi[site_of(p, n.x, n.y, n.zm)]);
    double mu;
    chem_stress(p, st, &mu, t);
}

// F_a = -sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)] / 2 at site q (the terms of
// each component summed in the order b = x, y, z).
__device__ __forceinline__ void force_from_phi(const KParams& p, const Geo& q,
                                               const double* __restrict__ phi, double F[3])
{
    // component of Pi_ab in the xx, xy, xz, yy, yz, zz storage
    constexpr int K[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    double div[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < 3; b++) {
        const Geo np = geo_xyz(p, b == 0 ? q.xp : q.x, b == 1 ? q.yp : q.y, b == 2 ? q.zp : q.z);
        const Geo nm = geo_xyz(p, b == 0 ? q.xm : q.x, b == 1 ? q.ym : q.y, b == 2 ? q.zm : q.z);
        double tp[6], tm[6];
        pi_of(p, np, phi, tp);
        pi_of(p, nm, phi, tm);
#pragma unroll
        for (int a = 0; a < 3; a++) div[a] += 0.5 * (tp[K[a][b]] - tm[K[a][b]]);
    }
#pragma unroll
    for (int a = 0; a < 3; a++) F[a] = -div[a];
}

// Workgroup barrier for LDS traffic only: every wave's LDS writes have
// completed (lgkmcnt) before any wave passes.  Unlike __syncthreads() it
// does not first wait for the wave's outstanding global loads and stores,
// which the single-pass kernels keep in flight across the barrier (no
// global data written in a launch is read back in it).  The clobber keeps
// the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------
// Block reduction of K FP64 values (fixed order): wavefront butterfly, then
// the block's NB/64 waves as a pairwise tree.  Thread 0 writes component k to
// out[k*gridDim.x + blockIdx.x].  Needs blockDim.x == NB.
// Final reduction of `nblocks` block partials of `ncomp` (at most 5)
// components, laid out as block_partials writes them, by one workgroup of
// kBlock threads in a fixed order (strided per-thread sums, a wavefront
// butterfly, then the four waves pairwise): out[k] = sum, or out[k] += sum.
// Every thread of the workgroup must call it.
__device__ __forceinline__ void reduce_partials_block(const double* __restrict__ partials,
                                                      int nblocks, int ncomp,
                                                      double* __restrict__ out, bool accumulate)
{
    static_assert(kBlock == 256, "four waves");
    constexpr int KMAX = 5;
    __shared__ double sm[KMAX][kBlock / 64];
    double v[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; k++) {
        v[k] = 0.0;
        if (k < ncomp)
            for (int j = threadIdx.x; j < nblocks; j += kBlock) v[k] += partials[k * nblocks + j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < KMAX; k++) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < KMAX; k++) sm[k][threadIdx.x >> 6] = v[k];
    __syncthreads();
    if (threadIdx.x < ncomp) {
        const int k = threadIdx.x;
        const double t = (sm[k][0] + sm[k][1]) + (sm[k][2] + sm[k][3]);
        out[k] = accumulate ? out[k] + t : t;
    }
}

template <int K, int NB = kBlock>
__device__ __forceinline__ void block_partials(double (&v)[K], double* out)
{
    constexpr int NW = NB / 64;
    static_assert(NW >= 1 && (NW & (NW - 1)) == 0, "power-of-two wave count");
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < K; k++) v[k] += __shfl_xor(v[k], off, 64);
    __shared__ double sm[K][NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; k++) sm[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; k++) {
            double t[NW];
#pragma unroll
            for (int w = 0; w < NW; w++) t[w] = sm[k][w];
#pragma unroll
            for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
                for (int w = 0; w < h; w++) t[w] = t[2 * w] + t[2 * w + 1];
            out[k * gridDim.x + blockIdx.x] = t[0];
        }
}

}  // namespace dev
}  // namespace lbk
