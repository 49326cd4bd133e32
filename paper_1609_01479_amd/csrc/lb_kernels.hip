// HIP kernels (gfx950) for the D3Q19 symmetric binary-fluid LB step and its
// adjoint.
//
// Storage (both precisions): a time level is f then g, each 19 components of
// `stride` elements (structure of arrays, the layout the paper finds best for
// GPUs, Sec. 4: coalesced access per component).  Component i of site s is
// element i*stride + s, with s = (x*ny + y)*nz + z.  A time level holds the
// post-collision, pre-propagation values f*_i(x); propagation is realised as
// a pull: the post-propagation value at x is f_i(x) = f*_i(x - c_i), read by
// the next kernel that needs it.  Periodic wrap is index arithmetic, so no
// halo copies exist.
//
// T = double: FP64 storage and arithmetic.  T = float with DEV = true: the
// FP32 deviation mode, where f is stored as f_i - w_i rho0 (g raw) and the
// collision works on deviations, so the O(1) rest part never enters FP32
// rounding; reductions stay FP64.
#include "lb_internal.h"

namespace lbk {
namespace {

constexpr int kBlock = 256;

// D3Q19 velocities: rest, +-x, +-y, +-z, 12 edges (same order as the ABI).
constexpr int CX[NV] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[NV] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[NV] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr double weight(int i)
{
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Site coordinates with periodic neighbours along each axis.
struct Geo {
    int x, y, z, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Geo geo_of(const KParams& p, int s)
{
    Geo q;
    q.z = s % p.nz;
    const int t = s / p.nz;
    q.y = t % p.ny;
    q.x = t / p.ny;
    q.xm = q.x == 0 ? p.nx - 1 : q.x - 1;
    q.xp = q.x == p.nx - 1 ? 0 : q.x + 1;
    q.ym = q.y == 0 ? p.ny - 1 : q.y - 1;
    q.yp = q.y == p.ny - 1 ? 0 : q.y + 1;
    q.zm = q.z == 0 ? p.nz - 1 : q.z - 1;
    q.zp = q.z == p.nz - 1 ? 0 : q.z + 1;
    return q;
}

__device__ __forceinline__ int site_of(const KParams& p, int x, int y, int z)
{
    return (x * p.ny + y) * p.nz + z;
}

// Coordinate v - c (pull source) and v + c (push destination) for c in {-1,0,1}.
__device__ __forceinline__ int minus_c(int c, int v, int vm, int vp) { return c > 0 ? vm : (c < 0 ? vp : v); }
__device__ __forceinline__ int plus_c(int c, int v, int vm, int vp) { return c > 0 ? vp : (c < 0 ? vm : v); }

// Site x - c_i and x + c_i.
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

// ---------------------------------------------------------------------------
// Local physics at one site.

// Order-parameter derivatives from the 7 stencil values.
template <typename T>
struct Stencil {
    T phi, gx, gy, gz, lap;
};

template <typename T>
__device__ __forceinline__ Stencil<T> stencil(T c, T xp, T xm, T yp, T ym, T zp, T zm)
{
    Stencil<T> s;
    s.phi = c;
    s.gx = T(0.5) * (xp - xm);
    s.gy = T(0.5) * (yp - ym);
    s.gz = T(0.5) * (zp - zm);
    s.lap = (xp + xm - T(2) * c) + (yp + ym - T(2) * c) + (zp + zm - T(2) * c);
    return s;
}

// Momentum moments of the 19 stored populations (raw, or deviations in DEV).
template <typename T>
struct Moments {
    T b;           // sum f (rho, or rho - rho0 in DEV)
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

// BGK collision of f and g in place.
//   mu = A phi + B phi^3 - kappa lap, Pi = iso I + kappa grad grad,
//   f_eq = w [b + 3 c.j + 9/2 Q:(Pi + j j / rho)],
//   g_eq = w [phi + 3 phi c.u + 9/2 (Gamma mu - phi/3)(|c|^2 - 1)
//             + 9/2 phi ((c.u)^2 - |u|^2/3)].
template <typename T, bool DEV>
__device__ __forceinline__ void collide(const KParams& p, T* f, T* g, const Stencil<T>& st)
{
    const T A = T(p.A), B = T(p.B), kap = T(p.kappa), gam = T(p.gamma);
    const T omf = T(p.omega_f), omg = T(p.omega_g);
    const T phi = st.phi, gx = st.gx, gy = st.gy, gz = st.gz, lap = st.lap;
    const T phi2 = phi * phi;
    const T mu = A * phi + B * phi2 * phi - kap * lap;
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

    const T sg = gam * mu - phi * T(1.0 / 3.0);
    const T uu3 = (ux * ux + uy * uy + uz * uz) * T(1.0 / 3.0);
    const T hp = h * phi;
    eq[0] = w0 * (phi - h * sg - hp * uu3);
    {
        const T p3f = wf3 * phi;
        const T sx = wf * (phi + hp * (ux * ux - uu3));
        const T sy = wf * (phi + hp * (uy * uy - uu3));
        const T sz = wf * (phi + hp * (uz * uz - uu3));
        eq[1] = sx + p3f * ux; eq[2] = sx - p3f * ux;
        eq[3] = sy + p3f * uy; eq[4] = sy - p3f * uy;
        eq[5] = sz + p3f * uz; eq[6] = sz - p3f * uz;
    }
    {
        const T p3e = we3 * phi;
        const T base = phi + h * sg - hp * uu3;
        const T c7 = ux + uy, c9 = ux - uy, c11 = ux + uz, c13 = ux - uz, c15 = uy + uz,
                c17 = uy - uz;
        const T s7 = we * (base + hp * c7 * c7), s9 = we * (base + hp * c9 * c9);
        const T s11 = we * (base + hp * c11 * c11), s13 = we * (base + hp * c13 * c13);
        const T s15 = we * (base + hp * c15 * c15), s17 = we * (base + hp * c17 * c17);
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

// ---------------------------------------------------------------------------
// Block reduction of K FP64 values: wavefront butterfly (fixed order), then
// the 4 wave results in a fixed order.  Thread 0 writes component k of this
// block to out[k*nblocks + blockIdx.x].
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* out)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < K; k++) v[k] += __shfl_xor(v[k], off, 64);
    __shared__ double sm[K][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; k++) sm[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; k++)
            out[k * gridDim.x + blockIdx.x] = (sm[k][0] + sm[k][1]) + (sm[k][2] + sm[k][3]);
}

// ---------------------------------------------------------------------------
// Forward kernels.

template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_init(KParams p, T* __restrict__ f, T* __restrict__ g,
                                                 const double* __restrict__ phi0)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        f[i * p.stride + s] = DEV ? T(0) : T(weight(i) * p.rho0);
        g[i * p.stride + s] = i == 0 ? T(phi0[s]) : T(0);
    }
}

// phi(x) = sum_i g_i(x) of the post-propagation state, i.e. sum_i g*_i(x - c_i).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_phi(KParams p, const T* __restrict__ g,
                                                T* __restrict__ phi)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    T acc = T(0);
#pragma unroll
    for (int i = 0; i < NV; i++) acc += g[i * p.stride + pull_site(p, q, i)];
    phi[s] = acc;
}

// Gradients + chemical stress + collision + propagation (as the pull of the
// next step) for one site per thread.
template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_step(KParams p, const T* __restrict__ sf,
                                                 const T* __restrict__ sg,
                                                 const T* __restrict__ phi,
                                                 T* __restrict__ df, T* __restrict__ dg)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    const Stencil<T> st = stencil<T>(phi[s], phi[site_of(p, q.xp, q.y, q.z)],
                                     phi[site_of(p, q.xm, q.y, q.z)],
                                     phi[site_of(p, q.x, q.yp, q.z)],
                                     phi[site_of(p, q.x, q.ym, q.z)],
                                     phi[site_of(p, q.x, q.y, q.zp)],
                                     phi[site_of(p, q.x, q.y, q.zm)]);
    T f[NV], g[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const int n = pull_site(p, q, i);
        f[i] = sf[i * p.stride + n];
        g[i] = sg[i * p.stride + n];
    }
    collide<T, DEV>(p, f, g, st);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        df[i * p.stride + s] = f[i];
        dg[i * p.stride + s] = g[i];
    }
}

// Dense FP64 moments of the post-propagation state and block partials of
// [rho, phi, jx, jy, jz] (grid-stride; FP64 accumulation).
template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_moments(KParams p, const T* __restrict__ f,
                                                    const T* __restrict__ g,
                                                    double* __restrict__ rho_out,
                                                    double* __restrict__ u_out,
                                                    double* __restrict__ phi_out,
                                                    double* __restrict__ partials)
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < p.nsites; s += gridDim.x * kBlock) {
        const Geo q = geo_of(p, s);
        double fv[NV], ph = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const int n = pull_site(p, q, i);
            fv[i] = double(f[i * p.stride + n]);
            ph += double(g[i * p.stride + n]);
        }
        double b = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) b += fv[i];
        const double rho = DEV ? p.rho0 + b : b;
        double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            jx += CX[i] * fv[i];
            jy += CY[i] * fv[i];
            jz += CZ[i] * fv[i];
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

// out[k] (+)= sum over nblocks partials of component k, one block, fixed order.
__global__ __launch_bounds__(kBlock) void k_sums_final(const double* __restrict__ partials,
                                                       int nblocks, int ncomp,
                                                       double* __restrict__ out, int accumulate)
{
    __shared__ double sm[kBlock];
    for (int k = 0; k < ncomp; k++) {
        double v = 0.0;
        for (int j = threadIdx.x; j < nblocks; j += kBlock) v += partials[k * nblocks + j];
        sm[threadIdx.x] = v;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = accumulate ? out[k] + sm[0] : sm[0];
        __syncthreads();
    }
}

template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_export(KParams p, const T* __restrict__ sf,
                                                   const T* __restrict__ sg,
                                                   double* __restrict__ f,
                                                   double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const int n = pull_site(p, q, i);
        if (f) f[(long long)i * p.nsites + s] = double(sf[i * p.stride + n]) + (DEV ? weight(i) * p.rho0 : 0.0);
        if (g) g[(long long)i * p.nsites + s] = double(sg[i * p.stride + n]);
    }
}

// Stored (pre-propagation) value at y is the post-propagation value at y + c_i.
template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_import(KParams p, T* __restrict__ sf, T* __restrict__ sg,
                                                   const double* __restrict__ f,
                                                   const double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const long long n = push_site(p, q, i) + (long long)i * p.nsites;
        sf[i * p.stride + s] = T(f[n] - (DEV ? weight(i) * p.rho0 : 0.0));
        sg[i * p.stride + s] = T(g[n]);
    }
}

// ---------------------------------------------------------------------------
// Reverse mode.
//
// An adjoint time level holds 39 components of `stride` elements:
//   lf[19]: dL/df_i(x)            (post-propagation populations)
//   lg[19]: the part of dL/dg_i(x) that is not common to all i
//   lp    : the common part, dL/dphi(x)
// so that dL/dg_i(x) = lg_i(x) + lp(x).  adj_scratch holds the stencil
// cotangents a (direct dL/dphi), b_a (dL/d(d_a phi)), c (dL/d lap phi).

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_seed(KParams p, T* __restrict__ adj,
                                                     const double* __restrict__ dphi)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
#pragma unroll
    for (int i = 0; i < 2 * NV; i++) adj[i * p.stride + s] = T(0);
    adj[2 * NV * p.stride + s] = T(dphi[s]);
}

// Transposed propagation (gather lambda*_i(x) = lambda_i(x + c_i)), then the
// transposed local collision Jacobian at x, recomputing the forward locals
// from the saved state.  Writes lf, lg of the previous level and the stencil
// cotangents; block partials of d/d(A, B, kappa).
template <typename T, bool DEV>
__global__ __launch_bounds__(kBlock) void k_adj_local(KParams p, const T* __restrict__ sf,
                                                      const T* __restrict__ sg,
                                                      const T* __restrict__ phi,
                                                      const T* __restrict__ an,
                                                      T* __restrict__ ap,
                                                      T* __restrict__ sc,
                                                      double* __restrict__ partials)
{
    double dth[3] = {0.0, 0.0, 0.0};
    const long long S = p.stride;
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < p.nsites; s += gridDim.x * kBlock) {
        const Geo q = geo_of(p, s);
        T lf[NV], lg[NV], f[NV], g[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const int d = push_site(p, q, i);
            lf[i] = an[i * S + d];
            lg[i] = an[(NV + i) * S + d] + an[2 * NV * S + d];
            const int n = pull_site(p, q, i);
            f[i] = sf[i * S + n];
            g[i] = sg[i * S + n];
        }
        (void)g;
        const Stencil<T> st = stencil<T>(phi[s], phi[site_of(p, q.xp, q.y, q.z)],
                                         phi[site_of(p, q.xm, q.y, q.z)],
                                         phi[site_of(p, q.x, q.yp, q.z)],
                                         phi[site_of(p, q.x, q.ym, q.z)],
                                         phi[site_of(p, q.x, q.y, q.zp)],
                                         phi[site_of(p, q.x, q.y, q.zm)]);
        const T A = T(p.A), B = T(p.B), kap = T(p.kappa), gam = T(p.gamma);
        const T omf = T(p.omega_f), omg = T(p.omega_g);
        const Moments<T> m = moments_of<T, DEV>(p, f);
        const T rho = m.rho, ri = T(1) / rho;
        const T ux = m.jx * ri, uy = m.jy * ri, uz = m.jz * ri;
        const T phi_c = st.phi, gx = st.gx, gy = st.gy, gz = st.gz, lap = st.lap;

        // Weighted moments of Lambda = omega * lambda*:
        //   S0 = sum w L, S1 = sum w L c, S2 = sum w L (c c - I/3)  (f part)
        //   T0, T1, T2 likewise for the g part.
        T s0 = 0, s1x = 0, s1y = 0, s1z = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
        T t0 = 0, t1x = 0, t1y = 0, t1z = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const T wl = T(weight(i)) * omf * lf[i];
            const T wg = T(weight(i)) * omg * lg[i];
            s0 += wl; t0 += wg;
            if (CX[i]) { s1x += CX[i] * wl; t1x += CX[i] * wg; }
            if (CY[i]) { s1y += CY[i] * wl; t1y += CY[i] * wg; }
            if (CZ[i]) { s1z += CZ[i] * wl; t1z += CZ[i] * wg; }
            if (CX[i]) { sxx += wl; txx += wg; }
            if (CY[i]) { syy += wl; tyy += wg; }
            if (CZ[i]) { szz += wl; tzz += wg; }
            if (CX[i] * CY[i]) { sxy += CX[i] * CY[i] * wl; txy += CX[i] * CY[i] * wg; }
            if (CX[i] * CZ[i]) { sxz += CX[i] * CZ[i] * wl; txz += CX[i] * CZ[i] * wg; }
            if (CY[i] * CZ[i]) { syz += CY[i] * CZ[i] * wl; tyz += CY[i] * CZ[i] * wg; }
        }
        const T third = T(1.0 / 3.0);
        sxx -= third * s0; syy -= third * s0; szz -= third * s0;
        txx -= third * t0; tyy -= third * t0; tzz -= third * t0;
        const T trs = sxx + syy + szz, trt = txx + tyy + tzz;
        // S2.u, T2.u, S2:uu, T2:uu, S2.grad, grad.S2.grad
        const T s2ux = sxx * ux + sxy * uy + sxz * uz;
        const T s2uy = sxy * ux + syy * uy + syz * uz;
        const T s2uz = sxz * ux + syz * uy + szz * uz;
        const T t2ux = txx * ux + txy * uy + txz * uz;
        const T t2uy = txy * ux + tyy * uy + tyz * uz;
        const T t2uz = txz * ux + tyz * uy + tzz * uz;
        const T s2uu = s2ux * ux + s2uy * uy + s2uz * uz;
        const T t2uu = t2ux * ux + t2uy * uy + t2uz * uz;
        const T t1u = t1x * ux + t1y * uy + t1z * uz;
        const T s2gx = sxx * gx + sxy * gy + sxz * gz;
        const T s2gy = sxy * gx + syy * gy + syz * gz;
        const T s2gz = sxz * gx + syz * gy + szz * gz;
        const T gsg = s2gx * gx + s2gy * gy + s2gz * gz;
        const T h = T(4.5);
        const T pr = phi_c * ri;

        // d/d rho and d/d j of sum Lambda_f f_eq + Lambda_g g_eq
        const T arho = s0 - h * s2uu - T(3) * pr * t1u - T(9) * pr * t2uu;
        const T ajx = T(3) * s1x + T(9) * s2ux + T(3) * pr * t1x + T(9) * pr * t2ux;
        const T ajy = T(3) * s1y + T(9) * s2uy + T(3) * pr * t1y + T(9) * pr * t2uy;
        const T ajz = T(3) * s1z + T(9) * s2uz + T(3) * pr * t1z + T(9) * pr * t2uz;
        const T cf = T(1) - omf, cg = T(1) - omg;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            T v = cf * lf[i] + arho;
            if (CX[i]) v += CX[i] * ajx;
            if (CY[i]) v += CY[i] * ajy;
            if (CZ[i]) v += CZ[i] * ajz;
            ap[i * S + s] = v;
            ap[(NV + i) * S + s] = cg * lg[i];
        }
        // stencil cotangents
        const T phi2 = phi_c * phi_c;
        const T a_dir = h * trs * (A * phi_c + T(3) * B * phi2 * phi_c - kap * lap) + t0
                      + T(3) * t1u + h * (gam * (A + T(3) * B * phi2) - third) * trt + h * t2uu;
        const T hk = h * kap;
        sc[0 * S + s] = a_dir;
        sc[1 * S + s] = hk * (T(2) * s2gx - trs * gx);
        sc[2 * S + s] = hk * (T(2) * s2gy - trs * gy);
        sc[3 * S + s] = hk * (T(2) * s2gz - trs * gz);
        sc[4 * S + s] = -hk * (phi_c * trs + gam * trt);
        // parameter cotangents (FP64 accumulation)
        const double g2 = double(gx) * gx + double(gy) * gy + double(gz) * gz;
        const double dtrs = double(trs), dtrt = double(trt), dph = double(phi_c);
        dth[0] += 4.5 * (dtrs * 0.5 * dph * dph + p.gamma * dph * dtrt);
        dth[1] += 4.5 * (dtrs * 0.75 * dph * dph * dph * dph + p.gamma * dph * dph * dph * dtrt);
        dth[2] += 4.5 * (dtrs * (-dph * double(lap) - 0.5 * g2) + double(gsg)
                         - p.gamma * double(lap) * dtrt);
    }
    block_partials<3>(dth, partials);
}

// lp(x) = a(x) - sum_a D_a b_a (x) + lap c (x): the transposed stencil
// (D_a^T = -D_a, lap^T = lap on the periodic lattice).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_stencil(KParams p, const T* __restrict__ sc,
                                                        T* __restrict__ ap)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    const long long S = p.stride;
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
__global__ __launch_bounds__(kBlock) void k_adj_phi0(KParams p, const T* __restrict__ adj,
                                                     double* __restrict__ out)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    out[s] = double(adj[NV * p.stride + s]) + double(adj[2 * NV * p.stride + s]);
}

int grid_for(const KParams& p) { return (p.nsites + kBlock - 1) / kBlock; }

int reduction_grid(const KParams& p)
{
    const int g = grid_for(p);
    return g < kMaxPartialBlocks ? g : kMaxPartialBlocks;
}

template <typename T>
T* fpart(void* state) { return static_cast<T*>(state); }
template <typename T>
T* gpart(void* state, const KParams& p) { return static_cast<T*>(state) + NV * p.stride; }
template <typename T>
const T* fpart(const void* state) { return static_cast<const T*>(state); }
template <typename T>
const T* gpart(const void* state, const KParams& p) { return static_cast<const T*>(state) + NV * p.stride; }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

hipError_t launch_init(const KParams& p, bool fp32, void* state, const double* phi0, hipStream_t s)
{
    if (fp32)
        k_init<float, true><<<grid_for(p), kBlock, 0, s>>>(p, fpart<float>(state), gpart<float>(state, p), phi0);
    else
        k_init<double, false><<<grid_for(p), kBlock, 0, s>>>(p, fpart<double>(state), gpart<double>(state, p), phi0);
    return hipGetLastError();
}

hipError_t launch_step(const KParams& p, bool fp32, const void* src, void* dst, void* phi, hipStream_t s)
{
    if (fp32) {
        k_phi<float><<<grid_for(p), kBlock, 0, s>>>(p, gpart<float>(src, p), static_cast<float*>(phi));
        k_step<float, true><<<grid_for(p), kBlock, 0, s>>>(p, fpart<float>(src), gpart<float>(src, p),
                                                           static_cast<const float*>(phi),
                                                           fpart<float>(dst), gpart<float>(dst, p));
    } else {
        k_phi<double><<<grid_for(p), kBlock, 0, s>>>(p, gpart<double>(src, p), static_cast<double*>(phi));
        k_step<double, false><<<grid_for(p), kBlock, 0, s>>>(p, fpart<double>(src), gpart<double>(src, p),
                                                             static_cast<const double*>(phi),
                                                             fpart<double>(dst), gpart<double>(dst, p));
    }
    return hipGetLastError();
}

hipError_t launch_moments(const KParams& p, bool fp32, const void* state, double* rho, double* u,
                          double* phi, double* partials, int* nblocks_out, hipStream_t s)
{
    const int nb = reduction_grid(p);
    *nblocks_out = nb;
    if (fp32)
        k_moments<float, true><<<nb, kBlock, 0, s>>>(p, fpart<float>(state), gpart<float>(state, p), rho, u, phi, partials);
    else
        k_moments<double, false><<<nb, kBlock, 0, s>>>(p, fpart<double>(state), gpart<double>(state, p), rho, u, phi, partials);
    return hipGetLastError();
}

hipError_t launch_sums_final(const double* partials, int nblocks, int ncomp, double* out,
                             bool accumulate, hipStream_t s)
{
    k_sums_final<<<1, kBlock, 0, s>>>(partials, nblocks, ncomp, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_export(const KParams& p, bool fp32, const void* state, double* f, double* g, hipStream_t s)
{
    if (fp32)
        k_export<float, true><<<grid_for(p), kBlock, 0, s>>>(p, fpart<float>(state), gpart<float>(state, p), f, g);
    else
        k_export<double, false><<<grid_for(p), kBlock, 0, s>>>(p, fpart<double>(state), gpart<double>(state, p), f, g);
    return hipGetLastError();
}

hipError_t launch_import(const KParams& p, bool fp32, void* state, const double* f, const double* g,
                         hipStream_t s)
{
    if (fp32)
        k_import<float, true><<<grid_for(p), kBlock, 0, s>>>(p, fpart<float>(state), gpart<float>(state, p), f, g);
    else
        k_import<double, false><<<grid_for(p), kBlock, 0, s>>>(p, fpart<double>(state), gpart<double>(state, p), f, g);
    return hipGetLastError();
}

hipError_t launch_adj_seed(const KParams& p, bool fp32, void* adj, const double* dphi, hipStream_t s)
{
    if (fp32)
        k_adj_seed<float><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<float*>(adj), dphi);
    else
        k_adj_seed<double><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<double*>(adj), dphi);
    return hipGetLastError();
}

hipError_t launch_adj_step(const KParams& p, bool fp32, const void* state, void* phi,
                           const void* adj_next, void* adj_prev, void* adj_scratch,
                           double* partials, int* nblocks_out, hipStream_t s)
{
    const int nb = reduction_grid(p);
    *nblocks_out = nb;
    if (fp32) {
        k_phi<float><<<grid_for(p), kBlock, 0, s>>>(p, gpart<float>(state, p), static_cast<float*>(phi));
        k_adj_local<float, true><<<nb, kBlock, 0, s>>>(p, fpart<float>(state), gpart<float>(state, p),
                                                       static_cast<const float*>(phi),
                                                       static_cast<const float*>(adj_next),
                                                       static_cast<float*>(adj_prev),
                                                       static_cast<float*>(adj_scratch), partials);
        k_adj_stencil<float><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const float*>(adj_scratch),
                                                            static_cast<float*>(adj_prev));
    } else {
        k_phi<double><<<grid_for(p), kBlock, 0, s>>>(p, gpart<double>(state, p), static_cast<double*>(phi));
        k_adj_local<double, false><<<nb, kBlock, 0, s>>>(p, fpart<double>(state), gpart<double>(state, p),
                                                         static_cast<const double*>(phi),
                                                         static_cast<const double*>(adj_next),
                                                         static_cast<double*>(adj_prev),
                                                         static_cast<double*>(adj_scratch), partials);
        k_adj_stencil<double><<<grid_for(p), kBlock, 0, s>>>(p, static_cast<const double*>(adj_scratch),
                                                             static_cast<double*>(adj_prev));
    }
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

}  // namespace lbk
