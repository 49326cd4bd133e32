// Forward kernels (gfx950) of the D3Q19 symmetric binary-fluid LB step.
//
// The step of the paper's Ludwig timestep (Sec. 2.1.1) -- order-parameter
// gradients, chemical stress, collision, propagation -- runs as ONE kernel,
// k_step_fused_f32 / _f64: each workgroup owns a (y, z) tile of sites and marches
// along x over a segment of planes.  For plane x it needs phi at planes
// x-1, x, x+1 (7-point stencil); phi(x+1) is formed from the pulled g of
// plane x+1, which the same threads keep in registers for plane x+1's own
// collision one iteration later.  phi on the tile's (y, z) halo ring is
// formed by extra pulls that mostly hit in cache (the neighbouring tiles read
// the same lines).  phi planes live in a 4-slot LDS ring.  Every population
// is therefore read once and written once per step from HBM: the method's
// minimum traffic, instead of a separate phi pass plus a collision pass.
//
// k_phi + k_step_2s are the two-pass variant (phi kernel, then the fused
// stencil/collision/propagation kernel), kept for comparison.
#include <type_traits>

#include "lb_device.h"

namespace lbk {

using namespace dev;

namespace {

// Tile of the single-pass kernel: TZ contiguous z-sites per row (one
// wavefront row), TYB thread rows per 256-thread workgroup; a thread owns SY
// rows (SY = 2 in FP32 mode: twice the bytes in flight per workgroup and a
// halo ring of 28% instead of 53% of the tile).
constexpr int TZ = 64;
constexpr int TYB = kBlock / TZ;
#ifndef LB_SY32
#define LB_SY32 2
#endif
constexpr int SY32 = LB_SY32;
#ifndef LB_XCD_REMAP
#define LB_XCD_REMAP 1
#endif
#ifndef LB_ZFAST
#define LB_ZFAST 0
#endif
constexpr int SY64 = 1;



template <typename T>
struct Lvl {
    T* F;
    T* G;
    double* phic;  // FP32 mode only
};

template <typename T>
Lvl<T> level(void* state, const KParams& p, bool ref)
{
    T* base = static_cast<T*>(state);
    Lvl<T> l;
    l.F = base;
    l.G = base + size_t(NV) * p.stride;
    l.phic = ref ? reinterpret_cast<double*>(base + size_t(2 * NV) * p.stride) : nullptr;
    return l;
}

// ---------------------------------------------------------------------------

template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_init(KParams p, T* __restrict__ F, T* __restrict__ G,
                                                 double* __restrict__ phic,
                                                 const double* __restrict__ phi0)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const double ph = phi0[s];
#pragma unroll
    for (int i = 0; i < NV; i++) {
        F[i * p.stride + s] = DEV ? T(0) : T(weight(i) * p.rho0);
        const double gi = i == 0 ? ph : 0.0;
        G[i * p.stride + s] = REF ? T(gi - rweight(i) * ph) : T(gi);
    }
    if (REF) phic[s] = ph;
}

// phi(x) = sum_i g_i(x) of the post-propagation state (FP64).
template <typename T, bool REF>
__global__ __launch_bounds__(kBlock) void k_phi(KParams p, const T* __restrict__ G,
                                                const double* __restrict__ phic,
                                                double* __restrict__ phi)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    phi[s] = phi_at<T, REF>(p, geo_of(p, s), G, phic);
}

// Two-pass variant, second pass: stencil + chemical stress + collision, one
// site per thread; phi of the new state comes from k_phi.
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_step_2s(KParams p, const T* __restrict__ sF,
                                                    const T* __restrict__ sG,
                                                    const double* __restrict__ sphic,
                                                    const double* __restrict__ phi,
                                                    T* __restrict__ dF, T* __restrict__ dG)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    T f[NV], g[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) f[i] = sF[i * p.stride + pull_site(p, q, i)];
    double d[NV];
    const double pc = pull_g<T, REF>(p, q, sG, sphic, d);
    const Stencil st = stencil(pc, phi[site_of(p, q.xp, q.y, q.z)], phi[site_of(p, q.xm, q.y, q.z)],
                               phi[site_of(p, q.x, q.yp, q.z)], phi[site_of(p, q.x, q.ym, q.z)],
                               phi[site_of(p, q.x, q.y, q.zp)], phi[site_of(p, q.x, q.y, q.zm)]);
    g_local<T, REF>(d, pc, g);
    collide<T, DEV, REF>(p, f, g, st);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        dF[i * p.stride + s] = f[i];
        dG[i * p.stride + s] = g[i];
    }
}

// Wrap a coordinate v in [-2n, 3n) onto [0, n).
__device__ __forceinline__ int wrapg(int v, int n)
{
    if (v < 0) return v + n < 0 ? v + 2 * n : v + n;
    if (v >= n) return v - n >= n ? v - 2 * n : v - n;
    return v;
}

// Single-pass step (see the file comment).  Block -> (segment, tile) with
// an XCD-aware order: consecutive workgroup ids go round-robin over the 8
// XCDs, so ids are remapped to give each XCD a contiguous run of tiles,
// y-adjacent tiles first, whose halo rows then meet in the same L2.
//
// FP32 mode additionally stages the reference field phi_c of the source
// level in LDS, one plane per iteration with a 2-site (y, z) halo (the halo
// ring's own pulls reach 2 sites out), in a 6-slot ring: plane x+3 is
// prefetched while planes x-1..x+2 are in use.  Each pulled population then
// costs one FP32 global load; its reference term r_i phi_c(x - c_i) comes
// from LDS.
// Addressing: a thread's (y, z) never changes while it marches along x, so
// the 9 (y - cy, z - cz) byte offsets of its pulls are computed once; a plane
// and a component each contribute a uniform byte offset.  When a whole
// 19-component array is smaller than 4 GiB (SMALL) one 32-bit byte offset
// per load (component + plane + row) on a single base pointer suffices;
// larger lattices keep a uniform base pointer per component instead.
template <bool SMALL, typename T>
__device__ __forceinline__ T ldc(const T* __restrict__ base, unsigned stride, int i, unsigned off)
{
    if (SMALL) {
        const unsigned o = unsigned(i) * stride * unsigned(sizeof(T)) + off;
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + o);
    }
    const char* b = reinterpret_cast<const char*>(base + size_t(i) * stride);
    return *reinterpret_cast<const T*>(b + off);
}
template <bool SMALL, typename T>
__device__ __forceinline__ void stc(T* __restrict__ base, unsigned stride, int i, unsigned off, T v)
{
    if (SMALL) {
        const unsigned o = unsigned(i) * stride * unsigned(sizeof(T)) + off;
        *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + o) = v;
        return;
    }
    char* b = reinterpret_cast<char*>(base + size_t(i) * stride);
    *reinterpret_cast<T*>(b + off) = v;
}

// byte offsets of the 9 rows/columns (y + dy, z + dz), dy, dz in {-1, 0, 1}
struct Yz9 {
    unsigned o[3][3];
};
template <typename T>
__device__ __forceinline__ Yz9 yz9(const KParams& p, int y, int z)
{
    const int ys[3] = {wrapm(y, p.ny), y, wrapp(y, p.ny)};
    const int zs[3] = {wrapm(z, p.nz), z, wrapp(z, p.nz)};
    Yz9 r;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) r.o[a][c] = unsigned(ys[a] * p.nz + zs[c]) * unsigned(sizeof(T));
    return r;
}

template <typename T, bool DEV, bool REF, int SY, bool SMALL>
__device__ __forceinline__ void step_fused_body(const KParams& p, const TileCfg& tc,
                                                const T* __restrict__ sF,
                                                const T* __restrict__ sG,
                                                const double* __restrict__ sphic,
                                                T* __restrict__ dF, T* __restrict__ dG,
                                                double* __restrict__ dphic,
                                                double* __restrict__ partials)
{
    constexpr int TY = TYB * SY;  // site rows of the tile
    constexpr int PCS = REF ? 6 : 1, PCY = REF ? TY + 4 : 1, PCZ = REF ? TZ + 4 : 1;
    __shared__ double ph[4][TY + 2][TZ + 2];
    __shared__ double pc[PCS][PCY][PCZ];
    // value kept per direction between the phi pull and the collision:
    // the stored FP32 deviation (FP32 mode) or the FP64 population
    using K = typename std::conditional<REF, T, double>::type;
    const unsigned S = p.stride;

    int b = blockIdx.x;
    const int nb = gridDim.x;
    if (LB_XCD_REMAP && (nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tile = b % tc.ntiles, seg = b / tc.ntiles;
    const int y0 = (LB_ZFAST ? tile / tc.ntz : tile % tc.nty) * TY;
    const int z0 = (LB_ZFAST ? tile % tc.ntz : tile / tc.nty) * TZ;
    const int x0 = seg * tc.sx;
    const int x1 = min(x0 + tc.sx, p.nx);
    const int tya = min(TY, p.ny - y0), tza = min(TZ, p.nz - z0);
    const int lz = threadIdx.x % TZ, lyb = threadIdx.x / TZ;
    const int z = z0 + lz;
    const int plane = p.ny * p.nz;
    // this thread's rows: ly[k] = lyb + k*TYB
    int ly[SY];
    bool active[SY];
    Yz9 rows[SY];
#pragma unroll
    for (int k = 0; k < SY; k++) {
        ly[k] = lyb + k * TYB;
        active[k] = lz < tza && ly[k] < tya;
        rows[k] = yz9<T>(p, active[k] ? y0 + ly[k] : 0, active[k] ? z : 0);
    }

    // halo ring: rows y0-1 and y0+tya, then columns z0-1 and z0+tza
    const int r = threadIdx.x;
    const int nring = 2 * tza + 2 * tya;
    const bool ring = r < nring;
    int rly, rlz;
    if (r < tza) { rly = 0; rlz = r + 1; }
    else if (r < 2 * tza) { rly = tya + 1; rlz = r - tza + 1; }
    else if (r < 2 * tza + tya) { rly = r - 2 * tza + 1; rlz = 0; }
    else { rly = r - 2 * tza - tya + 1; rlz = tza + 1; }
    const int ry = wrapg(y0 + rly - 1, p.ny), rz = wrapg(z0 + rlz - 1, p.nz);
    const Yz9 rrow = yz9<T>(p, ry, rz);

    // plane indices run from x0-2 to x1+2 (nx may be 1): wrap without
    // division or branches (valid on [-2nx, 4nx))
    auto xw = [&](int X) {
        X += X < 0 ? p.nx : 0;
        X += X < 0 ? p.nx : 0;
        X -= X >= p.nx ? p.nx : 0;
        X -= X >= p.nx ? p.nx : 0;
        X -= X >= p.nx ? p.nx : 0;
        return X;
    };
    // byte base of plane X in a T array
    auto pbase = [&](int X) { return unsigned(xw(X) * plane) * unsigned(sizeof(T)); };

    // LDS slot of phi_c plane X is (X - x0 + 2) mod 6; `sl` below is the slot
    // of a site's own plane and sl +- 1 (mod 6) those of its neighbours
    auto add6 = [](int a, int d) {
        const int v = a + d;
        return v >= PCS ? v - PCS : (v < 0 ? v + PCS : v);
    };
    // phi_c plane X into LDS slot `slot`; cell (cy, cz) holds site
    // (y0 + cy - 2, z0 + cz - 2)
    auto load_pc = [&](int X, int slot) {
        if (REF) {
            const int W = tza + 4, n = W * (tya + 4);
            const int xx = xw(X);
            for (int t = threadIdx.x; t < n; t += kBlock) {
                const int cy = t / W, cz = t - cy * W;
                pc[REF ? slot : 0][REF ? cy : 0][REF ? cz : 0] =
                    sphic[site_of(p, xx, wrapg(y0 + cy - 2, p.ny), wrapg(z0 + cz - 2, p.nz))];
            }
        }
    };
    // g_i at a site as FP64, from the kept value kv of direction i; sl3 are the
    // slots of the planes X-1, X, X+1 and (cy, cz) the site's phi_c cell
    auto gval = [&](const int* sl3, int i, int cy, int cz, K kv) -> double {
        if (REF)
            return __builtin_fma(rweight(i),
                                 pc[REF ? sl3[1 - CX[i]] : 0][REF ? cy - CY[i] : 0][REF ? cz - CZ[i] : 0],
                                 double(kv));
        return double(kv);
    };
    // pull of plane X (slot sl) for a site with row offsets yz: kept values
    // into kv[] (if non-null), returns phi
    auto pull_phi = [&](int X, int sl, const Yz9& yz, int cy, int cz, K* kv) -> double {
        const unsigned pb[3] = {pbase(X - 1), pbase(X), pbase(X + 1)};
        const int sl3[3] = {add6(sl, -1), sl, add6(sl, 1)};
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const unsigned off = pb[1 - CX[i]] + yz.o[1 - CY[i]][1 - CZ[i]];
            const K v = K(ldc<SMALL>(sG, S, i, off));
            if (kv) kv[i] = v;
            acc += gval(sl3, i, cy, cz, v);
        }
        return acc;
    };

    K kcur[SY][NV], knext[SY][NV];
    // warm-up: phi_c planes x0-2 .. x0+2, then phi at planes x0-1 (slot 0)
    // and x0 (slot 1), keeping plane x0's populations
    for (int X = x0 - 2; X <= x0 + 2; X++) load_pc(X, X - x0 + 2);
    if (REF) __syncthreads();
#pragma unroll
    for (int k = 0; k < SY; k++)
        if (active[k])
            ph[0][ly[k] + 1][lz + 1] = pull_phi(x0 - 1, 1, rows[k], ly[k] + 2, lz + 2, nullptr);
    if (ring) ph[0][rly][rlz] = pull_phi(x0 - 1, 1, rrow, rly + 1, rlz + 1, nullptr);
#pragma unroll
    for (int k = 0; k < SY; k++)
        if (active[k])
            ph[1][ly[k] + 1][lz + 1] = pull_phi(x0, 2, rows[k], ly[k] + 2, lz + 2, kcur[k]);
    if (ring) ph[1][rly][rlz] = pull_phi(x0, 2, rrow, rly + 1, rlz + 1, nullptr);

    // conserved sums of the source level (FP64), if requested
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    int slx = 2;  // phi_c slot of plane x
    for (int x = x0; x < x1; x++, slx = add6(slx, 1)) {
        const int kk = x - x0 + 2;  // phi slot counter of plane x+1
        const int sn = kk & 3, sc = (kk - 1) & 3, sp = (kk - 2) & 3;
        const int slx3[3] = {add6(slx, -1), slx, add6(slx, 1)};
        load_pc(x + 3, add6(slx, 3));
        const unsigned pbx[3] = {pbase(x - 1), pbase(x), pbase(x + 1)};
        T f[SY][NV];
#pragma unroll
        for (int k = 0; k < SY; k++) {
            if (!active[k]) continue;
#pragma unroll
            for (int i = 0; i < NV; i++)
                f[k][i] = ldc<SMALL>(sF, S, i, pbx[1 - CX[i]] + rows[k].o[1 - CY[i]][1 - CZ[i]]);
        }
#pragma unroll
        for (int k = 0; k < SY; k++)
            if (active[k])
                ph[sn][ly[k] + 1][lz + 1] =
                    pull_phi(x + 1, slx3[2], rows[k], ly[k] + 2, lz + 2, knext[k]);
        if (ring) ph[sn][rly][rlz] = pull_phi(x + 1, slx3[2], rrow, rly + 1, rlz + 1, nullptr);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SY; k++) {
            if (!active[k]) continue;
            const int l = ly[k];
            const double c = ph[sc][l + 1][lz + 1];
            const Stencil st = stencil(c, ph[sn][l + 1][lz + 1], ph[sp][l + 1][lz + 1],
                                       ph[sc][l + 2][lz + 1], ph[sc][l][lz + 1],
                                       ph[sc][l + 1][lz + 2], ph[sc][l + 1][lz]);
            T g[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const double d = gval(slx3, i, l + 2, lz + 2, kcur[k][i]);
                g[i] = REF ? T(d - rweight(i) * c) : T(d);
            }
            if (partials) {
                // moments of the stored values, formed in FP64
                double bs = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
                for (int i = 0; i < NV; i++) {
                    const double v = double(f[k][i]);
                    bs += v;
                    if (CX[i]) jx += CX[i] * v;
                    if (CY[i]) jy += CY[i] * v;
                    if (CZ[i]) jz += CZ[i] * v;
                }
                acc[0] += DEV ? p.rho0 + bs : bs;
                acc[1] += c;
                acc[2] += jx;
                acc[3] += jy;
                acc[4] += jz;
            }
            collide<T, DEV, REF>(p, f[k], g, st);
            const unsigned so = pbx[1] + rows[k].o[1][1];
#pragma unroll
            for (int i = 0; i < NV; i++) {
                stc<SMALL>(dF, S, i, so, f[k][i]);
                stc<SMALL>(dG, S, i, so, g[i]);
            }
            if (REF) dphic[so / unsigned(sizeof(T))] = c;
#pragma unroll
            for (int i = 0; i < NV; i++) kcur[k][i] = knext[k][i];
        }
    }
    if (partials) block_partials<5>(acc, partials);
}

template <bool SMALL>
__global__ __launch_bounds__(kBlock) void k_step_fused_f32(
    KParams p, TileCfg tc, const float* __restrict__ sF, const float* __restrict__ sG,
    const double* __restrict__ sphic, float* __restrict__ dF, float* __restrict__ dG,
    double* __restrict__ dphic, double* __restrict__ partials)
{
    step_fused_body<float, true, true, SY32, SMALL>(p, tc, sF, sG, sphic, dF, dG, dphic, partials);
}

template <bool SMALL>
__global__ __launch_bounds__(kBlock) void k_step_fused_f64(
    KParams p, TileCfg tc, const double* __restrict__ sF, const double* __restrict__ sG,
    const double* __restrict__ sphic, double* __restrict__ dF, double* __restrict__ dG,
    double* __restrict__ dphic, double* __restrict__ partials)
{
    step_fused_body<double, false, false, SY64, SMALL>(p, tc, sF, sG, sphic, dF, dG, dphic,
                                                       partials);
}

template <typename T>
struct Fused;
template <>
struct Fused<float> {
    static constexpr auto small = k_step_fused_f32<true>;
    static constexpr auto large = k_step_fused_f32<false>;
};
template <>
struct Fused<double> {
    static constexpr auto small = k_step_fused_f64<true>;
    static constexpr auto large = k_step_fused_f64<false>;
};

// Dense FP64 moments of the post-propagation state and block partials of
// [rho, phi, jx, jy, jz] (grid-stride, FP64 accumulation).
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_moments(KParams p, const T* __restrict__ F,
                                                    const T* __restrict__ G,
                                                    const double* __restrict__ phic,
                                                    double* __restrict__ rho_out,
                                                    double* __restrict__ u_out,
                                                    double* __restrict__ phi_out,
                                                    double* __restrict__ partials)
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < p.nsites; s += gridDim.x * kBlock) {
        const Geo q = geo_of(p, s);
        double fv[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) fv[i] = double(F[i * p.stride + pull_site(p, q, i)]);
        const double ph = phi_at<T, REF>(p, q, G, phic);
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

// out[k] (+)= sum over nblocks partials of component k; one block, fixed order.
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

template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_export(KParams p, const T* __restrict__ F,
                                                   const T* __restrict__ G,
                                                   const double* __restrict__ phic,
                                                   double* __restrict__ f, double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    if (f)
#pragma unroll
        for (int i = 0; i < NV; i++)
            f[(long long)i * p.nsites + s] =
                double(F[i * p.stride + pull_site(p, q, i)]) + (DEV ? weight(i) * p.rho0 : 0.0);
    if (g) {
        double d[NV];
        pull_g<T, REF>(p, q, G, phic, d);
#pragma unroll
        for (int i = 0; i < NV; i++) g[(long long)i * p.nsites + s] = d[i];
    }
}

// Stored value at y is the post-propagation value at y + c_i.  In FP32 mode
// the reference phi_c(y) is the dense input's sum_i g_i(y).
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_import(KParams p, T* __restrict__ F, T* __restrict__ G,
                                                   double* __restrict__ phic,
                                                   const double* __restrict__ f,
                                                   const double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    double ref = 0.0;
    if (REF) {
#pragma unroll
        for (int i = 0; i < NV; i++) ref += g[(long long)i * p.nsites + s];
        phic[s] = ref;
    }
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const long long n = push_site(p, q, i) + (long long)i * p.nsites;
        F[i * p.stride + s] = T(f[n] - (DEV ? weight(i) * p.rho0 : 0.0));
        G[i * p.stride + s] = T(REF ? g[n] - rweight(i) * ref : g[n]);
    }
}

int grid_for(const KParams& p) { return (p.nsites + kBlock - 1) / kBlock; }

int reduction_grid(const KParams& p)
{
    const int g = grid_for(p);
    return g < kMaxPartialBlocks ? g : kMaxPartialBlocks;
}

// Instantiation dispatch: FP64 mode <double, false, false>, FP32 mode <float, true, true>.
#define LB_DISPATCH(fp32, CALL64, CALL32) \
    do {                                  \
        if (fp32) {                       \
            using T = float;              \
            constexpr bool DEV = true;    \
            constexpr bool REF = true;    \
            CALL32;                       \
        } else {                          \
            using T = double;             \
            constexpr bool DEV = false;   \
            constexpr bool REF = false;   \
            CALL64;                       \
        }                                 \
    } while (0)

// a 19-component array addressed with 32-bit byte offsets
bool small_arrays(const KParams& p, size_t elem)
{
    return size_t(NV) * p.stride * elem < (size_t(1) << 32);
}

}  // namespace

TileCfg tile_config(const KParams& p, int segment_x, bool fp32)
{
    const int ty = TYB * (fp32 ? SY32 : SY64);
    TileCfg tc;
    tc.nty = (p.ny + ty - 1) / ty;
    tc.ntz = (p.nz + TZ - 1) / TZ;
    tc.ntiles = tc.nty * tc.ntz;
    int sx = segment_x;
    if (sx <= 0) {
        // measured on MI355X at 256^3: the FP32 kernel wants ~2048 workgroups
        // (it is latency-bound and needs many in flight); the FP64 kernel
        // streams best with one workgroup per tile column (~256), i.e. the
        // fewest concurrent DRAM streams.  Segments of at least 8 planes.
        const long long target = fp32 ? 2048 : 256;
        const long long want = (long long)p.nx * tc.ntiles / target;
        sx = int(want < 8 ? 8 : want);
    }
    if (sx > p.nx) sx = p.nx;
    tc.sx = sx;
    tc.nseg = (p.nx + sx - 1) / sx;
    return tc;
}

hipError_t launch_init(const KParams& p, bool fp32, void* state, const double* phi0, hipStream_t s)
{
#define CALL                                                                                   \
    {                                                                                          \
        Lvl<T> l = level<T>(state, p, REF);                                                    \
        k_init<T, DEV, REF><<<grid_for(p), kBlock, 0, s>>>(p, l.F, l.G, l.phic, phi0);        \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_step(const KParams& p, const TileCfg& tc, bool fp32, int variant,
                       const void* src, void* dst, double* phi_work, double* partials,
                       double* sums_out, hipStream_t s)
{
    int nparts = 0;
#define CALL                                                                                    \
    {                                                                                           \
        Lvl<T> a = level<T>(const_cast<void*>(src), p, REF);                                    \
        Lvl<T> d = level<T>(dst, p, REF);                                                       \
        if (variant == 0) {                                                                     \
            nparts = tc.ntiles * tc.nseg;                                                       \
            auto kern = small_arrays(p, sizeof(T)) ? Fused<T>::small : Fused<T>::large;        \
            kern<<<nparts, kBlock, 0, s>>>(p, tc, a.F, a.G, a.phic, d.F, d.G, d.phic,           \
                                           sums_out ? partials : nullptr);                      \
        } else {                                                                                \
            if (sums_out) {                                                                     \
                nparts = reduction_grid(p);                                                     \
                k_moments<T, DEV, REF><<<nparts, kBlock, 0, s>>>(p, a.F, a.G, a.phic, nullptr,  \
                                                                 nullptr, nullptr, partials);   \
            }                                                                                   \
            double* phin = REF ? d.phic : phi_work;                                             \
            k_phi<T, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.G, a.phic, phin);                 \
            k_step_2s<T, DEV, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, phin,    \
                                                                  d.F, d.G);                    \
        }                                                                                       \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    if (sums_out) k_sums_final<<<1, kBlock, 0, s>>>(partials, nparts, 5, sums_out, 0);
    return hipGetLastError();
}

hipError_t launch_phi(const KParams& p, bool fp32, const void* state, double* phi, hipStream_t s)
{
#define CALL                                                                              \
    {                                                                                     \
        Lvl<T> a = level<T>(const_cast<void*>(state), p, REF);                            \
        k_phi<T, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.G, a.phic, phi);                \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_moments(const KParams& p, bool fp32, const void* state, double* rho, double* u,
                          double* phi, double* partials, int* nblocks_out, hipStream_t s)
{
    const int nb = reduction_grid(p);
    *nblocks_out = nb;
#define CALL                                                                                  \
    {                                                                                         \
        Lvl<T> a = level<T>(const_cast<void*>(state), p, REF);                                \
        k_moments<T, DEV, REF><<<nb, kBlock, 0, s>>>(p, a.F, a.G, a.phic, rho, u, phi,       \
                                                     partials);                               \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_sums_final(const double* partials, int nblocks, int ncomp, double* out,
                             bool accumulate, hipStream_t s)
{
    k_sums_final<<<1, kBlock, 0, s>>>(partials, nblocks, ncomp, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_export(const KParams& p, bool fp32, const void* state, double* f, double* g,
                         hipStream_t s)
{
#define CALL                                                                                  \
    {                                                                                         \
        Lvl<T> a = level<T>(const_cast<void*>(state), p, REF);                                \
        k_export<T, DEV, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, f, g);      \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_import(const KParams& p, bool fp32, void* state, const double* f,
                         const double* g, hipStream_t s)
{
#define CALL                                                                                  \
    {                                                                                         \
        Lvl<T> a = level<T>(state, p, REF);                                                   \
        k_import<T, DEV, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, f, g);      \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

}  // namespace lbk
