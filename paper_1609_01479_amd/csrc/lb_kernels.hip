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

// Tuning knobs of the single-pass kernel (compile-time; defaults are the
// measured best on MI355X).
#ifndef LB_TZ
#define LB_TZ 64  // tile extent along z (contiguous)
#endif
#ifndef LB_RING_SPREAD
#define LB_RING_SPREAD 0  // 1: spread halo-ring sites evenly over the waves
#endif
#ifndef LB_PREFETCH_F
#define LB_PREFETCH_F 0  // 1: load plane x+1's f while plane x is stored
#endif
#ifndef LB_NT_STORE
#define LB_NT_STORE 0  // 1: nontemporal stores of the new time level
#endif
#ifndef LB_WPE32
#define LB_WPE32 0  // >0: waves-per-EU hint for the FP32 instantiation
#endif
#ifndef LB_RELOAD_G
#define LB_RELOAD_G 0  // 1: re-read plane x's g (an L2 hit) instead of keeping it
#endif
#ifndef LB_WPE64
#define LB_WPE64 0  // >0: waves-per-EU hint for the FP64 instantiation
#endif

constexpr int TZ = LB_TZ;
constexpr int TY = kBlock / TZ;

template <typename T>
__device__ __forceinline__ void store_out(T* ptr, T v)
{
    if (LB_NT_STORE) __builtin_nontemporal_store(v, ptr);
    else *ptr = v;
}

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
    l.G = base + NV * p.stride;
    l.phic = ref ? reinterpret_cast<double*>(base + 2 * NV * p.stride) : nullptr;
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
template <typename T, bool DEV, bool REF>
__device__ __forceinline__ void step_fused_body(const KParams& p, const TileCfg& tc,
                                                const T* __restrict__ sF,
                                                const T* __restrict__ sG,
                                                const double* __restrict__ sphic,
                                                T* __restrict__ dF, T* __restrict__ dG,
                                                double* __restrict__ dphic,
                                                double* __restrict__ partials)
{
    constexpr int PCS = REF ? 6 : 1, PCY = REF ? TY + 4 : 1, PCZ = REF ? TZ + 4 : 1;
    __shared__ double ph[4][TY + 2][TZ + 2];
    __shared__ double pc[PCS][PCY][PCZ];
    // value kept per direction between the phi pull and the collision:
    // the stored FP32 deviation (FP32 mode) or the FP64 population
    using K = typename std::conditional<REF, T, double>::type;

    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tile = b % tc.ntiles, seg = b / tc.ntiles;
    const int y0 = (tile % tc.nty) * TY, z0 = (tile / tc.nty) * TZ;
    const int x0 = seg * tc.sx;
    const int x1 = min(x0 + tc.sx, p.nx);
    const int tya = min(TY, p.ny - y0), tza = min(TZ, p.nz - z0);
    const int lz = threadIdx.x % TZ, ly = threadIdx.x / TZ;
    const bool active = lz < tza && ly < tya;
    const int y = y0 + ly, z = z0 + lz;

    // halo ring: rows y0-1 and y0+tya, then columns z0-1 and z0+tza
    const int r = LB_RING_SPREAD ? (threadIdx.x & 63) * (kBlock / 64) + (threadIdx.x >> 6)
                                 : int(threadIdx.x);
    const int nring = 2 * tza + 2 * tya;
    const bool ring = r < nring;
    int rly, rlz;
    if (r < tza) { rly = 0; rlz = r + 1; }
    else if (r < 2 * tza) { rly = tya + 1; rlz = r - tza + 1; }
    else if (r < 2 * tza + tya) { rly = r - 2 * tza + 1; rlz = 0; }
    else { rly = r - 2 * tza - tya + 1; rlz = tza + 1; }
    const int ry = wrapg(y0 + rly - 1, p.ny), rz = wrapg(z0 + rlz - 1, p.nz);

    // plane indices run from x0-2 to x1+2: wrap them with a full modulo (nx may be 1)
    auto xw = [&](int X) { return ((X % p.nx) + p.nx) % p.nx; };
    // phi_c plane X (logical index X - x0 + 2) into its LDS slot; cell
    // (cy, cz) holds site (y0 + cy - 2, z0 + cz - 2)
    auto load_pc = [&](int X) {
        if (REF) {
            const int slot = (X - x0 + 2) % PCS;
            const int W = tza + 4, n = W * (tya + 4);
            const int xx = xw(X);
            for (int t = threadIdx.x; t < n; t += kBlock) {
                const int cy = t / W, cz = t - cy * W;
                pc[slot % PCS][REF ? cy : 0][REF ? cz : 0] =
                    sphic[site_of(p, xx, wrapg(y0 + cy - 2, p.ny), wrapg(z0 + cz - 2, p.nz))];
            }
        }
    };
    // g_i at a site of plane X as FP64, from the kept value kv of direction i;
    // (cy, cz) is the site's phi_c cell
    auto gval = [&](int X, int i, int cy, int cz, K kv) -> double {
        if (REF) {
            const int slot = (X - CX[i] - x0 + 2) % PCS;
            return __builtin_fma(rweight(i), pc[slot % PCS][REF ? cy - CY[i] : 0][REF ? cz - CZ[i] : 0],
                                 double(kv));
        }
        return double(kv);
    };
    // pull of plane X at (yy, zz): kept values into kv[] (if non-null), returns phi
    auto pull_phi = [&](int X, int yy, int zz, int cy, int cz, K* kv) -> double {
        const Geo q = geo_xyz(p, xw(X), yy, zz);
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const K v = K(sG[i * p.stride + pull_site(p, q, i)]);
            if (kv) kv[i] = v;
            acc += gval(X, i, cy, cz, v);
        }
        return acc;
    };

    K kcur[NV], knext[NV];
    // warm-up: phi_c planes x0-2 .. x0+2, then phi at planes x0-1 (slot 0)
    // and x0 (slot 1), keeping plane x0's populations
    for (int X = x0 - 2; X <= x0 + 2; X++) load_pc(X);
    if (REF) __syncthreads();
    if (active) ph[0][ly + 1][lz + 1] = pull_phi(x0 - 1, y, z, ly + 2, lz + 2, nullptr);
    if (ring) ph[0][rly][rlz] = pull_phi(x0 - 1, ry, rz, rly + 1, rlz + 1, nullptr);
    if (active) ph[1][ly + 1][lz + 1] = pull_phi(x0, y, z, ly + 2, lz + 2, kcur);
    if (ring) ph[1][rly][rlz] = pull_phi(x0, ry, rz, rly + 1, rlz + 1, nullptr);

    // conserved sums of the source level (FP64), if requested
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    T f[NV];
    auto load_f = [&](int X) {
        const Geo qc = geo_xyz(p, X, y, z);
#pragma unroll
        for (int i = 0; i < NV; i++) f[i] = sF[i * p.stride + pull_site(p, qc, i)];
    };
    if (LB_PREFETCH_F && active) load_f(x0);

    for (int x = x0; x < x1; x++) {
        const int k = x - x0 + 2;  // phi slot counter of plane x+1
        const int sn = k & 3, sc = (k - 1) & 3, sp = (k - 2) & 3;
        load_pc(x + 3);
        if (active) {
            if (!LB_PREFETCH_F) load_f(x);
            if (LB_RELOAD_G) {
                const Geo qc = geo_xyz(p, x, y, z);
#pragma unroll
                for (int i = 0; i < NV; i++) kcur[i] = K(sG[i * p.stride + pull_site(p, qc, i)]);
            }
            ph[sn][ly + 1][lz + 1] = pull_phi(x + 1, y, z, ly + 2, lz + 2, LB_RELOAD_G ? nullptr : knext);
        }
        if (ring) ph[sn][rly][rlz] = pull_phi(x + 1, ry, rz, rly + 1, rlz + 1, nullptr);
        __syncthreads();
        if (active) {
            const double c = ph[sc][ly + 1][lz + 1];
            const Stencil st = stencil(c, ph[sn][ly + 1][lz + 1], ph[sp][ly + 1][lz + 1],
                                       ph[sc][ly + 2][lz + 1], ph[sc][ly][lz + 1],
                                       ph[sc][ly + 1][lz + 2], ph[sc][ly + 1][lz]);
            T g[NV];
#pragma unroll
            for (int i = 0; i < NV; i++) {
                const double d = gval(x, i, ly + 2, lz + 2, kcur[i]);
                g[i] = REF ? T(d - rweight(i) * c) : T(d);
            }
            if (partials) {
                const Moments<T> m = moments_of<T, DEV>(p, f);
                acc[0] += DEV ? p.rho0 + double(m.b) : double(m.rho);
                acc[1] += c;
                acc[2] += double(m.jx);
                acc[3] += double(m.jy);
                acc[4] += double(m.jz);
            }
            collide<T, DEV, REF>(p, f, g, st);
            const int s = site_of(p, x, y, z);
#pragma unroll
            for (int i = 0; i < NV; i++) {
                store_out(dF + i * p.stride + s, f[i]);
                store_out(dG + i * p.stride + s, g[i]);
            }
            if (REF) store_out(dphic + s, c);
            if (!LB_RELOAD_G)
#pragma unroll
                for (int i = 0; i < NV; i++) kcur[i] = knext[i];
            if (LB_PREFETCH_F && x + 1 < x1) load_f(x + 1);
        }
    }
    if (partials) block_partials<5>(acc, partials);
}

#if LB_WPE32 > 0
#define LB_ATTR32 __attribute__((amdgpu_waves_per_eu(LB_WPE32)))
#else
#define LB_ATTR32
#endif
#if LB_WPE64 > 0
#define LB_ATTR64 __attribute__((amdgpu_waves_per_eu(LB_WPE64)))
#else
#define LB_ATTR64
#endif

__global__ __launch_bounds__(kBlock) LB_ATTR32 void k_step_fused_f32(
    KParams p, TileCfg tc, const float* __restrict__ sF, const float* __restrict__ sG,
    const double* __restrict__ sphic, float* __restrict__ dF, float* __restrict__ dG,
    double* __restrict__ dphic, double* __restrict__ partials)
{
    step_fused_body<float, true, true>(p, tc, sF, sG, sphic, dF, dG, dphic, partials);
}

__global__ __launch_bounds__(kBlock) LB_ATTR64 void k_step_fused_f64(
    KParams p, TileCfg tc, const double* __restrict__ sF, const double* __restrict__ sG,
    const double* __restrict__ sphic, double* __restrict__ dF, double* __restrict__ dG,
    double* __restrict__ dphic, double* __restrict__ partials)
{
    step_fused_body<double, false, false>(p, tc, sF, sG, sphic, dF, dG, dphic, partials);
}

template <typename T>
struct Fused;
template <>
struct Fused<float> {
    static constexpr auto kernel = k_step_fused_f32;
};
template <>
struct Fused<double> {
    static constexpr auto kernel = k_step_fused_f64;
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

}  // namespace

TileCfg tile_config(const KParams& p, int segment_x)
{
    TileCfg tc;
    tc.nty = (p.ny + TY - 1) / TY;
    tc.ntz = (p.nz + TZ - 1) / TZ;
    tc.ntiles = tc.nty * tc.ntz;
    int sx = segment_x;
    if (sx <= 0) {
        // aim for ~2048 workgroups (8 per CU) with segments of at least 8 planes
        const long long want = (long long)p.nx * tc.ntiles / 2048;
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
            Fused<T>::kernel<<<nparts, kBlock, 0, s>>>(p, tc, a.F, a.G, a.phic, d.F, d.G,       \
                                                        d.phic, sums_out ? partials : nullptr); \
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
