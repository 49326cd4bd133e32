// Forward kernels (gfx950) of the D3Q19 symmetric binary-fluid LB step.
//
// The step of the paper's Ludwig timestep (Sec. 2.1.1) -- order-parameter
// gradients, chemical stress, collision, propagation -- runs as ONE kernel,
// k_step_fused_f32 / _f64: each workgroup owns a (y, z) tile of 4 x 128 (or
// 8 x 64, or 2 x 256) sites and marches along x over a segment of planes.  For plane x it needs phi at
// planes x-1, x, x+1 (7-point stencil); phi(x+1) is formed from the pulled g
// of plane x+1, which the same threads keep in registers for plane x+1's own
// collision one iteration later.  phi on the tile's (y, z) halo ring is
// formed by extra pulls that mostly hit in cache (the neighbouring tiles read
// the same lines).  phi planes live in a 4-slot LDS ring.  Every population
// is therefore read once and written once per step from HBM: the method's
// minimum traffic, instead of a separate phi pass plus a collision pass.
//
// k_phi + k_step_2s are the two-pass variant (phi kernel, then the
// stencil/collision/propagation kernel), kept for comparison; both variants
// produce bit-identical levels.  The force coupling runs the marching kernel
// of lb_force.hip (or k_phi and its one-site-per-thread collision pass);
// the finite-difference order parameter has
// its own kernels in lb_fd.hip.
#include <type_traits>

#include "lb_device.h"

namespace lbk {

using namespace dev;

namespace {

// Tiles of the single-pass kernel: TY rows of TZ contiguous z-sites, one
// site per thread of a kFused-thread workgroup: 4 x 128 (measured on MI355X at
// 256^3 against 4 x 64 and 8 x 64: the longer z runs give each component
// stream 512-byte (FP32) contiguous pieces), or 8 x 64 where that covers nz
// with fewer idle lanes (e.g. nz = 192: 64 + 64 + 64 instead of 128 + 64), or
// with FP32 storage and nz = 256, 2 x 256: whole rows (tile_config).
constexpr int kFused = 512;
// one thread per halo-ring cell (2 rows, 2 columns, 4 corners; a 2 x 256
// tile spans the periodic z extent and pulls the 2 rows only)
static_assert(2 * 128 + 2 * (kFused / 128) + 4 <= kFused, "halo ring larger than the workgroup");
static_assert(2 * 64 + 2 * (kFused / 64) + 4 <= kFused, "halo ring larger than the workgroup");

// ---------------------------------------------------------------------------

// Post-propagation state rho = rho0, u = 0, g_0 = phi0, g_{i>0} = 0.  In FP32
// mode phi_c is phi0's reference, and the stored deviation of direction i at
// y is g_i(y + c_i) - r_i phi_c(y + c_i).  In an x-slab shard phi0 also holds
// the planes -1 and nx (the neighbours'), first and last.
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_init(KParams p, T* __restrict__ F, T* __restrict__ G,
                                                 unsigned* __restrict__ phic,
                                                 const double* __restrict__ phi0)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    const double* ph = phi0 + (p.xh ? p.ny * p.nz : 0);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const unsigned d = dist_own(p, q, i);
        F[d] = DEV ? T(0) : T(weight(i) * p.rho0);
        if (REF) {
            const double pd = ph[push_site(p, q, i)];
            G[d] = T((i == 0 ? pd : 0.0) - rweight(i) * phic_round(pd));
        } else {
            G[d] = i == 0 ? T(ph[s]) : T(0);
        }
    }
    if (REF) phic[phic_site(p, q.x, q.y, q.z)] = phic_word(ph[s]);
}

// phi(x) = sum_i g_i(x) of the post-propagation state (FP64); with dphic
// (FP32 mode) also the reference field phi_c of the level a step makes.
template <typename T, bool REF>
__global__ __launch_bounds__(kBlock) void k_phi(KParams p, const T* __restrict__ G,
                                                const unsigned* __restrict__ phic,
                                                double* __restrict__ phi,
                                                unsigned* __restrict__ dphic)
{
    const int s = xcd_block() * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    const double v = phi_at<T, REF>(p, q, G, phic);
    phi[s] = v;
    if (REF && dphic) dphic[phic_site(p, q.x, q.y, q.z)] = phic_word(v);
}

// Two-pass variant, second pass: stencil + chemical stress + collision, one
// site per thread; phi of the post-propagation source level (all sites)
// comes from k_phi.
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_step_2s(KParams p, const T* __restrict__ sF,
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
        g[i] = sG[dist_pull(p, q, i)];
    }
    const double c = phi[s];
    const Stencil st = stencil(c, phi[site_of(p, q.xp, q.y, q.z)], phi[site_of(p, q.xm, q.y, q.z)],
                               phi[site_of(p, q.x, q.yp, q.z)], phi[site_of(p, q.x, q.ym, q.z)],
                               phi[site_of(p, q.x, q.y, q.zp)], phi[site_of(p, q.x, q.y, q.zm)]);
    if (REF) {
        const double dphi = c - phic_value(sphic[phic_site(p, q.x, q.y, q.z)]);
#pragma unroll
        for (int i = 0; i < NV; i++) g[i] = pre_collision_dev(i, g[i], dphi);
    }
    collide<T, DEV, REF>(p, f, g, st);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        dF[dist_own(p, q, i)] = f[i];
        dG[dist_own(p, q, i)] = REF ? to_dest_ref(i, g[i], c, phi[push_site(p, q, i)]) : g[i];
    }
}

// Register copy the compiler cannot merge away: the source register is free
// once the copy has executed, so a load issued after it can land in that
// register.  The memory clobber keeps later loads after the copy.
__device__ __forceinline__ float vcopy(float v)
{
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v) : "memory");
    return r;
}
__device__ __forceinline__ unsigned vcopy(unsigned v)
{
    unsigned r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v) : "memory");
    return r;
}
__device__ __forceinline__ double vcopy(double v)
{
    double r;
    asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "v"(v) : "memory");
    return r;
}

// Wrap a coordinate v in [-2n, 3n) onto [0, n).
__device__ __forceinline__ int wrapg(int v, int n)
{
    if (v < 0) return v + n < 0 ? v + 2 * n : v + n;
    if (v >= n) return v - n >= n ? v - 2 * n : v - n;
    return v;
}

// Addressing (layout of didx()): a thread's (y, z) never changes while it
// marches along x, so the byte offsets of the 9 rows/columns (y - cy, z - cz)
// within a plane are computed once (32-bit: one plane of F or G is under
// 4 GiB, checked at creation); a component adds a uniform in-plane offset
// and a plane a uniform plane offset -- 32-bit when the whole F or G region
// is under 4 GiB (SMALL), else 64-bit, added to the base pointer.
template <bool SMALL>
using OffT = typename std::conditional<SMALL, unsigned, size_t>::type;

template <bool SMALL, typename T>
__device__ __forceinline__ T ldc(const T* __restrict__ base, OffT<SMALL> pl, int i,
                                 unsigned compb, unsigned row)
{
    const char* b = reinterpret_cast<const char*>(base);
    if (SMALL) return *reinterpret_cast<const T*>(b + (unsigned(pl) + unsigned(i) * compb + row));
    // uniform 64-bit pointer to the component's run in the plane, then the row
    const char* bi = b + (size_t(pl) + size_t(i) * compb);
    return *reinterpret_cast<const T*>(bi + row);
}
// Stores are non-temporal: the new level is not read again in this launch,
// so it should not displace the source lines that neighbouring tiles still
// pull through L2.
template <bool SMALL, typename T>
__device__ __forceinline__ void stc(T* __restrict__ base, OffT<SMALL> pl, int i, unsigned compb,
                                    unsigned row, T v)
{
    char* b = reinterpret_cast<char*>(base);
    T* q = SMALL ? reinterpret_cast<T*>(b + (unsigned(pl) + unsigned(i) * compb + row))
                 : reinterpret_cast<T*>((b + (size_t(pl) + size_t(i) * compb)) + row);
    __builtin_nontemporal_store(v, q);
}

// byte offsets of the 9 rows/columns (y + dy, z + dz), dy, dz in {-1, 0, 1},
// within a plane of an F or G region
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
        for (int c = 0; c < 3; c++) r.o[a][c] = row_off(p, ys[a], zs[c]) * unsigned(sizeof(T));
    return r;
}

// Single-pass step (see the file comment).  Block -> (segment, tile) with
// an XCD-aware order: consecutive workgroup ids go round-robin over the 8
// XCDs, so ids are remapped to give each XCD a contiguous run of tiles, z
// fastest.  An XCD then owns slabs of whole (y) rows: the cache lines that
// z-shifted pulls and the halo columns share with the z-neighbouring tile,
// and the halo rows shared with y-neighbours, are fetched into the same L2.
//
// FP32 mode: the pull of a site needs only its own phi_c (one 32-bit load
// per site); the store of direction i needs phi at the destination y + c_i, which
// the LDS phi ring already holds (its halo then includes the tile's 4 corner
// cells, for the directions with c_x = 0 and c_y, c_z != 0).
// COLL = false is the kernel's memory-only twin (LB_KERNEL_STREAM): every
// load, LDS ring, phi sum and store of the step, with the collision left out,
// so the populations stream freely, f_i(x + c_i, t+1) = f_i(x, t).
template <typename T, bool DEV, bool REF, bool SMALL, bool PIPE, int TZ, bool COLL>
__device__ __forceinline__ void step_fused_body(const KParams& p, const TileCfg& tc,
                                                const T* __restrict__ sF,
                                                const T* __restrict__ sG,
                                                const unsigned* __restrict__ sphic,
                                                T* __restrict__ dF, T* __restrict__ dG,
                                                unsigned* __restrict__ dphic,
                                                double* __restrict__ phi_out,
                                                double* __restrict__ partials)
{
    constexpr int TY = kFused / TZ;
    __shared__ double ph[4][TY + 2][TZ + 2];
    // value kept per direction between the phi pull and the collision: the
    // stored FP32 deviation (FP32 mode) or the FP64 population
    using K = typename std::conditional<REF, T, double>::type;
    using O = OffT<SMALL>;
    const unsigned compb = p.cs * unsigned(sizeof(T));   // one component step
    const O planeb = O(p.plane_e) * O(sizeof(T));        // one plane of F or G

    const int b = xcd_block();
    const int tile = b % tc.ntiles, seg = b / tc.ntiles;
    const int y0 = (tile / tc.ntz) * TY, z0 = (tile % tc.ntz) * TZ;
    const int x0 = seg * tc.sx;
    const int x1 = min(x0 + tc.sx, p.nx);
    const int tya = min(TY, p.ny - y0), tza = min(TZ, p.nz - z0);
    const int lz = threadIdx.x % TZ, ly = threadIdx.x / TZ;
    const bool active = lz < tza && ly < tya;
    const int plane = p.ny * p.nz;
    // lanes outside the lattice hold a valid site's offsets and do nothing;
    // rowsite is the in-plane site index (for phi_c)
    const int sy = active ? y0 + ly : 0, sz = active ? z0 + lz : 0;
    const Yz9 row = yz9<T>(p, sy, sz);
    const unsigned rowsite = unsigned(sy * p.nz + sz);

    // halo ring: rows y0-1 and y0+tya, columns z0-1 and z0+tza, and in FP32
    // mode the 4 corners; cell r at LDS position (rly, rlz).  A tile that
    // spans the whole periodic z extent pulls only the two rows: its halo
    // columns are its own last and first columns, which put() below copies
    // into LDS columns 0 and tza + 1 as it stores them (the corners with
    // the rows' cells).
    const bool fullz = tza == p.nz;
    const int nside = fullz ? 2 * tza : 2 * tza + 2 * tya;
    const int nring = nside + (REF && !fullz ? 4 : 0);
    auto ring_cell = [&](int r, int& a, int& c) {
        if (r < tza) { a = 0; c = r + 1; }
        else if (r < 2 * tza) { a = tya + 1; c = r - tza + 1; }
        else if (r < 2 * tza + tya) { a = r - 2 * tza + 1; c = 0; }
        else if (r < nside) { a = r - 2 * tza - tya + 1; c = tza + 1; }
        else { a = ((r - nside) & 1) ? tya + 1 : 0; c = ((r - nside) & 2) ? tza + 1 : 0; }
    };
    const int r = threadIdx.x;
    const bool ring = r < nring;
    int rly, rlz;
    ring_cell(r, rly, rlz);
    const int ry = wrapg(y0 + rly - 1, p.ny), rz = wrapg(z0 + rlz - 1, p.nz);
    const Yz9 rrow = yz9<T>(p, ring ? ry : 0, ring ? rz : 0);
    const unsigned rsite = unsigned((ring ? ry : 0) * p.nz + (ring ? rz : 0));
    // phi into LDS cell (a, c) of slot sl, and into the wrap column of a
    // full-z tile
    auto put = [&](int sl, int a, int c, double v) __attribute__((always_inline)) {
        ph[sl][a][c] = v;
        if (fullz) {
            if (c == tza) ph[sl][a][0] = v;
            if (c == 1) ph[sl][a][tza + 1] = v;
        }
    };

    // plane indices run from x0-2 to x1+2 (nx may be 1): wrap without
    // division or branches (valid on [-2nx, 4nx)).  An x-slab shard has no
    // wrap: its regions hold planes -2 .. nx+1 of F and G (the halo planes
    // of the neighbours' populations) and -1 .. nx of phi_c; indices beyond
    // those occur only in the prefetch past a segment's end, whose values
    // go unused, and are clamped onto the last halo plane.
    auto xw = [&](int X) {
        X += X < 0 ? p.nx : 0;
        X += X < 0 ? p.nx : 0;
        X -= X >= p.nx ? p.nx : 0;
        X -= X >= p.nx ? p.nx : 0;
        X -= X >= p.nx ? p.nx : 0;
        return X;
    };
    auto xf = [&](int X) { return p.xh ? min(max(X, -2), p.nx + 1) + 2 : xw(X); };
    auto xc = [&](int X) { return p.xh ? min(max(X, -1), p.nx) + 1 : xw(X); };
    // byte base of plane X in F or G; element base of plane X in phi_c
    auto pbase = [&](int X) { return O(xf(X)) * planeb; };
    auto pcbase = [&](int X) { return unsigned(xc(X) * plane); };
    // pull of plane X for a site with row offsets yz and in-plane index
    // `site`: kept values into kv[] and the site's phi_c word into *pc (if
    // non-null); returns phi
    auto pull_phi = [&](int X, const Yz9& yz, unsigned site, K* kv, unsigned* pc)
                        __attribute__((always_inline)) -> double {
        const O pb[3] = {pbase(X - 1), pbase(X), pbase(X + 1)};
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const K v = K(ldc<SMALL>(sG, pb[1 - CX[i]], i, compb, yz.o[1 - CY[i]][1 - CZ[i]]));
            if (kv) kv[i] = v;
            acc += double(v);
        }
        if (REF) {
            const unsigned w = sphic[pcbase(X) + site];
            if (pc) *pc = w;
            return phic_value(w) + acc;
        }
        return acc;
    };

    // conserved sums of the source level (FP64), if requested
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    // collision of this thread's site at plane x and the stores of its new
    // values, from the pulled f[], the kept g values kc[] (and the site's
    // phi_c word pcc), with phi of planes x-1, x, x+1 in LDS slots sp, sc, sn
    auto update = [&](int x, T* f, const K* kc, unsigned pcc, int sp, int sc, int sn)
                      __attribute__((always_inline)) {
        const int psl[3] = {sp, sc, sn};
        const double c = ph[sc][ly + 1][lz + 1];
        const Stencil st = stencil(c, ph[sn][ly + 1][lz + 1], ph[sp][ly + 1][lz + 1],
                                   ph[sc][ly + 2][lz + 1], ph[sc][ly][lz + 1],
                                   ph[sc][ly + 1][lz + 2], ph[sc][ly + 1][lz]);
        T g[NV];
        if (REF) {
            const double dphi = c - phic_value(pcc);
#pragma unroll
            for (int i = 0; i < NV; i++) g[i] = pre_collision_dev(i, T(kc[i]), dphi);
        } else {
#pragma unroll
            for (int i = 0; i < NV; i++) g[i] = T(kc[i]);
        }
        if (partials) {
            // moments of the stored values, formed in FP64; with FP32 storage
            // from the sums and differences of the direction pairs
            // (2k+1, 2k+2), in short chains (0.5% faster than running sums;
            // FP64 storage keeps the running sums, 0.2% faster there)
            double bs = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            if constexpr (REF) {
                double v[NV];
#pragma unroll
                for (int i = 0; i < NV; i++) v[i] = double(f[i]);
                double sp[9], dp[9];
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    sp[k] = v[2 * k + 1] + v[2 * k + 2];
                    dp[k] = v[2 * k + 1] - v[2 * k + 2];
                }
                bs = ((v[0] + (sp[0] + sp[1])) + ((sp[2] + sp[3]) + (sp[4] + sp[5])))
                   + ((sp[6] + sp[7]) + sp[8]);
                jx = ((dp[0] + dp[3]) + (dp[4] + dp[5])) + dp[6];
                jy = ((dp[1] + dp[3]) - dp[4]) + (dp[7] + dp[8]);
                jz = ((dp[2] + dp[5]) - dp[6]) + (dp[7] - dp[8]);
            } else {
#pragma unroll
                for (int i = 0; i < NV; i++) {
                    const double v = double(f[i]);
                    bs += v;
                    if (CX[i]) jx += CX[i] * v;
                    if (CY[i]) jy += CY[i] * v;
                    if (CZ[i]) jz += CZ[i] * v;
                }
            }
            acc[0] += DEV ? p.rho0 + bs : bs;
            acc[1] += c;
            acc[2] += jx;
            acc[3] += jy;
            acc[4] += jz;
        }
        if (COLL) collide<T, DEV, REF>(p, f, g, st);
        const O pso = pbase(x);
        const unsigned so = row.o[1][1];
#pragma unroll
        for (int i = 0; i < NV; i++) {
            stc<SMALL>(dF, pso, i, compb, so, f[i]);
            const T gi = REF ? to_dest_ref(i, g[i], c,
                                           ph[psl[1 + CX[i]]][ly + 1 + CY[i]][lz + 1 + CZ[i]])
                             : g[i];
            stc<SMALL>(dG, pso, i, compb, so, gi);
        }
        // FP32: the new level's reference field; phi of the source level,
        // if asked for
        if (REF) dphic[pcbase(x) + rowsite] = phic_word(c);
        if (phi_out) phi_out[unsigned(x * plane) + rowsite] = c;
    };

    // Software-pipelined march (full tiles): the loads of plane x+2's g
    // (interior and ring) and phi_c and of plane x+1's f are issued before
    // plane x's collision and stores and consumed one iteration later, so
    // the workgroup keeps them in flight across its arithmetic and stores.
    // The path is branch-free -- every lane of a full tile is a site, the
    // ring cells are spread evenly over all waves (spare lanes repeat a cell
    // of their wave), the last iteration's prefetch of planes beyond the
    // segment is issued and left unused -- so the compiler's completion waits
    // follow the issue order exactly: each wait covers loads issued a whole
    // iteration earlier, never the stores issued since.
    const bool full = tya == TY && tza == TZ;
    if (PIPE && full) {
        constexpr int NW = kFused / 64;
        // ring cells per wave (a 2 x 256 tile is always full-z: its ring is
        // the two rows, one cell per lane)
        constexpr int RPW_ALL = (2 * TZ + 2 * TY + 4 + NW - 1) / NW;
        constexpr int RPW = RPW_ALL <= 64 ? RPW_ALL : 2 * TZ / NW;
        static_assert(RPW <= 64, "more ring cells than lanes");
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        int qly, qlz;
        ring_cell(min(w * RPW + (lane < RPW ? lane : 0), nring - 1), qly, qlz);
        const int qy = wrapg(y0 + qly - 1, p.ny), qz = wrapg(z0 + qlz - 1, p.nz);
        const Yz9 qrow = yz9<T>(p, qy, qz);
        const unsigned qsite = unsigned(qy * p.nz + qz);

        T fq[NV], fc[NV];
        K gq[NV], rq[NV], kn[NV], kcur[NV];
        unsigned pq = 0, rpq = 0, pcn = 0, pccur = 0;
        // g and phi_c of plane X+1 (interior, ring); f(X)
        auto issue = [&](int X) __attribute__((always_inline)) {
            const O pf[3] = {pbase(X - 1), pbase(X), pbase(X + 1)};
            const O pg[3] = {pf[1], pf[2], pbase(X + 2)};
            // issue order fixed (scheduling barriers): interior g, ring g,
            // f -- the order in which the next iteration consumes them
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < NV; i++)
                gq[i] = K(ldc<SMALL>(sG, pg[1 - CX[i]], i, compb, row.o[1 - CY[i]][1 - CZ[i]]));
            if (REF) pq = sphic[pcbase(X + 1) + rowsite];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < NV; i++)
                rq[i] = K(ldc<SMALL>(sG, pg[1 - CX[i]], i, compb, qrow.o[1 - CY[i]][1 - CZ[i]]));
            if (REF) rpq = sphic[pcbase(X + 1) + qsite];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < NV; i++)
                fq[i] = ldc<SMALL>(sF, pf[1 - CX[i]], i, compb, row.o[1 - CY[i]][1 - CZ[i]]);
            __builtin_amdgcn_sched_barrier(0);
        };
        put(0, ly + 1, lz + 1, pull_phi(x0 - 1, row, rowsite, nullptr, nullptr));
        put(0, qly, qlz, pull_phi(x0 - 1, qrow, qsite, nullptr, nullptr));
        put(1, ly + 1, lz + 1, pull_phi(x0, row, rowsite, kcur, &pccur));
        put(1, qly, qlz, pull_phi(x0, qrow, qsite, nullptr, nullptr));
        issue(x0);
        // enter the loop with these loads completed (an empty asm reading
        // each register makes the compiler wait for it here): the waits at
        // the loop's top then follow its steady state -- loads issued an
        // iteration ago, stores issued since -- not this entry path
#pragma unroll
        for (int i = 0; i < NV; i++) asm volatile("" ::"v"(gq[i]), "v"(rq[i]), "v"(fq[i]));
        asm volatile("" ::"v"(pq), "v"(rpq));
        for (int x = x0; x < x1; x++) {
            const int kk = x - x0 + 2;  // phi slot counter of plane x+1
            const int sn = kk & 3, sc = (kk - 1) & 3, sp = (kk - 2) & 3;
            // phi of plane x+1 from the loads issued one iteration ago, in
            // the index order every kernel uses
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int i = 0; i < NV; i++) a += double(gq[i]);
            put(sn, ly + 1, lz + 1, REF ? phic_value(pq) + a : a);
#pragma unroll
            for (int i = 0; i < NV; i++) b += double(rq[i]);
            put(sn, qly, qlz, REF ? phic_value(rpq) + b : b);
            lds_barrier();
#pragma unroll
            for (int i = 0; i < NV; i++) {
                fc[i] = vcopy(fq[i]);
                kn[i] = vcopy(gq[i]);
            }
            pcn = vcopy(pq);
            issue(x + 1);
            update(x, fc, kcur, pccur, sp, sc, sn);
#pragma unroll
            for (int i = 0; i < NV; i++) kcur[i] = kn[i];
            pccur = pcn;
        }
    } else {
        // Plain march (FP64, and FP32 ragged tiles), with the f pull of
        // plane x+1 issued before plane x's collision so that those loads
        // are in flight across its arithmetic and stores.  The registers for
        // them come from parking the kept g values of plane x+1 in LDS (each
        // thread its own slots) between their pull and their collision one
        // iteration later; measured in FP64 at 256^3: 4% faster, now within
        // 1% of the memory-only twin.
        K kcur[NV], knext[NV];
        __shared__ K kst[NV][kFused];
        unsigned pccur = 0, pcnext = 0;
        // warm-up: phi at planes x0-1 (slot 0) and x0 (slot 1), keeping
        // plane x0's populations
        if (active) put(0, ly + 1, lz + 1, pull_phi(x0 - 1, row, rowsite, nullptr, nullptr));
        if (ring) put(0, rly, rlz, pull_phi(x0 - 1, rrow, rsite, nullptr, nullptr));
        if (active) put(1, ly + 1, lz + 1, pull_phi(x0, row, rowsite, kcur, &pccur));
        if (ring) put(1, rly, rlz, pull_phi(x0, rrow, rsite, nullptr, nullptr));
        T fn[NV];
        auto pull_f = [&](int X) __attribute__((always_inline)) {
            const O pbx[3] = {pbase(X - 1), pbase(X), pbase(X + 1)};
#pragma unroll
            for (int i = 0; i < NV; i++)
                fn[i] = ldc<SMALL>(sF, pbx[1 - CX[i]], i, compb, row.o[1 - CY[i]][1 - CZ[i]]);
        };
        if (active) pull_f(x0);
        for (int x = x0; x < x1; x++) {
            const int kk = x - x0 + 2;  // phi slot counter of plane x+1
            const int sn = kk & 3, sc = (kk - 1) & 3, sp = (kk - 2) & 3;
            T f[NV];
            if (active) {
                put(sn, ly + 1, lz + 1, pull_phi(x + 1, row, rowsite, knext, &pcnext));
#pragma unroll
                for (int i = 0; i < NV; i++) kst[i][threadIdx.x] = knext[i];
            }
            if (ring) put(sn, rly, rlz, pull_phi(x + 1, rrow, rsite, nullptr, nullptr));
            lds_barrier();
            if (active) {
#pragma unroll
                for (int i = 0; i < NV; i++) f[i] = vcopy(fn[i]);
                if (x + 1 < x1) pull_f(x + 1);
                update(x, f, kcur, pccur, sp, sc, sn);
#pragma unroll
                for (int i = 0; i < NV; i++) kcur[i] = kst[i][threadIdx.x];
                pccur = pcnext;
            }
        }
    }
    if (partials) block_partials<5, kFused>(acc, partials);
}

template <bool SMALL, int TZ, bool COLL>
__global__ __launch_bounds__(kFused) void k_step_fused_f32(
    KParams p, TileCfg tc, const float* __restrict__ sF, const float* __restrict__ sG,
    const unsigned* __restrict__ sphic, float* __restrict__ dF, float* __restrict__ dG,
    unsigned* __restrict__ dphic, double* __restrict__ phi_out, double* __restrict__ partials)
{
    step_fused_body<float, true, true, SMALL, true, TZ, COLL>(p, tc, sF, sG, sphic, dF, dG, dphic,
                                                              phi_out, partials);
}

template <bool SMALL, int TZ, bool COLL>
__global__ __launch_bounds__(kFused) void k_step_fused_f64(
    KParams p, TileCfg tc, const double* __restrict__ sF, const double* __restrict__ sG,
    const unsigned* __restrict__ sphic, double* __restrict__ dF, double* __restrict__ dG,
    unsigned* __restrict__ dphic, double* __restrict__ phi_out, double* __restrict__ partials)
{
    step_fused_body<double, false, false, SMALL, false, TZ, COLL>(p, tc, sF, sG, sphic, dF, dG,
                                                                  dphic, phi_out, partials);
}

// the single-pass kernel (or, coll = false, its free-streaming twin) for an
// offset width and a tile width
template <typename T>
struct Fused;
template <>
struct Fused<float> {
    using K = decltype(&k_step_fused_f32<true, 128, true>);
    template <bool COLL>
    static K pick(bool small, int tz)
    {
        if (tz == 256) return small ? k_step_fused_f32<true, 256, COLL> : k_step_fused_f32<false, 256, COLL>;
        if (tz == 64) return small ? k_step_fused_f32<true, 64, COLL> : k_step_fused_f32<false, 64, COLL>;
        return small ? k_step_fused_f32<true, 128, COLL> : k_step_fused_f32<false, 128, COLL>;
    }
    static K get(bool small, int tz, bool coll)
    {
        return coll ? pick<true>(small, tz) : pick<false>(small, tz);
    }
};
template <>
struct Fused<double> {
    using K = decltype(&k_step_fused_f64<true, 128, true>);
    template <bool COLL>
    static K pick(bool small, int tz)
    {
        if (tz == 64) return small ? k_step_fused_f64<true, 64, COLL> : k_step_fused_f64<false, 64, COLL>;
        return small ? k_step_fused_f64<true, 128, COLL> : k_step_fused_f64<false, 128, COLL>;
    }
    static K get(bool small, int tz, bool coll)
    {
        return coll ? pick<true>(small, tz) : pick<false>(small, tz);
    }
};

// Dense FP64 moments of the post-propagation state and block partials of
// [rho, phi, jx, jy, jz] (grid-stride, FP64 accumulation).
// With fphi (force coupling: phi of this state, all sites) the velocity is
// (j + F/2)/rho, F = -div Pi of this state, and the momentum sums are those
// of j + F/2.
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_moments(KParams p, const T* __restrict__ F,
                                                    const T* __restrict__ G,
                                                    const unsigned* __restrict__ phic,
                                                    const double* __restrict__ fphi,
                                                    double* __restrict__ rho_out,
                                                    double* __restrict__ u_out,
                                                    double* __restrict__ phi_out,
                                                    double* __restrict__ partials)
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = xcd_block() * kBlock + threadIdx.x; s < p.nsites; s += gridDim.x * kBlock) {
        const Geo q = geo_of(p, s);
        double fv[NV];
#pragma unroll
        for (int i = 0; i < NV; i++) fv[i] = double(F[dist_pull(p, q, i)]);
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
        if (fphi) {
            double fo[3];
            force_from_phi(p, q, fphi, fo);
            jx += 0.5 * fo[0];
            jy += 0.5 * fo[1];
            jz += 0.5 * fo[2];
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

// out[k] (+)= sum over nblocks partials of component k (k < ncomp <= 5), one
// workgroup.
__global__ __launch_bounds__(kBlock) void k_sums_final(const double* __restrict__ partials,
                                                       int nblocks, int ncomp,
                                                       double* __restrict__ out, int accumulate)
{
    reduce_partials_block(partials, nblocks, ncomp, out, accumulate != 0);
}

template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_export(KParams p, const T* __restrict__ F,
                                                   const T* __restrict__ G,
                                                   const unsigned* __restrict__ phic,
                                                   double* __restrict__ f, double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
    if (f)
#pragma unroll
        for (int i = 0; i < NV; i++)
            f[(long long)i * p.nsites + s] =
                double(F[dist_pull(p, q, i)]) + (DEV ? weight(i) * p.rho0 : 0.0);
    if (g) {
        double d[NV];
        pull_g<T, REF>(p, q, G, phic, d);
#pragma unroll
        for (int i = 0; i < NV; i++) g[(long long)i * p.nsites + s] = d[i];
    }
}

// FP32 mode, first half of an import: the reference phi_c(x) of
// phi(x) = sum_i g_i(x) of the dense post-propagation input.
__global__ __launch_bounds__(kBlock) void k_import_ref(KParams p, unsigned* __restrict__ phic,
                                                       const double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NV; i++) acc += g[(long long)i * p.nsites + s];
    phic[s] = phic_word(acc);
}

// The stored value of direction i at y is the post-propagation value at
// y + c_i (FP32 mode: minus w_i rho0 for f, minus r_i phi_c(y + c_i) for g).
template <typename T, bool DEV, bool REF>
__global__ __launch_bounds__(kBlock) void k_import(KParams p, T* __restrict__ F, T* __restrict__ G,
                                                   const unsigned* __restrict__ phic,
                                                   const double* __restrict__ f,
                                                   const double* __restrict__ g)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= p.nsites) return;
    const Geo q = geo_of(p, s);
#pragma unroll
    for (int i = 0; i < NV; i++) {
        const int d = push_site(p, q, i);
        const long long n = d + (long long)i * p.nsites;
        F[dist_own(p, q, i)] = T(f[n] - (DEV ? weight(i) * p.rho0 : 0.0));
        G[dist_own(p, q, i)] = T(REF ? g[n] - rweight(i) * phic_value(phic[d]) : g[n]);
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
            (void)DEV;                    \
            CALL32;                       \
        } else {                          \
            using T = double;             \
            constexpr bool DEV = false;   \
            constexpr bool REF = false;   \
            (void)DEV;                    \
            CALL64;                       \
        }                                 \
    } while (0)

// a 19-component F or G region addressed with 32-bit byte offsets
bool small_arrays(const KParams& p, size_t elem)
{
    return size_t(NV) * p.stride * elem < (size_t(1) << 32);
}

}  // namespace

void set_layout(KParams& k, int layout, int aosoa_len)
{
    const unsigned ny = unsigned(k.ny), nz = unsigned(k.nz), nv = unsigned(NV);
    k.vs = 31;  // z >> 31 == 0: no z-blocks
    k.vm = 0xffffffffu;
    k.zb = 0;
    k.plane_e = ny * nz * nv;
    k.ry = nz * nv;
    switch (layout) {
    case 1:  // one array per component
        k.plane_e = ny * nz;
        k.ry = nz;
        k.cs = k.stride;
        break;
    case 2:  // a site's components together
        k.vs = 0;
        k.vm = 0;
        k.zb = nv;
        k.cs = 1;
        break;
    case 3: {  // blocks of V z-sites
        unsigned v = unsigned(aosoa_len), sh = 0;
        while ((1u << sh) < v) sh++;
        k.vs = sh;
        k.vm = v - 1;
        k.zb = nv * v;
        k.cs = v;
        break;
    }
    default:  // row-blocked
        k.cs = nz;
        break;
    }
}

// Number of CUs of an MI355X: with 512-thread workgroups at 2 waves per SIMD,
// one workgroup per CU runs at a time.
constexpr int kCUs = 256;

TileCfg tile_config(const KParams& p, int segment_x, bool fp32)
{
    TileCfg tc;
    // tile width: 128 unless 64 leaves fewer idle lanes along z
    const long long w128 = 128LL * ((p.nz + 127) / 128), w64 = 64LL * ((p.nz + 63) / 64);
    tc.tz = w64 < w128 ? 64 : 128;
    // FP32 storage with z-rows of 256 sites (the LB step; the
    // finite-difference kernel has its own widths): 2 x 256 tiles, each a
    // pair of whole rows, which need no z halo and read every component's
    // row in one contiguous piece.  Measured at 256^3, same buffers: 2.5%
    // faster than 4 x 128 (the memory-only twin 3.4%); in FP64 storage 3.8%
    // slower, so FP64 keeps 4 x 128.
    if (fp32 && p.nz == 256 && !p.fd) tc.tz = 256;
    const int ty = kFused / tc.tz;
    tc.nty = (p.ny + ty - 1) / ty;
    tc.ntz = (p.nz + tc.tz - 1) / tc.tz;
    tc.ntiles = tc.nty * tc.ntz;
    int sx = segment_x;
    if (sx <= 0) {
        // Segments along x: a workgroup marches sx planes after 2 warm-up
        // planes, and workgroups run in rounds of kCUs.  Pick the segment
        // count minimising rounds * (sx + 2) (fewest workgroups on ties);
        // this fits measured times at 128^3 to 256^3 within 10%.
        long long best = -1;
        for (int nseg = 1; nseg <= p.nx; nseg++) {
            const int s = (p.nx + nseg - 1) / nseg;
            const long long nb = (long long)tc.ntiles * ((p.nx + s - 1) / s);
            const long long rounds = (nb + kCUs - 1) / kCUs;
            const long long cost = rounds * (s + 2);
            if (best < 0 || cost < best) {
                best = cost;
                sx = s;
            }
        }
    }
    if (sx > p.nx) sx = p.nx;
    tc.sx = sx;
    tc.nseg = (p.nx + sx - 1) / sx;
    tc.seg_req = segment_x;
    return tc;
}

int step_sums_blocks(const KParams& p, const TileCfg& tc, int variant)
{
    if (variant == 1) return reduction_grid(p);
    if (p.force) return force_sums_blocks(p, tc.seg_req);
    return tc.ntiles * tc.nseg;
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
                       double* sums_out, double* phi_src_out, hipStream_t s)
{
    // phi of src goes to phi_src_out if given (the work field otherwise,
    // where a pass needs one)
    double* phi64 = phi_src_out ? phi_src_out : phi_work;
    int nparts = 0;
    if (p.force) {
        // the two-pass variant first forms phi (and in FP32 mode the new
        // level's phi_c), and with sums the moments pass (momentum sums of
        // j + F/2 from that phi); the single pass sums phi from its own pulls
        // and leaves the block partials itself
#define CALL                                                                                   \
    {                                                                                          \
        Lvl<T> a = level<T>(const_cast<void*>(src), p, REF);                                   \
        Lvl<T> d = level<T>(dst, p, REF);                                                      \
        if (variant == 1) {                                                                    \
            k_phi<T, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.G, a.phic, phi64, d.phic);       \
            if (sums_out) {                                                                    \
                nparts = reduction_grid(p);                                                    \
                k_moments<T, DEV, REF><<<nparts, kBlock, 0, s>>>(p, a.F, a.G, a.phic, phi64,   \
                                                                 nullptr, nullptr, nullptr,    \
                                                                 partials);                    \
            }                                                                                  \
        }                                                                                      \
    }
        LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
        if (variant != 1 && sums_out) nparts = force_sums_blocks(p, tc.seg_req);
        {
            hipError_t e = launch_force_collide(p, tc, fp32, variant, src, dst,
                                                variant == 1 ? phi64 : phi_src_out,
                                                sums_out ? partials : nullptr, s);
            if (e != hipSuccess) return e;
        }
        if (sums_out) k_sums_final<<<1, kBlock, 0, s>>>(partials, nparts, 5, sums_out, 0);
        return hipGetLastError();
    }
#define CALL                                                                                    \
    {                                                                                           \
        Lvl<T> a = level<T>(const_cast<void*>(src), p, REF);                                    \
        Lvl<T> d = level<T>(dst, p, REF);                                                       \
        if (variant != 1) {                                                                     \
            nparts = tc.ntiles * tc.nseg;                                                       \
            auto kern = Fused<T>::get(small_arrays(p, sizeof(T)), tc.tz, variant == 0);        \
            kern<<<nparts, kFused, 0, s>>>(p, tc, a.F, a.G, a.phic, d.F, d.G, d.phic,           \
                                           phi_src_out, sums_out ? partials : nullptr);         \
        } else {                                                                                \
            if (sums_out) {                                                                     \
                nparts = reduction_grid(p);                                                     \
                k_moments<T, DEV, REF><<<nparts, kBlock, 0, s>>>(p, a.F, a.G, a.phic, nullptr,  \
                                                                 nullptr, nullptr, nullptr,     \
                                                                 partials);                     \
            }                                                                                   \
            k_phi<T, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.G, a.phic, phi64, d.phic);        \
            k_step_2s<T, DEV, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, phi64,   \
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
        k_phi<T, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.G, a.phic, phi, nullptr);       \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_moments(const KParams& p, bool fp32, const void* state, double* rho, double* u,
                          double* phi, double* work, double* partials, int* nblocks_out,
                          hipStream_t s)
{
    const int nb = reduction_grid(p);
    *nblocks_out = nb;
    double* fphi = nullptr;
    if (p.force && (u || partials)) {
        // F of this state: phi into the work field first
        fphi = work;
#define CALL                                                                                  \
    {                                                                                         \
        Lvl<T> a = level<T>(const_cast<void*>(state), p, REF);                                \
        k_phi<T, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.G, a.phic, work, nullptr);          \
    }
        LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    }
#define CALL                                                                                  \
    {                                                                                         \
        Lvl<T> a = level<T>(const_cast<void*>(state), p, REF);                                \
        k_moments<T, DEV, REF><<<nb, kBlock, 0, s>>>(p, a.F, a.G, a.phic, fphi, rho, u, phi, \
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
        if (REF) k_import_ref<<<grid_for(p), kBlock, 0, s>>>(p, a.phic, g);                   \
        k_import<T, DEV, REF><<<grid_for(p), kBlock, 0, s>>>(p, a.F, a.G, a.phic, f, g);      \
    }
    LB_DISPATCH(fp32, CALL, CALL);
#undef CALL
    return hipGetLastError();
}

}  // namespace lbk
