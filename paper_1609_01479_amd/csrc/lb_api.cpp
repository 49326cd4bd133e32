// C-ABI host layer: argument validation, buffer layout and launch sequencing
// for the kernels in lb_kernels.hip.  See include/lb.h for the contract.
#include "lb.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>

#include "lb_internal.h"

namespace {

thread_local char g_err[512] = "";

lb_status fail(lb_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

lb_status hip_fail(hipError_t e, const char* what)
{
    return fail(LB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int kAdjComponents = 2 * LB_NVEL + 1;  // lambda_f, lambda_g, lambda_phi
constexpr int kAdjScratchComponents = 5;         // a, b_x, b_y, b_z, c
constexpr int kAdjScratchForce = 8;              // ... and dL/dF (force coupling)

// Elements per component in a time level: N rounded up to 256, plus 4352
// (4096 + 256) of padding between the f region, the g region and phi_c, so
// those streams do not start at the same offset modulo large powers of two
// (HBM channel and bank interleave; measured on MI355X with one array per
// component, 2-4% faster than 256 or none).
size_t stride_for(long long n)
{
    const size_t r = (size_t(n) + 255) / 256 * 256;
    return r + 4352;
}

bool aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) % kAlign) == 0; }

// Sites a component of a time level holds: the lattice's, plus (x-slab
// shard) two halo planes on each side.
long long level_sites(const lb_params* p)
{
    return (long long)(p->nx + (p->halo_x ? 4 : 0)) * p->ny * p->nz;
}

lb_status validate(const lb_params* p)
{
    if (!p) return fail(LB_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LB_ESHAPE, "extents must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
    if (p->halo_x != 0 && p->halo_x != 1) return fail(LB_EINVAL, "halo_x must be 0 or 1");
    const long long n = level_sites(p);
    // element offsets in the kernels are 32-bit: component * stride + site with
    // up to 39 components (an adjoint level)
    if ((long long)(stride_for(n)) * 39 >= (1LL << 32))
        return fail(LB_ESHAPE, "lattice of %lld sites is too large (limit ~1.1e8 sites)", n);
    // one x-plane of the row-blocked f or g region is addressed with 32-bit
    // byte offsets (FP64: ny*nz < ~2.8e7)
    const long long elem = p->precision == LB_FP32_DEV ? 4 : 8;
    if ((long long)p->ny * p->nz * LB_NVEL * elem >= (1LL << 32))
        return fail(LB_ESHAPE, "x-plane of %lld sites is too large (ny*nz*19*%lld bytes >= 4 GiB)",
                    (long long)p->ny * p->nz, elem);
    if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5))
        return fail(LB_EINVAL, "tau_f and tau_g must exceed 1/2 (got %g, %g)", p->tau_f, p->tau_g);
    if (!(p->rho0 > 0.0)) return fail(LB_EINVAL, "rho0 must be positive (got %g)", p->rho0);
    if (p->precision != LB_FP64 && p->precision != LB_FP32_DEV)
        return fail(LB_EINVAL, "unknown precision %d", p->precision);
    if (p->kernel != LB_KERNEL_FUSED && p->kernel != LB_KERNEL_TWO_PASS &&
        p->kernel != LB_KERNEL_STREAM)
        return fail(LB_EINVAL, "unknown kernel variant %d", p->kernel);
    if (p->kernel == LB_KERNEL_STREAM &&
        (p->coupling != LB_COUPLING_STRESS || p->order_param != LB_OP_LB))
        return fail(LB_EINVAL, "LB_KERNEL_STREAM is the twin of the LB_OP_LB stress-coupled step");
    if (p->layout < LB_LAYOUT_ROWS || p->layout > LB_LAYOUT_AOSOA)
        return fail(LB_EINVAL, "unknown layout %d", p->layout);
    if (p->coupling != LB_COUPLING_STRESS && p->coupling != LB_COUPLING_FORCE)
        return fail(LB_EINVAL, "unknown coupling %d", p->coupling);
    if (p->order_param != LB_OP_LB && p->order_param != LB_OP_FD)
        return fail(LB_EINVAL, "unknown order_param %d", p->order_param);
    if (p->halo_x) {
        if (p->nx < 2) return fail(LB_ESHAPE, "an x-slab shard needs nx >= 2 (got %d)", p->nx);
        if (p->order_param != LB_OP_LB || p->coupling != LB_COUPLING_STRESS ||
            (p->kernel != LB_KERNEL_FUSED && p->kernel != LB_KERNEL_STREAM))
            return fail(LB_EINVAL, "x-slab shards (halo_x) run the single-pass LB_OP_LB step "
                                   "with LB_COUPLING_STRESS only");
    }
    if (p->layout == LB_LAYOUT_AOSOA) {
        const int v = p->aosoa_len;
        if (v < 1 || (v & (v - 1)) != 0 || p->nz % v != 0)
            return fail(LB_ESHAPE, "aosoa_len %d must be a power of two dividing nz = %d", v,
                        p->nz);
    }
    return LB_OK;
}

}  // namespace

struct lb_ctx {
    lb_params p;
    lb_sizes sz;
    lb_buffers b;
    hipStream_t stream;
    lbk::KParams kp;
    lbk::TileCfg tc;
    bool fp32;
    int cur;      // time level holding the current state
    int adj_cur;  // adjoint level holding the current lambda
    bool has_adj;
};

// ---- allocation-free lb_step_sums --------------------------------------
// The reduction partials of lb_step_sums_noalloc live in this array instead
// of the caller's scratch buffer: one copy per GPU the library runs on, held
// until the process ends.  On the host the name `scratch` is only a stand-in
// for the symbol, never a device address: host code takes the address of
// each GPU's copy from hipGetSymbolAddress (with that GPU current) and uses
// only that.  Every block of a reducing step writes its own five slots
// before the final pass reads them, so nothing has to start at zero.
static __device__ __align__(256) double scratch[LB_NOALLOC_MAX_PARTIALS * 5];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch` (looked up once per
// device, then reused).
lb_status noalloc_scratch(lb_ctx* ctx, double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "lb_step_sums_noalloc (hipGetDevice)");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LB_ESTATE, "lb_step_sums_noalloc: device %d is beyond the %d the library "
                               "tracks", dev, kMaxDevices);
    if (ctx->stream) {
        int sdev = -1;
        e = hipStreamGetDevice(ctx->stream, &sdev);
        if (e != hipSuccess) return hip_fail(e, "lb_step_sums_noalloc (hipStreamGetDevice)");
        if (sdev != dev)
            return fail(LB_ESTATE, "lb_step_sums_noalloc: the current device (%d) is not the "
                                   "context stream's (%d)", dev, sdev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "lb_step_sums_noalloc (hipGetSymbolAddress)");
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return LB_OK;
}

}  // namespace

extern "C" {

int32_t lb_abi_version(void) { return LB_ABI_VERSION; }

const char* lb_status_string(lb_status s)
{
    switch (s) {
        case LB_OK: return "ok";
        case LB_EINVAL: return "invalid argument";
        case LB_ESHAPE: return "invalid lattice shape";
        case LB_EALIGN: return "device pointer not 256-byte aligned";
        case LB_EHIP: return "HIP runtime error";
        case LB_ESTATE: return "call not valid in this state";
    }
    return "unknown status";
}

const char* lb_last_error(void) { return g_err; }

lb_status lb_query_sizes(const lb_params* p, lb_sizes* out)
{
    lb_status st = validate(p);
    if (st != LB_OK) return st;
    if (!out) return fail(LB_EINVAL, "out is NULL");
    const long long n = (long long)p->nx * p->ny * p->nz;
    const size_t e = p->precision == LB_FP64 ? 8 : 4;
    const size_t stride = stride_for(level_sites(p));
    out->elem_bytes = e;
    out->stride_elems = stride;
    const bool fd = p->order_param == LB_OP_FD;
    if (fd) {
        // f, then the FP64 phi field; work fields mu, u_x, u_y, u_z
        out->state_bytes = LB_NVEL * stride * e + stride * 8;
        out->phi_bytes = 4 * stride * 8;
    } else {
        // f and g, plus the 32-bit reference order parameter in FP32 mode
        out->state_bytes = 2 * LB_NVEL * stride * e + (p->precision == LB_FP32_DEV ? stride * 4 : 0);
        // FP64 work field: phi
        out->phi_bytes = stride * 8;
    }
    // block partials of the reductions: 5 FP64 per block of the largest grid
    lbk::KParams k{};
    k.nx = p->nx;
    k.ny = p->ny;
    k.nz = p->nz;
    k.fd = fd;
    const lbk::TileCfg tc = lbk::tile_config(k, p->segment_x, p->precision == LB_FP32_DEV);
    k.nsites = int(n);
    size_t nparts = std::max<size_t>(size_t(tc.ntiles) * tc.nseg, lbk::kMaxPartialBlocks);
    if (fd) nparts = std::max<size_t>(nparts, size_t(lbk::fd_step_partial_blocks(k, p->segment_x)));
    else if (p->coupling == LB_COUPLING_FORCE)
        nparts = std::max<size_t>(nparts, size_t(lbk::force_sums_blocks(k, p->segment_x)));
    out->scratch_bytes = nparts * 5 * 8;
    out->adj_bytes = size_t(kAdjComponents) * stride * e;
    out->face_bytes = p->halo_x ? lbk::face_bytes(k, p->precision == LB_FP32_DEV) : 0;
    out->adj_scratch_bytes =
        size_t(p->coupling == LB_COUPLING_FORCE ? kAdjScratchForce : kAdjScratchComponents) *
        stride * e;
    return LB_OK;
}

lb_status lb_create(const lb_params* p, const lb_buffers* b, void* hip_stream, lb_ctx** out)
{
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    lb_sizes sz;
    lb_status st = lb_query_sizes(p, &sz);
    if (st != LB_OK) return st;
    if (!b) return fail(LB_EINVAL, "buffers is NULL");
    const void* req[] = {b->state[0], b->state[1], b->phi, b->scratch};
    for (const void* q : req) {
        if (!q) return fail(LB_EINVAL, "state[0], state[1], phi and scratch are required");
        if (!aligned(q)) return fail(LB_EALIGN, "buffer %p is not 256-byte aligned", q);
    }
    const bool any_adj = b->adj[0] || b->adj[1] || b->adj_scratch;
    const bool all_adj = b->adj[0] && b->adj[1] && b->adj_scratch;
    if (any_adj && !all_adj)
        return fail(LB_EINVAL, "adj[0], adj[1] and adj_scratch must be given together");
    if (all_adj && (!aligned(b->adj[0]) || !aligned(b->adj[1]) || !aligned(b->adj_scratch)))
        return fail(LB_EALIGN, "adjoint buffers must be 256-byte aligned");
    if (b->state[0] == b->state[1]) return fail(LB_EINVAL, "state[0] and state[1] alias");

    lb_ctx* c = new (std::nothrow) lb_ctx;
    if (!c) return fail(LB_EINVAL, "out of host memory");
    c->p = *p;
    c->sz = sz;
    c->b = *b;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->fp32 = p->precision == LB_FP32_DEV;
    c->cur = 0;
    c->adj_cur = 0;
    c->has_adj = all_adj;
    lbk::KParams& k = c->kp;
    k.nx = p->nx;
    k.ny = p->ny;
    k.nz = p->nz;
    k.nsites = p->nx * p->ny * p->nz;
    k.stride = unsigned(sz.stride_elems);
    lbk::set_layout(k, p->layout, p->aosoa_len);
    k.A = p->A;
    k.B = p->B;
    k.kappa = p->kappa;
    k.gamma = p->gamma;
    k.omega_f = 1.0 / p->tau_f;
    k.omega_g = 1.0 / p->tau_g;
    k.rho0 = p->rho0;
    k.force = p->coupling == LB_COUPLING_FORCE;
    k.fd = p->order_param == LB_OP_FD;
    k.mobility = p->gamma * (p->tau_g - 0.5);
    k.xh = p->halo_x ? 2 : 0;
    c->tc = lbk::tile_config(k, p->segment_x, c->fp32);
    *out = c;
    return LB_OK;
}

void lb_destroy(lb_ctx* ctx) { delete ctx; }

lb_status lb_set_stream(lb_ctx* ctx, void* hip_stream)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return LB_OK;
}

lb_status lb_init_phi(lb_ctx* ctx, const double* phi0_dev)
{
    if (!ctx || !phi0_dev) return fail(LB_EINVAL, "ctx and phi0_dev are required");
    ctx->cur = 0;
    hipError_t e = ctx->kp.fd
                       ? lbk::launch_fd_init(ctx->kp, ctx->fp32, ctx->b.state[0], phi0_dev, ctx->stream)
                       : lbk::launch_init(ctx->kp, ctx->fp32, ctx->b.state[0], phi0_dev, ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_init_phi");
}

// One step from src to dst with the context's scheme.
static hipError_t one_step(lb_ctx* ctx, const void* src, void* dst, double* sums_dev,
                           double* phi_src_out = nullptr, double* part = nullptr)
{
    double* work = static_cast<double*>(ctx->b.phi);
    if (!part) part = static_cast<double*>(ctx->b.scratch);
    if (ctx->kp.fd)
        return lbk::launch_fd_step(ctx->kp, ctx->tc, ctx->fp32, ctx->p.kernel, src, dst, work, part,
                                   sums_dev, ctx->stream);
    return lbk::launch_step(ctx->kp, ctx->tc, ctx->fp32, ctx->p.kernel, src, dst, work, part,
                            sums_dev, phi_src_out, ctx->stream);
}

static lb_status step_n(lb_ctx* ctx, int32_t nsteps, double* sums_dev, const char* name,
                        double* part = nullptr)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0 (got %d)", nsteps);
    if (ctx->kp.xh && nsteps > 1)
        return fail(LB_EINVAL, "an x-slab shard advances one step per call (its halo planes "
                               "are exchanged between steps); got nsteps = %d", nsteps);
    for (int32_t t = 0; t < nsteps; t++) {
        hipError_t e = one_step(ctx, ctx->b.state[ctx->cur], ctx->b.state[1 - ctx->cur],
                                sums_dev ? sums_dev + 5 * size_t(t) : nullptr, nullptr, part);
        if (e != hipSuccess) return hip_fail(e, name);
        ctx->cur = 1 - ctx->cur;
    }
    return LB_OK;
}

lb_status lb_step(lb_ctx* ctx, int32_t nsteps) { return step_n(ctx, nsteps, nullptr, "lb_step"); }

lb_status lb_step_sums(lb_ctx* ctx, int32_t nsteps, double* sums_dev)
{
    if (!sums_dev) return fail(LB_EINVAL, "sums_dev is required");
    return step_n(ctx, nsteps, sums_dev, "lb_step_sums");
}

lb_status lb_step_sums_noalloc(lb_ctx* ctx, int32_t nsteps, double* sums_dev)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (!sums_dev) return fail(LB_EINVAL, "sums_dev is required");
    if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0 (got %d)", nsteps);
    // the partial blocks this context's steps reduce over
    const size_t need = size_t(ctx->kp.fd ? lbk::fd_sums_blocks(ctx->kp, ctx->tc, ctx->p.kernel)
                                          : lbk::step_sums_blocks(ctx->kp, ctx->tc, ctx->p.kernel));
    if (need > size_t(LB_NOALLOC_MAX_PARTIALS))
        return fail(LB_EINVAL, "lb_step_sums_noalloc: this lattice reduces over %zu partial "
                               "blocks, the library's array holds %d (use lb_step_sums)",
                    need, LB_NOALLOC_MAX_PARTIALS);
    double* part = nullptr;
    lb_status st = noalloc_scratch(ctx, &part);
    if (st != LB_OK) return st;
    return step_n(ctx, nsteps, sums_dev, "lb_step_sums_noalloc", part);
}

lb_status lb_step_from(lb_ctx* ctx, const void* src_dev, void* dst_dev)
{
    if (!ctx || !src_dev || !dst_dev) return fail(LB_EINVAL, "ctx, src_dev and dst_dev are required");
    if (src_dev == dst_dev) return fail(LB_EINVAL, "src_dev and dst_dev must differ");
    if (!aligned(src_dev) || !aligned(dst_dev))
        return fail(LB_EALIGN, "src_dev and dst_dev must be 256-byte aligned");
    hipError_t e = one_step(ctx, src_dev, dst_dev, nullptr);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_step_from");
}

lb_status lb_step_from_phi(lb_ctx* ctx, const void* src_dev, void* dst_dev, double* phi_dev)
{
    if (!ctx || !phi_dev) return fail(LB_EINVAL, "ctx and phi_dev are required");
    if (ctx->kp.xh) return fail(LB_ESTATE, "lb_step_from_phi is not available on a shard");
    if (ctx->kp.fd)
        return fail(LB_EINVAL, "lb_step_from_phi is for LB_OP_LB (LB_OP_FD holds phi in the "
                               "level itself)");
    if (!aligned(phi_dev)) return fail(LB_EALIGN, "phi_dev is not 256-byte aligned");
    if (!src_dev || !dst_dev) return fail(LB_EINVAL, "src_dev and dst_dev are required");
    if (src_dev == dst_dev) return fail(LB_EINVAL, "src_dev and dst_dev must differ");
    if (!aligned(src_dev) || !aligned(dst_dev))
        return fail(LB_EALIGN, "src_dev and dst_dev must be 256-byte aligned");
    hipError_t e = one_step(ctx, src_dev, dst_dev, nullptr, phi_dev);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_step_from_phi");
}

// Moments of the current level, and block partials of its sums in scratch.
static hipError_t moments(lb_ctx* ctx, double* rho, double* u, double* phi, int* nb)
{
    double* part = static_cast<double*>(ctx->b.scratch);
    if (ctx->kp.fd)
        return lbk::launch_fd_moments(ctx->kp, ctx->fp32, ctx->b.state[ctx->cur], rho, u, phi, part,
                                      nb, ctx->stream);
    return lbk::launch_moments(ctx->kp, ctx->fp32, ctx->b.state[ctx->cur], rho, u, phi,
                               static_cast<double*>(ctx->b.phi), part, nb, ctx->stream);
}

lb_status lb_moments(lb_ctx* ctx, double* rho_dev, double* u_dev, double* phi_dev)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    int nb = 0;
    hipError_t e = moments(ctx, rho_dev, u_dev, phi_dev, &nb);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_moments");
}

lb_status lb_sums(lb_ctx* ctx, double* out5_dev)
{
    if (!ctx || !out5_dev) return fail(LB_EINVAL, "ctx and out5_dev are required");
    int nb = 0;
    double* part = static_cast<double*>(ctx->b.scratch);
    hipError_t e = moments(ctx, nullptr, nullptr, nullptr, &nb);
    if (e != hipSuccess) return hip_fail(e, "lb_sums (partials)");
    e = lbk::launch_sums_final(part, nb, 5, out5_dev, false, ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_sums (final)");
}

lb_status lb_get_state(lb_ctx* ctx, void* dst_dev)
{
    if (!ctx || !dst_dev) return fail(LB_EINVAL, "ctx and dst_dev are required");
    hipError_t e = hipMemcpyAsync(dst_dev, ctx->b.state[ctx->cur], ctx->sz.state_bytes,
                                  hipMemcpyDeviceToDevice, ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_get_state");
}

lb_status lb_set_state(lb_ctx* ctx, const void* src_dev)
{
    if (!ctx || !src_dev) return fail(LB_EINVAL, "ctx and src_dev are required");
    hipError_t e = hipMemcpyAsync(ctx->b.state[ctx->cur], src_dev, ctx->sz.state_bytes,
                                  hipMemcpyDeviceToDevice, ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_set_state");
}

lb_status lb_export_dist(lb_ctx* ctx, double* f_dev, double* g_dev)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (ctx->kp.fd && g_dev) return fail(LB_EINVAL, "LB_OP_FD has no g: g_dev must be NULL");
    if (!f_dev && !g_dev) return LB_OK;
    hipError_t e = ctx->kp.fd ? lbk::launch_fd_export(ctx->kp, ctx->fp32, ctx->b.state[ctx->cur],
                                                      f_dev, ctx->stream)
                              : lbk::launch_export(ctx->kp, ctx->fp32, ctx->b.state[ctx->cur],
                                                   f_dev, g_dev, ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_export_dist");
}

lb_status lb_import_dist(lb_ctx* ctx, const double* f_dev, const double* g_dev)
{
    if (!ctx || !f_dev) return fail(LB_EINVAL, "ctx and f_dev are required");
    if (ctx->kp.xh)
        return fail(LB_ESTATE, "a shard cannot import post-propagation values: the populations "
                               "leaving it are its neighbours'");
    hipError_t e;
    if (ctx->kp.fd) {
        if (g_dev) return fail(LB_EINVAL, "LB_OP_FD has no g: g_dev must be NULL");
        e = lbk::launch_fd_import(ctx->kp, ctx->fp32, ctx->b.state[ctx->cur], f_dev, ctx->stream);
    } else {
        if (!g_dev) return fail(LB_EINVAL, "g_dev is required");
        e = lbk::launch_import(ctx->kp, ctx->fp32, ctx->b.state[ctx->cur], f_dev, g_dev,
                               ctx->stream);
    }
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_import_dist");
}

lb_status lb_adjoint_seed(lb_ctx* ctx, const double* dphi_dev)
{
    if (!ctx || !dphi_dev) return fail(LB_EINVAL, "ctx and dphi_dev are required");
    if (!ctx->has_adj) return fail(LB_ESTATE, "context was created without adjoint buffers");
    if (ctx->p.kernel == LB_KERNEL_STREAM)
        return fail(LB_ESTATE, "LB_KERNEL_STREAM (free streaming) has no reverse mode");
    if (ctx->kp.xh) return fail(LB_ESTATE, "x-slab shards have no reverse mode");
    ctx->adj_cur = 0;
    hipError_t e = lbk::launch_adj_seed(ctx->kp, ctx->fp32, ctx->b.adj[0], ctx->b.adj[1], dphi_dev,
                                        ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_adjoint_seed");
}

static lb_status adjoint_step(lb_ctx* ctx, const void* state_t_dev, const double* phi_t_dev,
                              double* dtheta3_dev);

lb_status lb_adjoint_step(lb_ctx* ctx, const void* state_t_dev, double* dtheta3_dev)
{
    return adjoint_step(ctx, state_t_dev, nullptr, dtheta3_dev);
}

lb_status lb_adjoint_step_phi(lb_ctx* ctx, const void* state_t_dev, const double* phi_t_dev,
                              double* dtheta3_dev)
{
    if (!ctx || !phi_t_dev) return fail(LB_EINVAL, "ctx and phi_t_dev are required");
    if (ctx->kp.fd) return fail(LB_EINVAL, "lb_adjoint_step_phi is for LB_OP_LB");
    if (!aligned(phi_t_dev)) return fail(LB_EALIGN, "phi_t_dev is not 256-byte aligned");
    return adjoint_step(ctx, state_t_dev, phi_t_dev, dtheta3_dev);
}

static lb_status adjoint_step(lb_ctx* ctx, const void* state_t_dev, const double* phi_t_dev,
                              double* dtheta3_dev)
{
    if (!ctx || !state_t_dev) return fail(LB_EINVAL, "ctx and state_t_dev are required");
    if (!ctx->has_adj) return fail(LB_ESTATE, "context was created without adjoint buffers");
    if (ctx->p.kernel == LB_KERNEL_STREAM)
        return fail(LB_ESTATE, "LB_KERNEL_STREAM (free streaming) has no reverse mode");
    if (ctx->kp.xh) return fail(LB_ESTATE, "x-slab shards have no reverse mode");
    if (!aligned(state_t_dev)) return fail(LB_EALIGN, "state_t_dev is not 256-byte aligned");
    double* part = static_cast<double*>(ctx->b.scratch);
    // FD scheme: phi is part of the level
    hipError_t e =
        ctx->kp.fd ? lbk::launch_fd_adj_step(ctx->kp, ctx->fp32, state_t_dev,
                                             static_cast<double*>(ctx->b.phi),
                                             ctx->b.adj[ctx->adj_cur], ctx->b.adj[1 - ctx->adj_cur],
                                             ctx->b.adj_scratch, part, dtheta3_dev, ctx->stream)
                   : lbk::launch_adj_step(ctx->kp, ctx->fp32, state_t_dev, phi_t_dev,
                                          static_cast<double*>(ctx->b.phi),
                                          ctx->b.adj[ctx->adj_cur], ctx->b.adj[1 - ctx->adj_cur],
                                          ctx->b.adj_scratch, part, dtheta3_dev, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "lb_adjoint_step");
    ctx->adj_cur = 1 - ctx->adj_cur;
    return LB_OK;
}

lb_status lb_adjoint_phi0(lb_ctx* ctx, double* dphi0_dev)
{
    if (!ctx || !dphi0_dev) return fail(LB_EINVAL, "ctx and dphi0_dev are required");
    if (!ctx->has_adj) return fail(LB_ESTATE, "context was created without adjoint buffers");
    hipError_t e = lbk::launch_adj_phi0(ctx->kp, ctx->fp32, ctx->b.adj[ctx->adj_cur], dphi0_dev,
                                        ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_adjoint_phi0");
}

static lb_status faces(lb_ctx* ctx, void* lo, void* hi, bool pack, const char* name)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (!ctx->kp.xh) return fail(LB_ESTATE, "%s: the context is not an x-slab shard", name);
    if ((lo && !aligned(lo)) || (hi && !aligned(hi)))
        return fail(LB_EALIGN, "%s: face buffers must be 256-byte aligned", name);
    if (lo && lo == hi) return fail(LB_EINVAL, "%s: the two face buffers alias", name);
    const int nx = ctx->p.nx;
    void* st = ctx->b.state[ctx->cur];
    hipError_t e = hipSuccess;
    // packed: the face sent down (planes 0 and 1, c_x = -1) and the one sent
    // up (planes nx-1 and nx-2, c_x = +1); unpacked: the lower neighbour's
    // upward face into planes -1 and -2, the upper one's downward face into
    // planes nx and nx+1
    if (lo) e = lbk::launch_face(ctx->kp, ctx->fp32, st, lo, pack ? -1 : +1, pack ? 0 : -1, pack,
                                 ctx->stream);
    if (e == hipSuccess && hi)
        e = lbk::launch_face(ctx->kp, ctx->fp32, st, hi, pack ? +1 : -1, pack ? nx - 1 : nx, pack,
                             ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, name);
}

lb_status lb_pack_faces(lb_ctx* ctx, void* send_lo_dev, void* send_hi_dev)
{
    return faces(ctx, send_lo_dev, send_hi_dev, true, "lb_pack_faces");
}

lb_status lb_unpack_faces(lb_ctx* ctx, const void* recv_lo_dev, const void* recv_hi_dev)
{
    return faces(ctx, const_cast<void*>(recv_lo_dev), const_cast<void*>(recv_hi_dev), false,
                 "lb_unpack_faces");
}

lb_status lb_adjoint_export(lb_ctx* ctx, double* df_dev, double* dg_dev)
{
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (!ctx->has_adj) return fail(LB_ESTATE, "context was created without adjoint buffers");
    if (ctx->kp.fd && dg_dev) return fail(LB_EINVAL, "LB_OP_FD has no g: dg_dev must be NULL");
    if ((df_dev && !aligned(df_dev)) || (dg_dev && !aligned(dg_dev)))
        return fail(LB_EALIGN, "df_dev and dg_dev must be 256-byte aligned");
    if (!df_dev && !dg_dev) return LB_OK;
    hipError_t e = lbk::launch_adj_export(ctx->kp, ctx->fp32, ctx->b.adj[ctx->adj_cur], df_dev,
                                          dg_dev, ctx->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "lb_adjoint_export");
}

}  // extern "C"
