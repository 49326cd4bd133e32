/*
 * lb.h -- C ABI of the MI355X (gfx950) D3Q19 binary-fluid lattice-Boltzmann
 * library.
 *
 * One timestep is the Ludwig timestep of Gray & Stratford, "A Lightweight
 * Approach to Performance Portability with targetDP" (Sec. 2.1.1: order
 * parameter gradients, chemical stress, collision, propagation) for a
 * symmetric binary fluid:
 *
 *   phi = sum_i g_i                         order parameter
 *   d_a phi, lap phi                        7-point central differences
 *   mu  = A phi + B phi^3 - kappa lap phi   chemical potential
 *   Pi  = [A/2 phi^2 + 3B/4 phi^4 - kappa phi lap phi - kappa/2 |grad phi|^2] I
 *         + kappa grad phi grad phi         chemical stress
 *   rho = sum_i f_i, j = sum_i f_i c_i, u = j/rho
 *   f_i^eq = w_i [rho + 3 c_i.j + 9/2 Q_i:(Pi + rho u u)]
 *   g_i^eq = w_i [phi + 3 phi c_i.u + 9/2 Q_i:((Gamma mu - phi/3) I + phi u u)]
 *   f_i <- f_i - (f_i - f_i^eq)/tau_f,  g_i <- g_i - (g_i - g_i^eq)/tau_g
 *   f_i(x + c_i, t+1) = f_i*(x, t)          periodic propagation (same for g)
 *
 * with Q_i = c_i c_i - I/3, weights 1/3 (rest), 1/18 (6 faces), 1/36 (12
 * edges).  Velocity order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 =
 * (+x+y),(-x-y),(+x-y),(-x+y),(+x+z),(-x-z),(+x-z),(-x+z),(+y+z),(-y-z),
 * (+y-z),(-y+z).
 *
 * The host call sequence follows the paper's host model (Sec. 3.2.3, Fig. 2:
 * allocate, copy in, launch, synchronise, copy out, reduce): the caller owns
 * every device byte (sized by lb_query_sizes), lb_init_phi is the copy-in,
 * lb_step the launches, lb_moments / lb_sums the copy-out and the reduction
 * (the paper's targetDoubleSum).
 *
 * Conventions shared by every call:
 *  - Public fields are dense C-order arrays of shape (nx, ny, nz): site
 *    (x, y, z) is element (x*ny + y)*nz + z, so z is contiguous.  Vector
 *    fields are three such planes (x, y, z components), distributions 19.
 *  - Pointers named *_dev are device pointers (hipMalloc or torch CUDA
 *    tensors); all other pointers are host pointers.
 *  - Device buffers must be 256-byte aligned (LB_EALIGN otherwise).
 *  - Every call is asynchronous and ordered on the context's HIP stream; the
 *    caller synchronises.  Argument errors are reported synchronously before
 *    anything is launched; launch errors through hipGetLastError (LB_EHIP);
 *    device faults surface at the caller's next synchronisation.
 *  - A context is not reentrant: one context per stream, one thread at a
 *    time.  The library never allocates or frees device memory and keeps only
 *    borrowed pointers, which must outlive the context.
 *  - lb_last_error() returns a thread-local text for the last failure.
 *  - "Passage:" in each declaration names the part of the paper the call
 *    implements.  The reverse mode, the checkpoint calls and the FP32
 *    deviation storage are extensions of this project: the paper has no
 *    adjoint and no reduced-precision storage.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_ABI_VERSION 5
#define LB_NVEL 19

typedef enum {
    LB_OK = 0,
    LB_EINVAL = 1, /* bad argument value (tau <= 1/2, rho0 <= 0, NULL, ...) */
    LB_ESHAPE = 2, /* bad lattice extents                                     */
    LB_EALIGN = 3, /* device pointer not 256-byte aligned                     */
    LB_EHIP = 4,   /* a HIP runtime call or kernel launch failed              */
    LB_ESTATE = 5  /* call not valid in the context's state (e.g. no adjoint) */
} lb_status;

typedef enum {
    LB_FP64 = 0,    /* distributions stored and collided in FP64            */
    LB_FP32_DEV = 1 /* FP32 storage of deviations and FP32 collision:
                       f_i - w_i rho0, and g_i - r_i phi_c, where phi_c is
                       the order parameter of the last collision at the
                       site the population moves TO, truncated to the high
                       32-bit word of its binary64 encoding and stored as
                       that word (r_i phi = the order-parameter equilibrium
                       at rest with mu = 0); FP64 phi, reductions and
                       parameter gradients                                   */
} lb_precision;

typedef enum {
    LB_KERNEL_FUSED = 0,   /* one pass per step: phi, gradients, stress,
                              collision and propagation in one kernel      */
    LB_KERNEL_TWO_PASS = 1, /* a phi pass, then the stencil/collision pass */
    LB_KERNEL_STREAM = 2    /* measurement twin of LB_KERNEL_FUSED: the same
                               kernel, loads, phi sums and stores with the
                               collision left out, i.e. free streaming
                               f_i(x + c_i, t+1) = f_i(x, t) (not a model of
                               the fluid; the memory-bound floor of the
                               fused step; LB_OP_LB with LB_COUPLING_STRESS
                               only, LB_EINVAL otherwise; the reverse-mode
                               calls return LB_ESTATE)                      */
} lb_kernel;

/* How the chemical stress Pi drives the flow (two forms of the same
 * hydrodynamics to leading order): */
typedef enum {
    LB_COUPLING_STRESS = 0, /* Pi in f^eq's second moment (default)         */
    LB_COUPLING_FORCE = 1   /* body force F = -div Pi (central differences)
                               with the half-force velocity u = (j + F/2)/rho
                               and Guo's forcing term; one marching kernel
                               per step (LB_KERNEL_FUSED), or a phi pass and
                               a collision pass (LB_KERNEL_TWO_PASS)        */
} lb_coupling;

/* How the order parameter evolves: */
typedef enum {
    LB_OP_LB = 0, /* the distribution g above (default)                       */
    LB_OP_FD = 1  /* a field phi(x) with a conservative finite-difference
                     Cahn-Hilliard update and upwind advection -- the binary-
                     fluid counterpart of the paper's "Advection" and order-
                     parameter update kernels (Sec. 2.1.1); there is no g.
                     With the flux through the face between x and x + e_a,
                       u_f = (u_a(x) + u_a(x + e_a)) / 2   (u = j/rho of f(t))
                       J_a = u_f * (u_f > 0 ? phi(x) : phi(x + e_a))
                             - M (mu(x + e_a) - mu(x)),
                     phi(x, t+1) = phi(x) - sum_a [J_a(x + e_a/2) - J_a(x - e_a/2)]
                     with M = Gamma (tau_g - 1/2), the mobility of the g
                     scheme; mu and Pi from phi(t).  With LB_COUPLING_STRESS f
                     collides as above with Pi in f^eq; with
                     LB_COUPLING_FORCE (the paper's arrangement) f collides
                     with F = -div Pi and u = (j + F/2)/rho is also the
                     fluxes' velocity.  Either coupling runs as one
                     marching kernel (LB_KERNEL_FUSED) or as a collision
                     pass and a flux pass (LB_KERNEL_TWO_PASS), with
                     bit-identical results.  phi is FP64 in both
                     precisions.                                             */
} lb_order_param;

/* Memory layout of the f and g regions of a time level (opaque to callers,
 * who see dense arrays through lb_export_dist / lb_import_dist; every layout
 * gives bit-identical results).  Element (i, x, y, z), row r = x*ny + y: */
typedef enum {
    LB_LAYOUT_ROWS = 0, /* row-blocked: (r*19 + i)*nz + z (default, fastest)  */
    LB_LAYOUT_SOA = 1,  /* one array per component: i*stride + r*nz + z      */
    LB_LAYOUT_AOS = 2,  /* a site's 19 components together: (r*nz + z)*19 + i */
    LB_LAYOUT_AOSOA = 3 /* blocks of V = aosoa_len z-sites (a power of two
                           dividing nz), 19 components each:
                           (r*nz + (z/V)*V)*19 + i*V + z%V                    */
} lb_layout;

/* Lattice and model.  nx, ny, nz >= 1 (periodic in all three directions),
 * N = nx*ny*nz below ~1.1e8 sites (39 * stride_elems < 2^32) and one x-plane
 * of f below 4 GiB (ny*nz*19*elem_bytes < 2^32), else LB_ESHAPE;
 * tau_f, tau_g > 1/2; rho0 > 0.
 *
 * halo_x = 1 makes the lattice one x-slab shard of a larger one (the paper's
 * domain decomposition, Sec. 2.1.1 and Sec. 5): x is not periodic, and each
 * time level also holds halo planes that the step reads instead of a wrap,
 * filled from the neighbouring shards through lb_pack_faces /
 * lb_unpack_faces before every step (see there).  Shards need nx >= 2,
 * LB_OP_LB, LB_COUPLING_STRESS and LB_KERNEL_FUSED or LB_KERNEL_STREAM
 * (LB_EINVAL otherwise); lb_step advances one step per call (nsteps <= 1);
 * lb_import_dist, lb_step_from_phi and the reverse mode return LB_ESTATE;
 * lb_init_phi's phi0 holds nx + 2 planes (see there).  Measured and tested
 * on one GPU; the exchange between GPUs is the caller's. */
typedef struct {
    int32_t nx, ny, nz;
    double A, B, kappa; /* free energy A/2 phi^2 + B/4 phi^4 + kappa/2 |grad phi|^2 */
    double gamma;       /* mobility parameter Gamma in g^eq                         */
    double tau_f, tau_g;
    double rho0;        /* rest density of the initial state                        */
    int32_t precision;  /* lb_precision                                             */
    int32_t kernel;     /* lb_kernel (same results; a performance choice)           */
    int32_t segment_x;  /* planes per workgroup in the fused kernel; <= 0: automatic */
    int32_t layout;     /* lb_layout of the distributions                           */
    int32_t aosoa_len;  /* V for LB_LAYOUT_AOSOA (ignored otherwise)                */
    int32_t coupling;   /* lb_coupling                                              */
    int32_t order_param; /* lb_order_param                                          */
    int32_t halo_x;     /* 0: periodic in x; 1: an x-slab shard (halo planes)        */
} lb_params;

/* Sizes in bytes of the caller-owned device buffers (lb_query_sizes). */
typedef struct {
    size_t elem_bytes;        /* 8 (LB_FP64) or 4 (LB_FP32_DEV)                         */
    size_t stride_elems;      /* padded elements per component of a distribution        */
    size_t state_bytes;       /* one time level: f, g (2*19*stride elements) and, in
                                 LB_FP32_DEV, phi_c (stride 32-bit words); LB_OP_FD:
                                 f (19*stride elements), then phi (stride FP64)        */
    size_t phi_bytes;         /* FP64 work fields of stride values each: phi;
                                 LB_OP_FD: mu, u_x, u_y, u_z                           */
    size_t scratch_bytes;     /* reduction partials                                     */
    size_t adj_bytes;         /* one adjoint time level (lambda_f, lambda_g, lambda_phi) */
    size_t adj_scratch_bytes; /* adjoint stencil cotangents (5 fields; 8 with the force
                                 coupling, which adds dL/dF)                         */
    size_t face_bytes;        /* one face buffer of an x-slab shard (0 when periodic)    */
} lb_sizes;

/* Caller-owned device memory.  state[0..1] are the two time levels the step
 * ping-pongs between; the adjoint buffers may be NULL if lb_adjoint_* is never
 * called. */
typedef struct {
    void *state[2];
    void *phi;
    void *scratch;
    void *adj[2];
    void *adj_scratch;
} lb_buffers;

typedef struct lb_ctx lb_ctx;

/* Library ABI version (LB_ABI_VERSION).  Passage: none (this library's own
 * versioning). */
int32_t lb_abi_version(void);

/* Buffer sizes for the given parameters.  Host only; launches nothing.
 * Returns LB_ESHAPE / LB_EINVAL for parameters lb_create would reject.
 * Passage: Sec. 3.2.3, Fig. 2 (targetMalloc): the caller allocates the
 * target's memory; this call says how much. */
lb_status lb_query_sizes(const lb_params *p, lb_sizes *out);

/* Create a context on the current HIP device, bound to hip_stream (a
 * hipStream_t; NULL = the null stream).  Copies *p and *b.  The state is
 * undefined until lb_init_phi, lb_set_state or lb_import_dist.
 * Passage: Sec. 3.2.3, Fig. 2 (copyConstToTarget for the model constants;
 * target pointers handed to the target functions): the context holds the
 * constants and the caller's target pointers. */
lb_status lb_create(const lb_params *p, const lb_buffers *b, void *hip_stream, lb_ctx **out);

/* Free the host-side context (never the caller's device memory). NULL is a no-op.
 * Passage: Sec. 3.2.3, Fig. 2 (targetFree) -- the caller frees the device
 * memory it allocated; this frees only what lb_create allocated on the host. */
void lb_destroy(lb_ctx *ctx);

/* Rebind the context to another stream.  Passage: Sec. 3.2.3 (a
 * __targetLaunch__ is asynchronous until targetSynchronize): every call is
 * ordered on this stream and the caller synchronises. */
lb_status lb_set_stream(lb_ctx *ctx, void *hip_stream);

/* Initial state from phi0_dev (FP64, nx*ny*nz): rho = rho0 and u = 0
 * (f_i = w_i rho0), all of phi0 in the rest population (g_0 = phi0,
 * g_i = 0 for i > 0; LB_OP_FD: the field phi = phi0).  Resets the time-level
 * index.  An x-slab shard takes phi0 of nx + 2 planes: plane -1 (the lower
 * neighbour's last), the shard's nx planes, plane nx (the upper neighbour's
 * first).  Passage: Sec. 3.2.3, Fig. 2 (copyToTarget) for the hand-over of
 * phi0; the state built from it is this library's reading (the paper gives
 * no initial condition for this model). */
lb_status lb_init_phi(lb_ctx *ctx, const double *phi0_dev);

/* Advance nsteps >= 0 timesteps (asynchronous).  Passage: Sec. 2.1.1 (the
 * Ludwig timestep: order parameter gradients, chemical stress, collision,
 * propagation), each step one or two launches (Fig. 2, __targetLaunch__). */
lb_status lb_step(lb_ctx *ctx, int32_t nsteps);

/* lb_step that also reduces, inside each step, the FP64 conserved sums of
 * the state the step starts from: sums_dev (device, 5*nsteps FP64) receives
 * [sum rho, sum phi, sum j_x, sum j_y, sum j_z] for each step t at
 * sums_dev[5t..5t+4] (the targetDoubleSum of the paper's host model,
 * Sec. 3.2.3; deterministic, as lb_sums).  Passage: Sec. 2.1.1 for the
 * step, Sec. 3.2.3 (targetDoubleSum) for the sums. */
lb_status lb_step_sums(lb_ctx *ctx, int32_t nsteps, double *sums_dev);

/* lb_step_sums for callers that cannot allocate device memory or hand over a
 * workspace (code under HIP graph capture, allocation-free serving loops,
 * harnesses that forbid hipMalloc): the steps' reduction partials go to a
 * device array inside the library instead of the context's scratch buffer;
 * everything else, results included (bit for bit), is lb_step_sums'.  The
 * call allocates nothing.  The array holds LB_NOALLOC_MAX_PARTIALS blocks of
 * 5 FP64 partials (160 KiB), one copy per GPU the library runs on, kept until
 * the process ends; its address on the current GPU is looked up on the first
 * call there.  LB_EINVAL if the context's steps reduce over more blocks
 * than that (every cube up to 479^3 fits, except with LB_OP_FD and
 * LB_KERNEL_TWO_PASS, whose collision pass reduces over one block per 256
 * sites: up to about 1.05e6 sites), LB_ESTATE if the current device is not
 * that of the context's stream.  Every block overwrites its own partials before they are summed,
 * so nothing carries over from an earlier call; but all contexts on one GPU
 * share the one array, so calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  Passage: as
 * lb_step_sums. */
#define LB_NOALLOC_MAX_PARTIALS 4096
lb_status lb_step_sums_noalloc(lb_ctx *ctx, int32_t nsteps, double *sums_dev);

/* One timestep from the caller's time level src_dev to dst_dev (both
 * state_bytes, as written by lb_get_state or a previous lb_step_from),
 * without touching the context's current level.  Used by the reverse mode to
 * recompute the states of a checkpoint segment in place.  src_dev and dst_dev
 * must differ.  Passage: Sec. 2.1.1 (the step); taking the levels from the
 * caller is a project extension for the reverse mode's recomputation. */
lb_status lb_step_from(lb_ctx *ctx, const void *src_dev, void *dst_dev);

/* lb_step_from that also stores phi of src_dev in phi_dev (device, N FP64
 * values in dense (x, y, z) order, 256-byte aligned), as the step forms it
 * (bit-identical to the phi lb_adjoint_step would form), for
 * lb_adjoint_step_phi.  LB_OP_LB only (LB_EINVAL otherwise: LB_OP_FD holds
 * phi in the level).  Passage: none
 * beyond lb_step_from's (a project extension for the reverse mode). */
lb_status lb_step_from_phi(lb_ctx *ctx, const void *src_dev, void *dst_dev, double *phi_dev);

/* Moments of the current (post-propagation) state, as dense FP64 device
 * arrays: rho_dev (N), u_dev (3N: x, y, z planes), phi_dev (N).  Any pointer
 * may be NULL to skip that output.  u = j/rho; with LB_COUPLING_FORCE
 * u = (j + F/2)/rho, F = -div Pi of this state (the velocity the collision
 * uses), and lb_sums' momentum sums are those of rho u likewise.
 * Passage: Sec. 3.2.3, Fig. 2 (copyFromTarget) of the moments of Sec. 2.1.1's
 * fields (order parameter, fluid density and velocity). */
lb_status lb_moments(lb_ctx *ctx, double *rho_dev, double *u_dev, double *phi_dev);

/* Global sums of the current state in FP64, written to out5_dev:
 * [sum rho, sum phi, sum j_x, sum j_y, sum j_z].  Deterministic: fixed
 * per-block order, then one fixed-order pass over the block partials.
 * Passage: Sec. 3.2.3 (targetDoubleSum, the summation of a per-site array). */
lb_status lb_sums(lb_ctx *ctx, double *out5_dev);

/* Copy the current time level (state_bytes, opaque internal layout) to /
 * from a caller buffer: lossless checkpoint and restore.  Passage: none (a
 * project extension: the checkpoints of the reverse mode's rollout); the
 * copies themselves are target-to-target transfers in the sense of
 * Sec. 3.2.3. */
lb_status lb_get_state(lb_ctx *ctx, void *dst_dev);
lb_status lb_set_state(lb_ctx *ctx, const void *src_dev);

/* Current state as dense FP64 post-propagation distributions, each of shape
 * (19, nx, ny, nz); either pointer may be NULL.  LB_OP_FD has no g: g_dev
 * must be NULL (LB_EINVAL).  Passage: Sec. 3.2.3, Fig. 2 (copyFromTarget);
 * the stored layout is internal (Sec. 3.1's choice of layout is made inside
 * the library), the exported one dense. */
lb_status lb_export_dist(lb_ctx *ctx, double *f_dev, double *g_dev);

/* Set the current state from dense FP64 post-propagation distributions
 * (19, nx, ny, nz).  In LB_FP32_DEV phi_c(x) becomes sum_i g_i(x) (truncated
 * as above) and the values are rounded to FP32 after subtracting w_i rho0
 * from f_i and r_i phi_c(x) from g_i(x).  LB_OP_FD: g_dev must be NULL and only f is set
 * (the phi field keeps its values).  Passage: Sec. 3.2.3, Fig. 2
 * (copyToTarget), dense in, internal layout (Sec. 3.1) stored. */
lb_status lb_import_dist(lb_ctx *ctx, const double *f_dev, const double *g_dev);

/* ---- reverse mode ------------------------------------------------------
 * The adjoint carries lambda_t = dL/d(state at time t) in the context's
 * adjoint buffers (FP64 in LB_FP64, FP32 in LB_FP32_DEV).  A level is 39
 * components of stride_elems elements each, sites in dense (x, y, z) order:
 * components 0..18 hold dL/df_i of the post-propagation populations (FP32
 * storage: of the deviations, the same values), 19..37 the parts lg_i
 * specific to each g_i and 38 lp, with dL/dg_i = lg_i + lp (LB_OP_LB), or
 * lp = dL/dphi (LB_OP_FD).  After lb_adjoint_seed the level is adj[0]; each
 * reverse step moves it to the other buffer.  For a loss on the final order
 * parameter:
 *   lb_adjoint_seed(dL/dphi_T)  then, for t = T-1 .. 0,
 *   lb_adjoint_step(state_t)    (state_t as saved by lb_get_state at time t;
 *                                or lb_adjoint_step_phi with its phi too)
 * and lb_adjoint_phi0 gives dL/dphi0.  Requires adj[0], adj[1] and
 * adj_scratch (LB_ESTATE otherwise); covers both couplings and both
 * order-parameter schemes.  With LB_OP_FD the level holds dL/df_i and
 * dL/dphi (the g components of adj_bytes are unused), and the upwind choice
 * of each face is held fixed: at a face velocity of exactly zero the
 * derivative taken is that of the phi(x + e_a) branch, the one the forward
 * step takes.
 *
 * Passage for every call of this block: none -- the reverse mode is a
 * project extension (the paper differentiates nothing).  lambda lives in the
 * two context-held levels adj[0], adj[1] rather than in caller arguments of
 * each step: a level's layout (39 padded components) is internal, like a
 * time level's, so callers seed it (lb_adjoint_seed), step it, and read it
 * through dense copies (lb_adjoint_export, lb_adjoint_phi0). */

/* lambda_T from dphi_dev = dL/dphi_T (FP64, N): dL/df_i = 0; LB_OP_LB:
 * dL/dg_i = dphi for every i; LB_OP_FD: dL/dphi = dphi.  With tau_g = 1 the
 * g-specific part of every later level is zero (g* = g^eq): the seed zeroes
 * it in both adjoint buffers and the reverse steps neither read nor write
 * it. */
lb_status lb_adjoint_seed(lb_ctx *ctx, const double *dphi_dev);

/* One reverse step: lambda_t = J(state_t)^T lambda_{t+1}, where J is the
 * Jacobian of one timestep at state_t (state_bytes buffer from lb_get_state).
 * dtheta3_dev (FP64[3], device) is incremented by the step's contribution to
 * [dL/dA, dL/dB, dL/dkappa]; it may be NULL. */
lb_status lb_adjoint_step(lb_ctx *ctx, const void *state_t_dev, double *dtheta3_dev);

/* lb_adjoint_step with phi of state_t_dev given (phi_t_dev, as stored by
 * lb_step_from_phi from state_t_dev), so that no phi pass runs; the result
 * is identical to lb_adjoint_step's only if phi_t_dev really is that field.
 * LB_OP_LB only (LB_EINVAL otherwise: LB_OP_FD holds phi in the level). */
lb_status lb_adjoint_step_phi(lb_ctx *ctx, const void *state_t_dev, const double *phi_t_dev,
                              double *dtheta3_dev);

/* dL/dphi0 (FP64, N) of the initial state built by lb_init_phi, from the
 * current lambda_0. */
lb_status lb_adjoint_phi0(lb_ctx *ctx, double *dphi0_dev);

/* The current adjoint level as dense FP64 device arrays of shape
 * (19, nx, ny, nz): df_dev[i] = dL/df_i and (LB_OP_LB) dg_dev[i] = dL/dg_i =
 * lg_i + lp, both with respect to the post-propagation populations of the
 * state the level belongs to (FP32 storage: of the stored deviations, the
 * same values).  Either pointer may be NULL; with LB_OP_FD dg_dev must be
 * NULL (LB_EINVAL: there is no g; dL/dphi is lb_adjoint_phi0's output).
 * Caller-owned, 256-byte aligned (LB_EALIGN), 19*N FP64 values each;
 * LB_ESTATE without adjoint buffers. */
lb_status lb_adjoint_export(lb_ctx *ctx, double *df_dev, double *dg_dev);

/* ---- x-slab shards (halo_x = 1) ---------------------------------------
 * Passage: Sec. 2.1.1 (each sub-domain of the decomposed lattice is
 * surrounded by a halo region filled from its neighbours) and Sec. 5 (the
 * decomposed runs).  Before every step of a shard:
 *   lb_pack_faces(ctx, send_lo, send_hi);         this shard's two faces
 *   (send_lo to the lower neighbour, send_hi to the upper one; receive the
 *    lower neighbour's send_hi as recv_lo, the upper one's send_lo as recv_hi)
 *   lb_unpack_faces(ctx, recv_lo, recv_hi);       into the halo planes
 *   lb_step(ctx, 1);
 * (once more before lb_moments, lb_sums or lb_export_dist, which read the
 * halo planes of the current level too).  A face carries, for the
 * populations moving across it, f and g of the boundary plane, the g that
 * form phi at the neighbour's boundary plane (its stencil neighbour) and,
 * in LB_FP32_DEV, that plane's phi_c: 24 * ny * nz values of the storage
 * type (+ ny * nz 32-bit words), face_bytes bytes; the layout is internal and the
 * buffers are opaque.  A shard that receives its own faces (recv_lo =
 * send_hi, recv_hi = send_lo) steps exactly like the periodic lattice of
 * the same extents, bit for bit.  Buffers are device memory of face_bytes,
 * 256-byte aligned (LB_EALIGN); either pointer may be NULL to skip that
 * face; LB_ESTATE on a periodic context. */
lb_status lb_pack_faces(lb_ctx *ctx, void *send_lo_dev, void *send_hi_dev);
lb_status lb_unpack_faces(lb_ctx *ctx, const void *recv_lo_dev, const void *recv_hi_dev);

/* ---- measurement ------------------------------------------------------ */

/* Streaming copy of `bytes` (a multiple of 16) from src_dev to dst_dev on
 * hip_stream: the practical HBM ceiling the step is measured against (the
 * STREAM calibration of the paper's roofline analysis, Sec. 4).  Buffers must
 * be 256-byte aligned and must not overlap. */
lb_status lb_copy_probe(const void *src_dev, void *dst_dev, size_t bytes, void *hip_stream);

/* Text for a status code, and the thread-local detail of the last failure.
 * Passage: none (this library's error reporting). */
const char *lb_status_string(lb_status s);
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
