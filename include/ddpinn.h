/*
 * ddpinn.h -- C ABI of the MI355X (gfx950) fused subdomain training step for
 * domain-decomposed physics-informed neural networks (arXiv 2602.15883).
 *
 * One context holds one or more subdomain networks ("local experts",
 * section 2.2) of the same architecture: a fully connected tanh MLP
 * (x_1..x_d, t) -> (u_1..u_d, p) with H hidden layers of width W <= 256 (see pinn_config.width)
 * (section 2.1, network equation).  A training step evaluates, for every
 * subdomain at once in one grouped launch,
 *
 *   L = lam_obs L_obs + lam_PDE L_PDE + lam_gh_u L_gh_u
 *       + lam_gh_p^space L_gh_p^space + lam_gh_p^time L_gh_p^time + lam_anc L_anc
 *
 * (section 2.2, final local objective, plus the optional reference-anchor
 * pressure term L_anc; lam_gh_p^space is forced to 0 on master subdomains,
 * section 2.2 decoupled asymmetric weighting), its exact gradient, and one
 * Adam update (Algorithm 1, optimizer step), optionally after global-norm
 * gradient clipping and with a step-decayed learning rate (the 3D cylinder
 * recipe of section 3.3 and appendix B).  L_PDE is the mean squared
 * incompressible Navier-Stokes residual (section 2.1, residuals r1-r4);
 * every MSE sums over components and divides by the number of points; both
 * ghost pressure parts divide by the subdomain's total ghost count.
 *
 * Conventions for every entry point
 *   - All array pointers are DEVICE pointers, caller-owned, and must stay
 *     valid for the life of the context.  The library never allocates device
 *     memory: the caller passes a workspace sized by pinn_create's size query.
 *   - Points are float32 row-major [n][d+1] = (x_1..x_d, t).
 *   - Parameters are packed float32: W1[W][d+1], b1[W], W2[W][W], b2[W], ...,
 *     W_{H+1}[d+1][W], b_{H+1}[d+1]  (row-major [out][in]).
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Calls are stream-ordered and asynchronous unless stated otherwise.
 *   - Errors are returned as status codes; nothing aborts or throws across
 *     the ABI.  Argument errors return PINN_E_INVAL before any work is
 *     enqueued.  pinn_last_error() gives a message for the calling thread.
 */
#ifndef DDPINN_H
#define DDPINN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pinn_ctx pinn_ctx;

typedef enum {
  PINN_OK = 0,
  PINN_E_INVAL = -1,        /* bad argument (nothing was enqueued)            */
  PINN_E_NOMEM = -2,        /* workspace or scratch too small                 */
  PINN_E_DEVICE = -3,       /* a HIP runtime call failed                      */
  PINN_E_BUDGET = -4,       /* query larger than the configured point budget  */
  PINN_E_NONFINITE = -5,    /* PINN_CHECK_FINITE: a loss was NaN or Inf       */
  PINN_E_UNSUPPORTED = -6   /* configuration outside what the kernels cover   */
} pinn_status;

/* pinn_config.flags */
#define PINN_GRAPH 1u          /* capture the step (prep, fused, reduce+Adam)
                                  as one hipGraph at create and replay it     */

/* pinn_step flags */
#define PINN_NO_UPDATE 1u      /* compute loss and gradient, leave theta/m/v  */
#define PINN_CHECK_FINITE 2u   /* synchronize; PINN_E_NONFINITE if any loss
                                  is not finite                               */
#define PINN_PER_SUBDOMAIN 4u  /* one plain launch of the fused kernel per
                                  subdomain instead of the grouped launch
                                  (same results; for comparison)             */
#define PINN_TIME_KERNEL 8u    /* run the step without the graph, launching
                                  the fused kernel with HIP events tied to
                                  the dispatch (its start and end time
                                  stamps, kernel execution only); see
                                  pinn_kernel_time                            */

/* pinn_query `what` */
#define PINN_Q_VALUE 0u        /* out[n][d+1]   = (u_1..u_d, p)                */
#define PINN_Q_UVPW 1u         /* 2D only: out[n][4] = (u, v, p, v_x - u_y)   */
#define PINN_Q_CHANNELS 2u     /* out[n][2d+2][d+1]: value, d/dx_j, d/dt,
                                  d2/dx_j^2 of every output                   */
#define PINN_Q_RESIDUAL 3u     /* out[n][d+1]: Navier-Stokes residuals r_1..r_{d+1} */

typedef struct {
  int32_t dim;            /* 2 or 3 spatial dimensions                        */
  int32_t width;          /* W, 1..256.  Above 128 each wave of a workgroup
                             owns two 16-neuron row blocks; where the tile's
                             activation stacks do not fit in LDS (2D above
                             176, 3D above 144), the step keeps one forward
                             stack and runs the backward over column halves */
  int32_t depth;          /* H hidden layers, 1..16                           */
  int32_t n_sub;          /* number of subdomains, 1..4096                    */
  int32_t activation;     /* 0 = tanh, 1 = sin (the paper's cylinder networks) */
  uint32_t flags;         /* PINN_GRAPH                                       */
  double nu;              /* kinematic viscosity 1/Re                         */
  float lam[6];           /* obs, PDE, gh_u, gh_p^space, gh_p^time, anchor    */
  float lr, beta1, beta2, eps;   /* Adam                                      */
  int32_t tile_points;    /* collocation points per tile: 16 or 32; 0 means
                             16.  The shapes measured fastest per network
                             are in the package's tuning table (tune.py)   */
  int32_t blocks_per_cu;  /* persistent workgroups per CU: 0 = occupancy max  */
  int64_t max_query_points; /* largest n accepted by pinn_query (routing)     */
  float comp_w[3];        /* weights of the velocity components in L_obs and
                             L_gh_u (section 3.3 uses 1, 5, 100); all zero
                             means all ones                                   */
  float clip_norm;        /* clip each subdomain's gradient to this global L2
                             norm before Adam (section 3.3: 1.0); 0 = off     */
  float lr_factor;        /* step decay: lr_t = lr * lr_factor^floor((t-1) /  */
  int32_t lr_interval;    /*   lr_interval) (appendix B); interval 0 = off    */
  int32_t gemm_priority_off; /* launch knob: 0 = the younger half of each
                             workgroup's waves raises its priority for its
                             GEMMs (default), 1 = all waves at one priority */
  int32_t ranges_per_wg;  /* launch knob: item ranges per persistent
                             workgroup when several workgroups share a
                             compute unit (taken in turn); 0 = 4, 1..64     */
  int32_t guard_bytes;    /* memory-check mode: 0 = off; else a multiple of
                             256 up to 1 MiB left after every region of the
                             workspace and filled with a pattern at create;
                             pinn_check_guards counts the bytes a kernel
                             overwrote there.  The workspace grows by this
                             much per region                                */
} pinn_config;

typedef struct {
  float lo[4], hi[4];     /* interior box (x_1..x_d, t), half-open [lo, hi);
                             used by query routing                            */
  int32_t is_master;      /* box holds the anchor: lam_gh_p^space := 0         */
  float *theta;           /* [P] parameters, updated in place by Adam         */
  float *adam_m, *adam_v; /* [P] Adam moments, updated in place               */
  const float *pde_x;   int64_t n_pde;   /* collocation points [n_pde][d+1]   */
  const float *obs_x;                    /* observation points [n_obs][d+1]   */
  const float *obs_u;   int64_t n_obs;   /* observed velocity  [n_obs][d]     */
  const float *gh_x;                     /* ghost points       [n_gh][d+1]    */
  const float *gh_up;                    /* neighbour (u, p)   [n_gh][d+1]    */
  const uint8_t *gh_kind; int64_t n_gh;  /* 0 spatial, 1 temporal interface   */
  const float *anc_x;                    /* anchor points      [n_anc][d+1]   */
  const float *anc_p;   int64_t n_anc;   /* anchor pressure    [n_anc]        */
} pinn_subdomain;

/* Number of parameters P of one subdomain network. */
int64_t pinn_num_params(int32_t dim, int32_t width, int32_t depth);

/*
 * Create a context (section 2.2 domain decomposition: one local expert per
 * subdomain).  With workspace == NULL this is a size query: it validates the
 * arguments, writes the required workspace size to *workspace_bytes and
 * creates nothing.  Otherwise `workspace` is a device buffer of at least
 * *workspace_bytes bytes, 256-byte aligned, owned by the caller.  The
 * subdomain descriptors are copied; the arrays they point to are not.
 * Synchronizes `stream`.  Returns PINN_E_UNSUPPORTED for widths, depths or
 * dimensions the kernels do not cover.
 */
pinn_status pinn_create(const pinn_config *cfg, const pinn_subdomain *subs,
                        void *workspace, size_t *workspace_bytes,
                        void *stream, pinn_ctx **out);

/*
 * One training step for every subdomain (Algorithm 1 loop body): forward with
 * derivative channels, residuals, losses, hand-written adjoint, gradient
 * reduction and, unless PINN_NO_UPDATE, Adam at step t (1-based) in place on
 * theta, adam_m, adam_v.
 *   loss_out: device [n_sub][7] = {L_obs, L_PDE, L_gh_u, L_gh_p^space,
 *             L_gh_p^time, L_anc, L} (terms unweighted, L weighted), or NULL.
 *   grad_out: device [n_sub][P] gradient dL/dtheta (before clipping), or NULL.
 * The gradient sum is deterministic: the same inputs give bitwise the same
 * results on the same device and launch configuration.
 */
pinn_status pinn_step(pinn_ctx *ctx, int64_t t, uint32_t flags,
                      float *loss_out, float *grad_out, void *stream);

/*
 * Bytes of device scratch pinn_query needs for n routed points.
 */
size_t pinn_query_scratch_bytes(const pinn_ctx *ctx, int64_t n);

/*
 * Evaluate the networks at points x[n][d+1] (section 3, stitching of local
 * experts).  sub >= 0 evaluates subdomain `sub` at every point; sub == -1
 * routes each point to the subdomain whose half-open box contains it (the
 * global upper face counts as inside) and needs `scratch` of
 * pinn_query_scratch_bytes(ctx, n) bytes; points in no box give NaN.
 * Read-only on the parameters: queries on different streams with their own
 * scratch may overlap; a query must not overlap a pinn_step of the same
 * context.  n <= cfg.max_query_points when routing, else PINN_E_BUDGET.
 */
pinn_status pinn_query(pinn_ctx *ctx, const float *x, int64_t n, int32_t sub,
                       uint32_t what, float *out, void *scratch, size_t scratch_bytes,
                       void *stream);

/*
 * pinn_query without the scratch argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments and results as pinn_query (the same
 * kernels), but a routed query (sub == -1) uses a routing scratch the library
 * holds in a fixed device array of about 8.4 MB per GPU (kept until the
 * process ends), so n is limited to 1,048,576 routed points: PINN_E_BUDGET
 * beyond that (and beyond cfg.max_query_points), before anything is enqueued.
 * Calls no allocating routine.  Every call on one GPU shares that GPU's
 * array, whose contents persist between calls (the kernels write every part
 * they read before reading it): calls that may overlap on one GPU, from any
 * context or stream, race on it and must be ordered by the caller.
 */
pinn_status pinn_query_noalloc(pinn_ctx *ctx, const float *x, int64_t n, int32_t sub,
                               uint32_t what, float *out, void *stream);

/*
 * Ghost-target exchange (section 2.2 reference anchor normalisation,
 * Algorithm 1 exchange branch): for every subdomain a and every ghost point
 * of a listed in `faces`, write gh_up of a = (u_b, p_b - [b master] p_b(x_anc, t))
 * evaluated by the neighbour b that owns the point, into the device array
 * targets[a] (same layout as gh_up; may alias the gh_up the context reads).
 * faces: host array of n_faces records {a, b, first, count}.
 * x_anc: host [d] anchor location.
 * Stream-ordered and never synchronizing: each exchange runs on the device
 * after the previous exchange of the context (whatever its stream); a
 * changed face list or targets array is uploaded from a host copy the
 * library keeps until that upload has run, so the caller's arrays may be
 * reused as soon as the call returns.  PINN_E_NOMEM if the faces need more
 * work tiles than the workspace holds (sized at create for every ghost
 * point).
 */
typedef struct { int32_t a, b; int64_t first, count; } pinn_face;
pinn_status pinn_exchange(pinn_ctx *ctx, const pinn_face *faces, int32_t n_faces,
                          const float *x_anc, float *const *targets, void *stream);

/*
 * Durations of the fused-kernel launches recorded by PINN_TIME_KERNEL steps
 * since the previous call: waits for them, writes their sum in milliseconds
 * and their number, and forgets them.  With PINN_PER_SUBDOMAIN one recorded
 * launch spans all per-subdomain launches of the step, from the start of the
 * first to the end of the last.
 */
pinn_status pinn_kernel_time(pinn_ctx *ctx, double *total_ms, int64_t *launches);

/*
 * Memory check (test and debugging aid, not part of the method): with
 * pinn_config.guard_bytes > 0, waits for `stream`, copies every guard zone
 * of the workspace to the host and writes to *bad_bytes the number of bytes
 * that no longer hold the fill pattern (0 when no kernel wrote outside its
 * region).  With guard_bytes = 0 it writes 0.  Synchronizes; allocates a
 * host buffer of guard_bytes.  PINN_E_INVAL for a NULL argument.
 */
pinn_status pinn_check_guards(pinn_ctx *ctx, int64_t *bad_bytes, void *stream);

/*
 * Evaluation post-processing (section 3: stitching of local experts, the
 * master-rank anchor pinning p - p(x_anc, t), removal of the spatial mean of
 * pressure at each time, relative L2 error).  Points x[n][d+1] and the
 * reference ref[n][d+1] = (u_1..u_d, p) are grouped in snapshots: snapshot k
 * holds points snap_off[k] .. snap_off[k+1]-1 (host array, n_snap + 1
 * entries, nondecreasing, snap_off[n_snap] == n).  Writes err_out (device,
 * d + 2 floats): relative L2 of u_1..u_d, of the velocity vector, and of the
 * processed pressure.  Every point must lie in some subdomain box (else the
 * errors are NaN).  x_anc: host [d].  scratch of
 * pinn_evaluate_scratch_bytes(ctx, n, n_snap, max_snapshot_points) bytes.
 * Synchronizes `stream` once after copying snap_off.
 */
size_t pinn_evaluate_scratch_bytes(const pinn_ctx *ctx, int64_t n, int32_t n_snap,
                                   int64_t max_snapshot_points);
pinn_status pinn_evaluate(pinn_ctx *ctx, const float *x, const float *ref, int64_t n,
                          const int64_t *snap_off, int32_t n_snap, const float *x_anc,
                          float *err_out, void *scratch, size_t scratch_bytes, void *stream);

/* Rebuild the kernels' weight copies after theta was written outside pinn_step. */
pinn_status pinn_refresh(pinn_ctx *ctx, void *stream);

/* Synchronize and free host-side state; device memory stays the caller's. */
pinn_status pinn_destroy(pinn_ctx *ctx);

/* Launch configuration chosen at create: points per collocation tile,
 * persistent workgroups, work items; for benchmarks and tests. */
typedef struct {
  int32_t tile_points, value_points, n_wg, n_items, n_segments, threads;
  int64_t lds_bytes, stash_bytes, slab_floats;
} pinn_launch_info;
pinn_status pinn_get_launch_info(const pinn_ctx *ctx, pinn_launch_info *info);

/* Message of the last error on the calling thread ("" if none). */
const char *pinn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDPINN_H */
