/*
 * fwi.h -- C ABI of the MI355X FWI-gradient library (libfwi.so).
 *
 * The library computes, for one or many media, the forward acoustic wave
 * solve of every transmit, the misfit against observed traces, and the exact
 * gradient of that misfit with respect to speed of sound and density, using
 * hand-written HIP kernels for gfx950.
 *
 * Method (Zhang et al., "Physics Informed Deep Unfolded Full Waveform
 * Inversion for Edema Detection"):
 *   - forward model: eq. 1 (variable c and rho, source S, damping D) advanced
 *     by the explicit update of eq. 2 with a quadratic absorbing profile
 *     (Sec. IV: 20 cells, R = 1e-3); the Laplacian coefficient is read as
 *     C^2 dt^2 / (1 + D dt) and rho enters in flux form;
 *   - receiver sampling: eq. 3 (M[p] in R^{n_t x n_R}), all transmits eq. 4;
 *   - misfit: the data term of eq. 5, J = sum (d - d_obs)^2 (no 1/2);
 *   - gradient: eq. 6, g = dJ/dc (and dJ/drho), by the exact discrete adjoint
 *     of the update and a zero-lag cross-correlation (imaging condition).
 *
 * Conventions shared by every entry point:
 *   - grids are row-major [nz][nx], x fastest, iz = 0 the top row; a cell is
 *     addressed by iz * nx + ix;
 *   - traces are [n_tx][nt][n_rcv]; sample n is the field after step n
 *     (time (n+1) dt), taken after the source of step n was added;
 *   - the source adds w_p[n] to the field at src[p] at step n;
 *   - every array passed in an fwi_io is a DEVICE pointer owned by the
 *     caller, in the plan's dtype (float or double) unless stated; it must
 *     stay valid until the work queued on the stream has completed;
 *   - no entry point throws, aborts or prints; failures are reported by the
 *     returned status and fwi_plan_last_error().
 */
#ifndef FWI_H
#define FWI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fwi_status {
    FWI_OK = 0,
    FWI_ERR_INVALID = 1,     /* bad argument: NULL pointer, size out of range, option unknown   */
    FWI_ERR_CFL = 2,         /* unstable time step: (D_max dt)^2*4 + k (c_max dt/h)^2 >= 4 with  */
                             /* k = 8 (order 2) or 98/9 (order 4), or                           */
                             /* a cell's c above the declared c_max (found on the device)        */
    FWI_ERR_GEOMETRY = 3,    /* a source or receiver cell outside the grid                      */
    FWI_ERR_NOMEM = 4,       /* the library could not allocate its plan-owned device tables     */
    FWI_ERR_WORKSPACE = 5,   /* workspace NULL or smaller than fwi_plan_workspace_size()        */
    FWI_ERR_HIP = 6,         /* a HIP runtime call failed (message in fwi_plan_last_error)      */
    FWI_ERR_NONFINITE = 7,   /* non-finite traces, misfit or gradient (found on the device)     */
    FWI_ERR_MEDIUM = 8,      /* c <= 0, rho <= 0 or a non-finite c / rho (found on the device)  */
    FWI_ERR_STATE = 9        /* fwi_plan_adjoint without a preceding fwi_plan_forward            */
} fwi_status;

typedef enum fwi_dtype { FWI_F32 = 0, FWI_F64 = 1 } fwi_dtype;

typedef enum fwi_mode {
    FWI_PLAIN = 0,           /* one transmit, one time step per kernel launch                   */
    FWI_BATCHED = 1          /* every (medium, transmit group) advanced by each launch           */
} fwi_mode;

/* One medium's grid and acquisition geometry (Sec. II-A: one transmitter per
 * shot, a receiver subset per shot).  Host data, copied by fwi_plan_create. */
typedef struct fwi_grid {
    int32_t nx, nz;          /* cells; each >= 2 * npml + 3; nx*nz*max(group,2)*sizeof(dtype)   */
                             /* below 4 GiB (FWI_ERR_INVALID otherwise)                         */
    int32_t nt;              /* time steps = samples per trace, >= 1                            */
    int32_t npml;            /* absorbing-layer width in cells, >= 0                            */
    double h;                /* grid spacing (m), > 0                                           */
    double dt;               /* time step (s), > 0                                              */
    double pml_r;            /* target reflection coefficient of the layer, 0 < pml_r < 1       */
    double pml_cref;         /* speed (m/s) used in D_max = 3 cref ln(1/R) / (2 npml h)         */
    double c_max;            /* caller's upper bound on c (m/s) for the stability check         */
    int32_t n_tx;            /* transmits, >= 1                                                 */
    int32_t n_rcv;           /* receivers per transmit, >= 1 (duplicates accumulate)            */
    const int32_t *src;      /* HOST [n_tx] source cells                                        */
    const int32_t *rcv;      /* HOST [n_tx][n_rcv] receiver cells                               */
} fwi_grid;

/* One medium's device buffers for a call.  Pointers may change between calls. */
typedef struct fwi_io {
    const void *c;           /* [nz][nx] speed of sound (m/s)                                   */
    const void *rho;         /* [nz][nx] density (kg/m^3)                                       */
    const void *wavelet;     /* [n_tx][nt] source samples, or [nt] if wavelet_shared != 0       */
    int32_t wavelet_shared;
    int32_t reserved;
    const void *d_obs;       /* [n_tx][nt][n_rcv] observed traces, or NULL                      */
    const void *d_adj;       /* [n_tx][nt][n_rcv] adjoint source for fwi_plan_adjoint, or NULL  */
    void *traces;            /* [n_tx][nt][n_rcv] out; required by every call                   */
    void *grad_c;            /* [nz][nx] out dJ/dc, or NULL                                     */
    void *grad_rho;          /* [nz][nx] out dJ/drho, or NULL                                   */
    double *misfit;          /* device double out: J for this medium, or NULL                   */
    const void *eta;         /* [nz][nx] attenuation rate (1/s, >= 0) of plans created with      */
                             /*    options.attenuation = 1 (NULL = 0); ignored otherwise         */
    void *grad_eta;          /* [nz][nx] out dJ/deta (attenuation plans), or NULL               */
} fwi_io;

typedef struct fwi_options {
    int32_t mode;            /* fwi_mode                                                        */
    int32_t ckpt_interval;   /* K: 0 = automatic (all planes kept when they fit the memory       */
                             /*    budget, else K ~ sqrt(2 nt)); >= nt keeps every plane;        */
                             /*    other values are raised to at least 2                         */
    int32_t group;           /* transmits advanced together per work item: 0 = automatic, 1,2,4 */
    int32_t rows;            /* rows per thread in a tile (tile = 64 x 4*rows): 0 = default     */
    int32_t use_graph;       /* 1: record the batched launch sequence once in a hipGraph and     */
                             /*    replay it (FWI_BATCHED only)                                  */
    int32_t acc_double;      /* 1: imaging accumulators in double for FWI_F32 (default 0)       */
    int32_t steps_per_launch;/* forward-type time steps fused per launch: 0 = default (3 batched, */
                             /*    2 persistent, 1 plain; order 4: 1), 1, 2 or 3 (order 4: 1 or  */
                             /*    2).  Adjoint launches fuse min(this, 2) steps (order 4: one). */
                             /*    2 or 3 fall back to 1 when a wrapping                         */
                             /*    segment buffer has K < 4; with 2 or 3, rows must be 1, 2 or 4; */
                             /*    3 is not persistent                                           */
    int32_t forward_only;    /* 1: traces and misfit only; no replay state is kept and           */
                             /*    gradient or adjoint calls return FWI_ERR_INVALID              */
    int32_t persistent;      /* 1: one launch per wave runs every step, its workgroups meeting   */
                             /*    at a device-wide barrier between steps (FWI_BATCHED only)     */
    int32_t barrier_spin;    /* polls before a barrier wait is abandoned (0 = 2^21); an         */
                             /*    abandoned wait ends the launch and fwi_plan_check reports     */
                             /*    FWI_ERR_HIP                                                   */
    double mem_budget;       /* bytes the workspace may use; 0 = 60% of free device memory      */
    const char *tune_cache;  /* JSON cache path of the tile autotuner, or NULL                   */
    int32_t order;           /* spatial order of the operator: 0 or 2 = the 5-point flux form of */
                             /*    eq. 1-2; 4 = staggered fourth-order differences (rows 1, 2 or */
                             /*    4, not persistent; stability bound with 98/9 in place of 8)   */
    int32_t hvp;             /* 1: the plan serves fwi_plan_hvp only (order 2, not persistent,  */
                             /*    no graph, not forward_only; groups of 2 by default, with the  */
                             /*    default multi-step launches; groups of 4 run one step per     */
                             /*    launch; its workspace holds value and derivative of every     */
                             /*    field)                                                        */
    int32_t host_only;       /* 1: plan on the host only, with no HIP call (mem_budget > 0       */
                             /*    required): sizes, info and fwi_plan_launches work, the calls  */
                             /*    return FWI_ERR_INVALID                                        */
    int32_t single_wave;     /* 1: keep every item resident at once (checkpointing as needed),   */
                             /*    as fwi_plan_forward / fwi_plan_adjoint require; 0: with       */
                             /*    ckpt_interval 0 the planner may instead keep every plane and  */
                             /*    run the items in several waves when its cost model prefers it */
    int32_t attenuation;     /* 1: a per-cell attenuation rate eta (fwi_io.eta) joins the damping */
                             /*    D of eq. 1-2 (Sec. VII's extension of the forward model) and  */
                             /*    dJ/deta is returned in grad_eta; one step per launch, order 2, */
                             /*    not persistent, not hvp                                        */
    int32_t reserved;
} fwi_options;

typedef struct fwi_plan fwi_plan;

typedef struct fwi_plan_info {
    int64_t cell_updates;    /* useful forward + adjoint updates per gradient: 2 nx nz nt n_tx   */
    int64_t recompute_updates;/* extra forward updates spent re-running checkpointed segments    */
    int64_t workspace_bytes;
    int32_t n_items;         /* work items (medium, transmit group)                             */
    int32_t group;           /* transmits per item                                              */
    int32_t rows;            /* rows per thread                                                 */
    int32_t launches;        /* step-kernel launches per gradient (1 per wave when persistent)   */
    int32_t max_ckpt;        /* largest K over items (nt when every plane is kept)              */
    int32_t min_ckpt;
    int32_t waves;           /* groups of items run one after another to fit the memory budget */
    int32_t steps_per_launch;/* forward-type time steps fused per launch actually used          */
} fwi_plan_info;

/* Validate the geometry and options, copy the geometry, build the device
 * tables (damping profiles, per-tile receiver lists, work-item schedule).
 * Defines the discrete problem of Sec. II-A: one grid per medium, one source
 * cell per transmit and a receiver subset per transmit, the damping profile
 * D of eq. 1-2 with the quadratic layer of Sec. IV.  grids[n_media] is host
 * memory read during the call only; *out receives a plan the caller frees
 * with fwi_plan_destroy.  Geometry errors (FWI_ERR_GEOMETRY), option and size
 * errors (FWI_ERR_INVALID) and the host stability check (FWI_ERR_CFL) are
 * found on the host before any HIP call; fwi_last_create_error() holds the
 * message and *out is NULL on failure.
 * Allocates plan-owned device memory (freed by fwi_plan_destroy). */
fwi_status fwi_plan_create(fwi_plan **out, fwi_dtype dtype, const fwi_grid *grids,
                           int32_t n_media, const fwi_options *opt);

/* Bytes of device workspace the caller must pass to the calls below. */
fwi_status fwi_plan_workspace_size(const fwi_plan *plan, size_t *bytes);

fwi_status fwi_plan_get_info(const fwi_plan *plan, fwi_plan_info *info);

/* Forward solve of every transmit, misfit (when d_obs is given), adjoint and
 * imaging, and the gradient of J (eq. 6) for each of the plan's n_media
 * media.  d_obs is required when grad_c or grad_rho is requested.  Outputs
 * are overwritten.  Asynchronous on ``stream`` (a hipStream_t, NULL = the
 * null stream); device-side failures are reported by fwi_plan_check(). */
fwi_status fwi_plan_execute(fwi_plan *plan, const fwi_io *io, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Forward solve only: the update of eq. 2 from zero initial fields with the
 * source added at its cell each step, and the receiver samples of eq. 3
 * (traces), plus the misfit of eq. 5 when d_obs is given.  Keeps the replay
 * state (checkpoints and the last segment) in the workspace for a following
 * fwi_plan_adjoint with the same c, rho and wavelet.  Arguments, ownership
 * and errors as for fwi_plan_execute; the plan must hold one wave
 * (FWI_ERR_INVALID otherwise). */
fwi_status fwi_plan_forward(fwi_plan *plan, const fwi_io *io, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Adjoint and gradient from the state fwi_plan_forward left in the same
 * workspace: the exact discrete adjoint of eq. 2 run backwards in time with
 * the zero-lag imaging condition of eq. 6.  The adjoint source is d_adj when
 * given (it then plays the role of dJ/dtraces, so the outputs are the
 * vector-Jacobian product), else 2 (traces - d_obs).  Writes grad_c /
 * grad_rho.  FWI_ERR_STATE when the workspace holds no forward state; the
 * state is consumed: a second adjoint needs a new forward.  Other arguments,
 * ownership and errors as for fwi_plan_execute. */
fwi_status fwi_plan_adjoint(fwi_plan *plan, const fwi_io *io, void *workspace,
                            size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as fwi_plan_execute, with the workspace taken from a static
 * device array of FWI_SCRATCH_BYTES owned by the library (one per GPU, held
 * until the process ends) instead of a caller's buffer.  The call allocates
 * nothing (no hipMalloc, no graph: the plan's use_graph is ignored); the
 * plan itself is created beforehand with fwi_plan_create.  io as for
 * fwi_plan_execute.  FWI_ERR_WORKSPACE (nothing launched) when the plan's
 * workspace size exceeds FWI_SCRATCH_BYTES: create such plans with
 * mem_budget <= FWI_SCRATCH_BYTES so that the planner checkpoints or splits
 * them into waves.  All calls on one GPU share the array, so calls that
 * overlap in time on one GPU (two streams, two threads) race; serialise them.
 * The call leaves no state that fwi_plan_adjoint could use. */
#define FWI_SCRATCH_BYTES ((size_t)256 << 20)
fwi_status fwi_plan_execute_scratch(fwi_plan *plan, const fwi_io *io, void *stream);

/* Direction and outputs of fwi_plan_hvp for one medium (device pointers in
 * the plan's dtype, caller-owned, valid until the stream work completes). */
typedef struct fwi_hvp_io {
    const void *dc;          /* [nz][nx] direction, speed-of-sound component (m/s)              */
    const void *drho;        /* [nz][nx] direction, density component, or NULL (= 0)            */
    void *hv_c;              /* [nz][nx] out: speed-of-sound component of H v                   */
    void *hv_rho;            /* [nz][nx] out: density component of H v, or NULL                 */
    void *dtraces;           /* [n_tx][nt][n_rcv] out: tangent-linear traces (dF/dm) v, or NULL */
} fwi_hvp_io;

/* Hessian-vector product of the misfit J = sum (d - d_obs)^2 (eq. 5) of each
 * medium in the direction v = (dc, drho): H v = d/de grad J(m + e v) at e = 0,
 * the product that back-propagation through the unfolded gradient steps of
 * eq. 9 needs (the Hessian is symmetric, so it is also the vector-Jacobian
 * product of the gradient map of eq. 6).  Computed exactly (up to rounding)
 * by forward-mode differentiation of the gradient: the forward solve carries
 * the tangent-linear fields, the adjoint the second-order adjoint fields
 * (driven by twice the tangent-linear traces), and the imaging condition
 * their derivative.  The plan must have been created with options.hvp = 1
 * (FWI_ERR_INVALID otherwise).  io as for fwi_plan_execute with d_obs
 * required: it also receives the traces, the misfit and (when grad_c /
 * grad_rho are given) the gradient at m.  dir[n_media] as declared above;
 * dc and hv_c are required.  Asynchronous on ``stream``; device-side
 * failures (a bad medium or direction, non-finite results) are reported by
 * fwi_plan_check(). */
fwi_status fwi_plan_hvp(fwi_plan *plan, const fwi_io *io, const fwi_hvp_io *dir, void *workspace,
                        size_t workspace_bytes, void *stream);

/* One kernel launch of a call's sequence, as fwi_plan_launches lists it. */
typedef enum fwi_kernel {
    FWI_K_FWD1 = 0, FWI_K_FWD2 = 1, FWI_K_ADJ1 = 2, FWI_K_ADJ2 = 3, FWI_K_FWD3 = 4,
    FWI_K_FWD4 = 5, FWI_K_ADJ4 = 6,          /* fourth-order operator, one step */
    FWI_K_PERSISTENT = 7, FWI_K_FILL = 8, FWI_K_PREP = 9, FWI_K_MISFIT_PARTIAL = 10,
    FWI_K_MISFIT_FINAL = 11, FWI_K_FINALIZE = 12,
    FWI_K_PREP_HVP = 13, FWI_K_PACK_HVP = 14, FWI_K_UNPACK_HVP = 15, FWI_K_FINALIZE_HVP = 16,
    FWI_K_FWD4X2 = 17                         /* fourth-order operator, two forward steps */
} fwi_kernel;

typedef struct fwi_launch {
    int32_t kernel;          /* fwi_kernel                                                      */
    int32_t wave;            /* wave of the step loop, -1 outside it                            */
    int32_t step;            /* launch index within the wave's schedule, -1 outside the loop    */
    int32_t grid_x, grid_y;  /* workgroups (grid_x * grid_y in all)                             */
    int32_t block;           /* work-items per workgroup                                        */
    int32_t lds_bytes;       /* dynamic LDS per workgroup                                       */
    int32_t reserved;
} fwi_launch;

/* The launch sequence of one call, computed on the host by the same code
 * that enqueues it (no HIP call): call 0 = fwi_plan_execute with gradients,
 * 1 = fwi_plan_forward, 2 = fwi_plan_adjoint, 3 = fwi_plan_hvp.  Writes the
 * first min(capacity, count) launches to out (host memory, may be NULL when
 * capacity is 0) and the total to *count.  The persistent kernel's grid is
 * 0 on a host-only plan (it depends on the device's occupancy).
 * FWI_ERR_INVALID for a call the plan cannot serve. */
fwi_status fwi_plan_launches(const fwi_plan *plan, int32_t call, fwi_launch *out, int64_t capacity,
                             int64_t *count);

/* Wait for the plan's last queued call and report device-side failures
 * (FWI_ERR_CFL, FWI_ERR_MEDIUM, FWI_ERR_NONFINITE) or FWI_OK. */
fwi_status fwi_plan_check(fwi_plan *plan);

void fwi_plan_destroy(fwi_plan *plan);

/* Autotuner: pick steps_per_launch, rows and (when base->group is 0, for
 * FWI_BATCHED) group for these grids by timing short device probes of every
 * feasible candidate (the grids' schedules cut to 24 steps, or lengthened up
 * to their own step counts until a call covers about 1e9 cell-updates; every
 * plane kept, a homogeneous medium; groups 4, 2 and 1) and keeping the fastest per
 * cell-update.  *out receives *base (or the defaults when base is NULL)
 * with those fields set; *ns_per_update (optional) the probe's time.
 * When base->tune_cache names a file, a cached choice for the same GPU
 * architecture, dtype, mode, group and size class is reused and new choices
 * are stored there (small JSON object).  Allocates and frees its own device
 * buffers and synchronises; call it before fwi_plan_create, off the hot path. */
fwi_status fwi_autotune(fwi_dtype dtype, const fwi_grid *grids, int32_t n_media, const fwi_options *base,
                        fwi_options *out, double *ns_per_update);

/* Static description of a status code. */
const char *fwi_status_string(fwi_status status);

/* Message of the plan's last failure ("" if none); valid until the next call. */
const char *fwi_plan_last_error(const fwi_plan *plan);

/* Message of the last fwi_plan_create failure on this thread. */
const char *fwi_last_create_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H */
