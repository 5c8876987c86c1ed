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
    FWI_ERR_NONFINITE = 7,   /* non-finite traces or misfit were produced (found on the device) */
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
                             /*    2 persistent, 1 plain), 1, 2 or 3.  Adjoint launches fuse     */
                             /*    min(this, 2) steps.  2 or 3 fall back to 1 when a wrapping    */
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
                             /*    eq. 1-2; 4 = staggered fourth-order differences (one step per */
                             /*    launch, rows 1, 2 or 4, not persistent; stability bound with  */
                             /*    98/9 in place of 8)                                           */
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
 * Geometry errors are found on the host before any HIP call.
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

/* Forward solve only: traces (and the misfit when d_obs is given).  Keeps
 * the replay state (checkpoints and the last segment) in the workspace for
 * a following fwi_plan_adjoint with the same c, rho and wavelet. */
fwi_status fwi_plan_forward(fwi_plan *plan, const fwi_io *io, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Adjoint and gradient from the state fwi_plan_forward left in the same
 * workspace.  The adjoint source is d_adj when given (it then plays the role
 * of dJ/dtraces), else 2 (traces - d_obs).  Writes grad_c / grad_rho.
 * The workspace state is consumed: a second adjoint needs a new forward. */
fwi_status fwi_plan_adjoint(fwi_plan *plan, const fwi_io *io, void *workspace,
                            size_t workspace_bytes, void *stream);

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
