/*
 * fmap.h -- C ABI of the MI355X (gfx950) preconditioned NCG-MLS field-map
 * estimator of Lin & Fessler, "Efficient Regularized Field Map Estimation in
 * 3D MRI" (arXiv 2005.08661).
 *
 * What the library computes (Sec. II-III of the paper):
 *   minimise  Psi(f) = Phi(f) + (beta/2) ||C f||^2            (Sec. II eq. (cost))
 * over the field map f (Hz) inside a support mask, where Phi is the
 * coil-combined multi-echo data term of Sec. II eqs. (cost1), (r), (gamma),
 * C the first-order finite difference over x, y and z (one row per pair of
 * axis neighbours that are both inside the mask), by the preconditioned
 * nonlinear conjugate gradient of the Algorithm in Sec. III: gradient
 * (eq. (ls_grad)), IC(0) preconditioner of H = D + beta C^T C
 * (eqs. (precon_hess), (precon)), Polak-Ribiere conjugacy and the monotone
 * line search of Sec. III-C (eq. (ls_update)).
 *
 * Conventions shared by every entry point:
 *   - Grid nx*ny*nz, z fastest: voxel j = (x*ny + y)*nz + z.
 *   - Images y are complex64 (interleaved float re, im) with layout
 *     [ncoil][necho][nx][ny][nz]; coil maps are complex64 [ncoil][nx][ny][nz].
 *   - Field maps are float64 in Hz; echo times in seconds; the phase of echo
 *     l is 2*pi*f*t_l (Sec. II eq. (model) with omega = 2*pi*f); beta
 *     multiplies (beta/2)||C f||^2 with f in Hz.
 *   - Voxels outside the mask are held at f = 0 and do not enter the cost.
 *   - Every pointer argument named "dev" is device memory on the current HIP
 *     device, owned by the caller and left untouched except for outputs.
 *     Host pointers are marked "host".
 *   - Work is enqueued on the given stream (NULL = default stream); argument
 *     and shape checks run synchronously before anything is enqueued.
 *   - No entry point throws or aborts; each returns an fm_status and, on
 *     failure, fm_last_error() (thread-local) describes the cause.
 *   - A plan may be used by one stream at a time; calls on one plan must not
 *     overlap.
 */
#ifndef FMAP_H
#define FMAP_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FM_MAX_ECHO 16
#define FM_MAX_PEAK 16

typedef enum {
  FM_OK = 0,
  FM_ERR_ARG = 1,       /* invalid argument (NULL pointer, bad enum, beta < 0, ...) */
  FM_ERR_SHAPE = 2,     /* bad dimensions (non-positive sizes, necho < 2, too many echoes) */
  FM_ERR_ALLOC = 3,     /* device allocation failed */
  FM_ERR_HIP = 4,       /* a HIP runtime call failed */
  FM_ERR_NOT_PD = 5,    /* an IC(0) pivot was not positive (singular Hessian model) */
  FM_ERR_NONFINITE = 6, /* NaN/Inf met in the iteration */
  FM_ERR_STATE = 7,     /* call out of order (e.g. fm_eval before fm_setup) */
  FM_ERR_TIMEOUT = 8    /* a device-side wait (wavefront sweep, resident grid barrier) exceeded its bound */
} fm_status;

typedef enum { FM_FIELDMAP = 0, FM_WATERFAT = 1 } fm_model;
/* F64: FP64 storage and arithmetic throughout.  MIX: FP32 per-voxel storage
 * and arithmetic with FP64 pivots, reductions and scalars. */
typedef enum { FM_PREC_F64 = 0, FM_PREC_MIX = 1 } fm_precision;
/* Elimination order of the IC(0) factor (Sec. III-B eq. (precon)): natural
 * (lexicographic, z fastest), red-black (voxels with x+y+z even first, each
 * colour in natural order), or three-colour ((x+y+z) mod 3 = 0, 1, 2, each in
 * natural order; the order for second-order differences, whose 13-point
 * C^T C couples voxels 1 and 2 steps apart and so couples voxels of one
 * red-black colour; built for reg_order 2 with IC(0) only), or block
 * red-black (the (x, y) plane cut into tiles of 8 x 8 whole columns coloured
 * (x/8 + y/8) mod 2, colour 0 first, natural order inside a tile: between
 * natural and red-black order in quality, two launches per sweep; built for
 * reg_order 1 and ny * nz * 80 below 2^30, FM_ERR_SHAPE otherwise; fm_adjoint
 * preconditions its CG in natural order there). */
typedef enum {
  FM_ORDER_NATURAL = 0,
  FM_ORDER_REDBLACK = 1,
  FM_ORDER_COLOR3 = 2,
  FM_ORDER_BLOCKRB = 3
} fm_ordering;
/* Preconditioner: IC(0), diag(H), none, or incomplete Cholesky with a drop
 * tolerance (IC_t, the preconditioner of Sec. III-B and Sec. IV: entries of
 * the factor below ict_factor x H_max, scaled by their column's 1-norm, are
 * dropped; H_max is the largest magnitude in H).  IC_t runs in natural order
 * with its fill bounded to the level-ict_level pattern of natural-order IC
 * (fm_ict_offsets); it needs the first-order regulariser and is not available
 * to batches, fm_adjoint or the resident schedule. */
typedef enum { FM_PRECOND_IC0 = 0, FM_PRECOND_DIAG = 1, FM_PRECOND_NONE = 2, FM_PRECOND_ICT = 3 } fm_precond;

/* Largest number of lower offsets of an IC_t pattern (level 2). */
#define FM_ICT_MAXOFF 11

/* Columns of the per-iteration trace (see fm_get_trace). */
enum {
  FM_TR_COST = 0,    /* Psi(f^i) at the start of iteration i                 */
  FM_TR_GTP = 1,     /* g^T p                                                */
  FM_TR_MU = 2,      /* Polak-Ribiere mu used (0 on restart)                 */
  FM_TR_RESTART = 3, /* 1 if the direction was reset to -p                   */
  FM_TR_ALPHA = 4,   /* final line-search step size                          */
  FM_TR_ZTG = 5,     /* z^T g                                                */
  FM_TR_B = 6,       /* ||C z||^2                                            */
  FM_TR_GNORM2 = 7,  /* ||g||^2                                              */
  FM_TR_W = 8
};

/* Problem description.  Plain data: the struct owns no memory. */
typedef struct {
  int32_t nx, ny, nz;            /* grid, each >= 1 */
  int32_t ncoil;                 /* >= 1 */
  int32_t necho;                 /* L, 2 <= L <= FM_MAX_ECHO (Sec. II needs L >= 2) */
  double te[FM_MAX_ECHO];        /* echo times, seconds (first necho used) */
  double beta;                   /* regularisation weight, >= 0 */
  int32_t niter;                 /* outer NCG iterations, >= 0 */
  int32_t nmls;                  /* line-search steps per iteration, >= 1 */
  int32_t model;                 /* fm_model */
  int32_t npeak;                 /* water-fat: number of fat peaks */
  double fat_hz[FM_MAX_PEAK];    /* water-fat: peak offsets, Hz */
  double fat_amp[FM_MAX_PEAK];   /* water-fat: relative amplitudes */
  int32_t nsweep;                /* water-fat init: sweep values (Sec. III-A uses 100) */
  int32_t pwls_iters;            /* water-fat init: CG iterations of eq. (w0_wf) */
  int32_t precision;             /* fm_precision */
  int32_t ordering;              /* fm_ordering */
  int32_t precond;               /* fm_precond */
  int32_t reg_order;             /* C of eq. (cost): 1 (also when 0) first-order finite differences,
                                    2 second-order (rows f_{j-e} - 2 f_j + f_{j+e} with all three voxels
                                    in the volume and the mask); 2 needs, with IC(0), the three-colour
                                    order (FM_ERR_ARG otherwise); batches take it with the diagonal
                                    preconditioner or none */
  double ict_factor;             /* IC_t: drop tolerance = ict_factor x H_max (Sec. III-B uses 1e-3); >= 0,
                                    0 keeps every entry of the pattern */
  int32_t ict_level;             /* IC_t: fill bound, the level-of-fill pattern kept (0, 1 or 2) */
} fm_params;

typedef struct fm_plan fm_plan;

/* Validate the parameters and allocate the plan's device workspace on the
 * current device (about 70 B per voxel in MIX, 140 B in F64, some 20 B (MIX)
 * to 40 B (F64) more for IC(0) with second-order differences, plus the
 * reduction buffers).  *plan is set to NULL on failure. */
fm_status fm_plan_create(const fm_params *prm, fm_plan **plan);

/* Free the plan and its workspace.  NULL is accepted. */
fm_status fm_plan_destroy(fm_plan *plan);

/* The IC_t fill pattern of a level (Sec. III-B; host only, no device work):
 * the lower offsets (dx, dy, dz) such that L(j, j - o) may be nonzero, voxel
 * j - o being (x - dx, y - dy, z - dz), in descending lexicographic order.
 *   offsets host int32 [FM_ICT_MAXOFF][3]; count host int32.
 * FM_ERR_ARG for a level outside 0..2. */
fm_status fm_ict_offsets(int32_t level, int32_t *offsets, int32_t *count);

/* The IC_t factor of the plan's last preconditioner step (fm_precondition,
 * or the last iteration of fm_solve / fm_iterate): L with H ~ L L^T.
 *   L dev float64 [1 + count][nx][ny][nz]: block 0 the diagonal L_jj, block
 *     1 + u the entry L(j, j - o_u) for offset u of fm_ict_offsets(ict_level)
 *     (0 outside the mask, the volume, or where the drop test removed it)
 * FM_ERR_ARG if the plan's preconditioner is not IC_t. */
fm_status fm_get_factor(fm_plan *plan, double *L, hipStream_t stream);

/* Setup (Sec. II eq. (r) and the Algorithm's precompute step): coil-combine
 * the images into zhat_l = sum_c conj(s_c) y_cl / sqrt(sum_c |s_c|^2) and keep
 * the per-echo magnitude and phase in the plan; also records the mask.
 *   y    dev complex64 [ncoil][necho][nx][ny][nz]
 *   sens dev complex64 [ncoil][nx][ny][nz], or NULL for s = 1 (needs ncoil == 1)
 *   mask dev uint8 [nx][ny][nz], nonzero = unknown voxel */
fm_status fm_setup(fm_plan *plan, const void *y, const void *sens, const uint8_t *mask,
                   hipStream_t stream);

/* Initial map of Sec. III-A (eq. (w0) for field maps; sweep plus PWLS,
 * eq. (w0_wf), for water-fat) from the data given to fm_setup.
 *   f0 dev float64 [nx][ny][nz], written; 0 outside the mask. */
fm_status fm_init(fm_plan *plan, double *f0, hipStream_t stream);

/* Evaluate at a given map f (dev float64 [N]): per-voxel data cost phi,
 * its derivative dphi/df (eq. (ls_grad) without the regulariser), the Huber
 * curvature d (eq. (ls_huber)) and (C^T C f).  Any output may be NULL; all
 * are dev float64 [N] and 0 outside the mask.  Needs fm_setup. */
fm_status fm_eval(fm_plan *plan, const double *f, double *phi, double *dphi, double *curv,
                  double *lap, hipStream_t stream);

/* Preconditioner step of the Algorithm for a given curvature d and gradient
 * g (dev float64 [N]): builds the plan's preconditioner for
 * H = diag(d) + beta C^T C (IC(0) in the plan's ordering, diag(H), the
 * identity, or IC_t) and writes p = P^{-1} g (dev float64 [N]).  piv, if not
 * NULL, receives the pivots P_jj (dev float64 [N]; IC_t: L_jj^2).  Needs
 * fm_setup.
 * Returns FM_ERR_NOT_PD (after synchronising the stream) if a pivot is not
 * positive. */
fm_status fm_precondition(fm_plan *plan, const double *curv, const double *g, double *piv,
                          double *p, hipStream_t stream);

/* Full solve: fm_setup, then fm_init unless f0 is given, then niter
 * iterations of the Algorithm; writes the final map to f_out.
 *   f0    dev float64 [N] initial map, or NULL for the paper's initial map
 *   f_out dev float64 [N]
 * The iteration loop runs from a HIP graph without host round trips. */
fm_status fm_solve(fm_plan *plan, const void *y, const void *sens, const uint8_t *mask,
                   const double *f0, double *f_out, hipStream_t stream);

/* Run niter further iterations from the plan's current state (after fm_solve
 * or a previous fm_iterate) and write the map to f_out (dev float64 [N]). */
fm_status fm_iterate(fm_plan *plan, int32_t niter, double *f_out, hipStream_t stream);

/* Copy the trace of the last solve to host memory: trace is host float64
 * [niter+1][FM_TR_W] (row niter holds the final cost only).  Synchronises
 * the stream.  Also returns the device status word of the solve (FM_OK,
 * FM_ERR_NOT_PD or FM_ERR_NONFINITE). */
fm_status fm_get_trace(fm_plan *plan, double *trace, hipStream_t stream);

/* Schedule of the iteration loop (Sec. III Algorithm; the arithmetic is the
 * same in both).  STREAM: one launch per pass, the loop replayed from a HIP
 * graph.  RESIDENT: one launch for all iterations of a call; each workgroup
 * keeps the per-voxel state of a tile of whole columns in registers and LDS,
 * and the passes are separated by grid barriers or waits on the neighbour
 * tiles, so the whole grid must be resident on the device at once (a grid
 * kept from running by other work ends with FM_ERR_TIMEOUT).  RESIDENT
 * needs MIX precision, red-black IC(0), 2 <= necho <= 4, tiles of at most
 * 2048 voxels that can all be resident on the device at once (for example
 * 128x128x64: 512 tiles of 4x8 columns), and an even nz.  AUTO (the default) takes RESIDENT when the plan qualifies and
 * has at least 512 voxels per compute unit (smaller volumes run as fast or
 * faster streamed). */
enum { FM_SCHED_AUTO = 0, FM_SCHED_STREAM = 1, FM_SCHED_RESIDENT = 2 };

/* Select the schedule for later fm_solve / fm_iterate calls.  FM_ERR_ARG for
 * an unknown value or RESIDENT on a plan that does not qualify. */
fm_status fm_set_schedule(fm_plan *plan, int32_t sched);

/* The schedule the next fm_solve will use (FM_SCHED_STREAM or
 * FM_SCHED_RESIDENT), host int32. */
fm_status fm_get_schedule(fm_plan *plan, int32_t *sched);

/* Device status of the work enqueued so far on this plan (synchronises the
 * stream): FM_OK, or the first device-side error of the last solve
 * (FM_ERR_NOT_PD for a non-positive IC(0) pivot, FM_ERR_NONFINITE,
 * FM_ERR_TIMEOUT for an expired wavefront wait, FM_ERR_STATE for a broken
 * launch chain).  The word is cleared by the next fm_solve. */
fm_status fm_plan_status(fm_plan *plan, hipStream_t stream);

/* Number of voxels inside the mask given to the last fm_setup (host int64),
 * synchronising the stream. */
fm_status fm_mask_count(fm_plan *plan, int64_t *count, hipStream_t stream);

/* Component images at a field map, eq. (wf): for every voxel the least-squares
 * fit x = A^+ y_j with A = (diag(e^{i 2 pi f_j t}) gamma) (x) s_j, i.e. the
 * magnetisation m (field-map model, K = 1) or the water and fat images
 * (water-fat model, K = 2; gamma = [1, c], c_l the fat spectrum at t_l).
 *   y, sens as for fm_setup (the data of the map)
 *   f       dev float64 [N] map in Hz, or NULL for the map of the last
 *           fm_solve / fm_iterate
 *   m_out   dev complex64 [K][nx][ny][nz]; 0 outside the mask and where
 *           sum_c |s_c|^2 = 0
 * Computed in FP64 in both precision modes.  Needs fm_setup (or fm_solve). */
fm_status fm_components(fm_plan *plan, const void *y, const void *sens, const double *f, void *m_out,
                        hipStream_t stream);

/* Implicit adjoint of the map left by the last fm_solve / fm_iterate (not part
 * of the paper: it differentiates the minimiser of Sec. II eq. (cost), whose
 * gradient vanishes there).  With H = diag(h) + beta C^T C the exact Hessian
 * of the cost at the map (h_j from the cosines of the echo-pair terms, not
 * the Huber bound of Sec. III-B eq. (ls_huber)), it solves H v = dL/df by
 * conjugate gradients preconditioned as the iteration is (IC(0) of the Huber
 * model in the plan's ordering, its diagonal, or none; with reg_order 2, C^T C
 * the 13-point operator and the diagonal D + beta diag(C^T C) in place of
 * IC(0): v does not depend on the preconditioner), stopping once
 * ||r|| <= rtol ||dL/df|| or after maxit iterations, and returns
 *   dL/dbeta = -v^T C^T C f                               (host float64)
 *   dL/dy_cl = -(s_c / sqrt(sum |s|^2)) v d g / d zhat_l  (dev complex64,
 *              layout of y; d/dRe + i d/dIm convention, as torch uses)
 * where g is the gradient of the cost in f.
 *   dldf    dev float64 [N] (values outside the mask are ignored)
 *   sens    the coil maps given to fm_setup (NULL iff ncoil == 1); only read
 *           when dldy is not NULL
 *   dldy    dev complex64 [ncoil][necho][nx][ny][nz], or NULL
 *   v_out   dev float64 [N] (v, 0 outside the mask), or NULL
 *   dldbeta host float64, or NULL;  iters host int32 (CG iterations), or NULL
 * The derivative is that of the exact minimiser, so it describes the solver's
 * output to the extent that the iteration has converged.  Synchronises the
 * stream (convergence is checked every few CG iterations).  Returns
 * FM_ERR_STATE without a previous solve, FM_ERR_NOT_PD if the Hessian is not
 * positive definite along a CG direction (the map is not a strict local
 * minimum).  The first call allocates the adjoint workspace (about 10 values
 * per voxel). */
fm_status fm_adjoint(fm_plan *plan, const double *dldf, const void *sens, void *dldy, double *v_out,
                     double *dldbeta, int32_t maxit, double rtol, int32_t *iters, hipStream_t stream);

/* Change beta of an existing plan (for tuning beta by gradient without a new
 * plan).  The next call must be fm_solve. */
fm_status fm_set_beta(fm_plan *plan, double beta);

/* ---- Batches: many volumes in one launch per pass ------------------------
 * Not part of the paper: for throughput, nvol field-map volumes of possibly
 * different grid sizes and beta are solved together; every pass of the
 * Algorithm is one launch for all volumes (workgroups are partitioned among
 * the volumes in proportion to their sizes) and the iteration loop is one HIP
 * graph.  Each volume's iteration is the same as fm_solve's (its own scalar
 * state, line search and trace), up to the order of floating-point sums.
 * All volumes must share ncoil, necho, te, niter, nmls, precision, ordering
 * and preconditioner; supported: the field-map model with red-black IC(0),
 * the diagonal preconditioner or none. */
typedef struct fm_batch fm_batch;

/* prm: host array of nvol parameter sets (grid sizes and beta may differ). */
fm_status fm_batch_create(int32_t nvol, const fm_params *prm, fm_batch **batch);
fm_status fm_batch_destroy(fm_batch *batch);

/* Solve all volumes.  y, sens, mask, f0 and f_out are host arrays of nvol
 * device pointers with the layouts of fm_solve (sens may be NULL when
 * ncoil == 1; f0 may be NULL, or have NULL entries, for the paper's initial
 * map).  Synchronises the stream at the end. */
fm_status fm_batch_solve(fm_batch *batch, const void *const *y, const void *const *sens,
                         const uint8_t *const *mask, const double *const *f0, double *const *f_out,
                         hipStream_t stream);

/* Trace of volume v of the last batched solve (as fm_get_trace). */
fm_status fm_batch_get_trace(fm_batch *batch, int32_t v, double *trace, hipStream_t stream);

/* Workgroups of the batched launches (partitioned among the volumes); *used
 * receives the count actually used (at least nvol, at most one per chunk). */
fm_status fm_batch_set_grid(fm_batch *batch, int32_t grid, int32_t *used);

/* Autotuner: time probe_iters iterations on the given data for each
 * candidate workgroup count (256, 512, ... up to one per chunk of voxels),
 * keep the fastest, and report it (*grid_out) with its time per iteration in
 * milliseconds (*ms_out).  Either output may be NULL.  Leaves no solve
 * behind: call fm_batch_solve afterwards. */
fm_status fm_batch_autotune(fm_batch *batch, const void *const *y, const void *const *sens,
                            const uint8_t *const *mask, int32_t probe_iters, int32_t *grid_out,
                            double *ms_out, hipStream_t stream);

/* Kernel classes reported by fm_time_kernels. */
enum {
  FM_K_GRAD = 0,      /* gradient pass: data term, stencil, f update        */
  FM_K_PRECOND_A = 1, /* IC(0) forward sweep (natural) / black pass (red-black) / diagonal */
  FM_K_PRECOND_B = 2, /* IC(0) backward sweep (natural) / red pass (red-black) */
  FM_K_DOTS = 3,      /* conjugacy dot products                             */
  FM_K_DIR = 4,       /* direction and line-search setup                    */
  FM_K_MLS = 5,       /* further line-search passes                         */
  FM_K_RESIDENT = 6,  /* resident schedule: one launch for all the iterations */
  FM_NK = 7
};

/* Measurement: run niter further iterations from the plan's current state
 * (as fm_iterate, but launching kernel by kernel instead of from the graph;
 * the resident schedule runs them as one launch of class FM_K_RESIDENT)
 * with a HIP event pair around every launch on the given stream, and return
 * per kernel class the summed duration in milliseconds and the number of
 * launches (host float64 ms[FM_NK], host int32 launches[FM_NK]).  The map is
 * not written out.  Synchronises the stream. */
fm_status fm_time_kernels(fm_plan *plan, int32_t niter, double *ms, int32_t *launches,
                          hipStream_t stream);

/* ---- Allocation-free solve ------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as fm_solve (coil combination, the initial map of eq. (w0) unless f0
 * is given, niter iterations, the final map), on a problem described by prm
 * alone (no plan), with every piece of workspace taken from one fixed device
 * array of 48 MiB that the library holds on each GPU it runs on until the
 * process ends.  The call launches kernels on the stream and nothing else: no
 * device allocation or free, no memset, no copy, no graph; it does not
 * synchronise.  The first call on a device looks the array's device address
 * up (make that first call outside any stream capture).
 *   prm        host; the field-map model, first-order differences,
 *              necho <= 4, red-black IC(0) / diag(H) / none, at most 2^18
 *              voxels and 4096 iterations, and a workspace that fits the
 *              array (FM_ERR_SHAPE otherwise, FM_ERR_ARG for the rest)
 *   y, sens, mask, f0   as for fm_solve (f0 may be NULL)
 *   f_out      dev float64 [N], written
 *   status_out dev int32, or NULL: receives the device status word of the
 *              solve (FM_OK, FM_ERR_NOT_PD, FM_ERR_NONFINITE)
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents (the state the solve needs cleared is cleared by each call):
 * calls that overlap on one GPU (on different streams or threads) race and
 * must be serialised by the caller. */
fm_status fm_solve_noalloc(const fm_params *prm, const void *y, const void *sens, const uint8_t *mask,
                           const double *f0, double *f_out, int32_t *status_out, hipStream_t stream);

/* Human-readable text for a status code, and the last error message of the
 * calling thread. */
const char *fm_status_string(fm_status st);
const char *fm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
