/*
 * fmo.h -- FP64 CPU oracle for the preconditioned NCG-MLS field-map estimator
 * of Lin & Fessler, "Efficient Regularized Field Map Estimation in 3D MRI"
 * (arXiv 2005.08661).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * reference used by the tests, by the smoke check and by the benchmark's CPU
 * baseline.  The product path (the HIP library) never links, loads or calls
 * it, and it shares no code, header or table with that path.
 *
 * Conventions (all host pointers, all FP64):
 *   - volumes are nx*ny*nz voxels, z fastest: j = (x*ny + y)*nz + z;
 *   - complex arrays are interleaved (re, im) doubles;
 *   - the field map f is in Hz and echo times in seconds, so the phase of
 *     echo l is 2*pi*f*t_l (Sec. II eq. (model) with omega = 2*pi*f);
 *   - beta multiplies (beta/2)*||C f||^2 with f in Hz (Sec. II eq. (cost));
 *   - C is the first-order finite difference over the three axes, with a row
 *     only for pairs of axis neighbours that are both inside the mask, so
 *     C^T C is the graph Laplacian of the mask;
 *   - voxels outside the mask are fixed at f = 0 and excluded everywhere.
 *
 * Parity pins and the readings taken where the paper is silent are listed in
 * the header comment of fmo.c.
 *
 * Every function returns FMO_OK (0) or a nonzero error code.
 */
#ifndef FMO_H
#define FMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FMO_OK = 0, FMO_ERR_ARG = 1, FMO_ERR_NOT_PD = 5, FMO_ERR_NONFINITE = 6 };
/* Elimination orders of IC(0): natural (lexicographic, z fastest), red-black
 * ((x+y+z) mod 2, then natural), three-colour ((x+y+z) mod 3, then
 * natural; no two voxels of a colour are pattern neighbours of the
 * second-order C^T C, whose neighbours lie 1 or 2 steps along an axis) and
 * block red-black (the (x, y) plane cut into tiles of FMO_BLOCK x FMO_BLOCK
 * whole columns coloured (x/FMO_BLOCK + y/FMO_BLOCK) mod 2, colour 0 first,
 * natural order inside a tile; tiles of one colour share no face). */
enum { FMO_ORDER_NATURAL = 0, FMO_ORDER_REDBLACK = 1, FMO_ORDER_COLOR3 = 2, FMO_ORDER_BLOCKRB = 3 };
enum { FMO_BLOCK = 8 };
/* IC(0), diag(H), none, or incomplete Cholesky with a drop tolerance (IC_t,
 * natural order; see fmo_ict_factor). */
enum { FMO_PRECOND_IC0 = 0, FMO_PRECOND_DIAG = 1, FMO_PRECOND_NONE = 2, FMO_PRECOND_ICT = 3 };
/* Largest number of lower offsets of an IC_t fill pattern (level 2: 11). */
enum { FMO_ICT_MAXOFF = 16 };

/* Columns of the per-iteration trace written by fmo_solve. */
enum {
  FMO_TR_COST = 0,    /* Psi(f^i) before the update of iteration i            */
  FMO_TR_GTP = 1,     /* g^T p                                                */
  FMO_TR_MU = 2,      /* Polak-Ribiere mu actually used (0 on restart)        */
  FMO_TR_RESTART = 3, /* 1 if the direction was reset to -p                   */
  FMO_TR_ALPHA = 4,   /* final step size of the monotone line search          */
  FMO_TR_ZTG = 5,     /* z^T g of the direction used                          */
  FMO_TR_B = 6,       /* ||C z||^2                                            */
  FMO_TR_GNORM2 = 7,  /* ||g||^2                                              */
  FMO_TR_W = 8
};

typedef struct {
  int32_t nx, ny, nz;   /* grid, z fastest */
  int32_t necho;        /* L >= 2 */
  const double *te;     /* [L] echo times, seconds */
  const double *gam;    /* [L*L] interleaved complex, row-major Gamma_{mn} */
  double beta;          /* >= 0 */
  int32_t niter;        /* outer NCG iterations */
  int32_t nmls;         /* line-search steps per outer iteration, >= 1 */
  int32_t ordering;     /* FMO_ORDER_* (IC(0) ordering) */
  int32_t precond;      /* FMO_PRECOND_* */
  int32_t reg_order;    /* finite differences of C: 1 (also when 0) or 2 (Sec. II eq. (cost)) */
  double ict_factor;    /* IC_t: tolerance = ict_factor * H_max (Sec. III-B uses 1e-3); 0 keeps every entry */
  int32_t ict_level;    /* IC_t: fill bound, the level-of-fill pattern kept (1 or 2) */
} fmo_problem;

/* IC(0) of H = diag(curv) + beta C^T C on the pattern of H, in the problem's
 * elimination order, by the general recurrence of incomplete LDL^T (an entry
 * L_jk of an earlier pattern neighbour k gets the products L_jm L_km D_m of
 * the pattern neighbours m that both share and that precede k), then
 * p = (L D L^T)^{-1} g.  Works for either regulariser order; piv gets D
 * (may be NULL).  FMO_ERR_NOT_PD if a pivot is not positive. */
int fmo_ic_general(const fmo_problem *pb, const uint8_t *mask, const double *curv, const double *g,
                   double *p, double *piv);

/* Diagonal of C^T C per voxel (0 outside the mask). */
int fmo_reg_diag(const fmo_problem *pb, const uint8_t *mask, double *out);

/* Gamma = gamma (gamma^H gamma)^{-1} gamma^H, Sec. II eq. (gamma).
 * Field-map case: gamma = 1 (Gamma_mn = 1/L). */
int fmo_gamma_fieldmap(int32_t L, double *gam);
/* Water-fat case: gamma = [1, c], c_l = sum_p amp_p exp(i 2 pi hz_p t_l). */
int fmo_gamma_waterfat(int32_t L, const double *te, int32_t npeak, const double *fat_hz,
                       const double *fat_amp, double *gam);

/* Coil combination zhat_l = sum_c conj(s_c) y_cl / sqrt(sum_c |s_c|^2)
 * (0 where the sum of squares is 0).  y: [ncoil][L][n], s: [ncoil][n] or NULL
 * for s = 1 (then ncoil must be 1).  zhat: [L][n]. */
int fmo_combine(int64_t n, int32_t ncoil, int32_t L, const double *y, const double *s,
                double *zhat);

/* Field-map initialisation, Sec. III-A eq. (w0), in Hz; 0 outside the mask. */
int fmo_init_fieldmap(int64_t n, int32_t L, const double *zhat, const double *te,
                      const uint8_t *mask, double *f0);

/* Per-voxel data term at f (Sec. II eq. (cost1), Sec. III-B eqs. (ls_grad),
 * (ls_huber), (inner_funs)): phi_j, dphi_j/df_j and the Huber curvature d_j.
 * Any output may be NULL.  Outside the mask all three are 0. */
int fmo_data_term(const fmo_problem *pb, const double *zhat, const uint8_t *mask,
                  const double *f, double *phi, double *dphi, double *curv);

/* (C^T C f)_j.  First order: one row f_k - f_j per in-mask neighbour pair.
 * Second order: one row f_{j-e} - 2 f_j + f_{j+e} per voxel j and axis e
 * with j - e, j and j + e all inside the volume and the mask. */
int fmo_laplacian(const fmo_problem *pb, const uint8_t *mask, const double *f, double *out);

/* Incomplete Cholesky IC(0) of H = diag(curv) + beta C^T C in the problem's
 * ordering, sqrt-free form M = (P + E) P^{-1} (P + E^T) (Sec. III-B eq.
 * (precon)): piv[j] = pivot P_jj (0 outside the mask).  Returns FMO_ERR_NOT_PD
 * if a pivot is not positive. */
int fmo_factor(const fmo_problem *pb, const uint8_t *mask, const double *curv, double *piv);

/* p = M^{-1} g by forward then backward substitution with the IC(0) factor. */
int fmo_apply(const fmo_problem *pb, const uint8_t *mask, const double *piv, const double *g,
              double *p);

/* Full preconditioned NCG with monotone line search (Sec. III, Algorithm).
 * f0: initial map (Hz); f: output map.  trace: [niter+1][FMO_TR_W] or NULL
 * (row niter holds only the final cost).  mls: [niter][nmls+1] or NULL; if
 * given, the cost f(alpha_k) along the line is recorded for every line-search
 * step (extra cost evaluations used only for the monotonicity checks). */
int fmo_solve(const fmo_problem *pb, const double *zhat, const uint8_t *mask, const double *f0,
              double *f, double *trace, double *mls);

/* Total cost Psi(f) = sum_j phi_j + (beta/2) f^T C^T C f. */
int fmo_cost(const fmo_problem *pb, const double *zhat, const uint8_t *mask, const double *f,
             double *psi);

/* Water-fat initialisation (Sec. III-A): per-voxel sweep of nsweep equispaced
 * values over [-|dfat|/2, |dfat|/2] (ends included), keeping the one of least
 * per-voxel cost (first on ties). */
int fmo_init_waterfat_sweep(const fmo_problem *pb, const double *zhat, const uint8_t *mask,
                            double dfat_hz, int32_t nsweep, double *ftilde);

/* PWLS weights rho_j = sum_{m,n} sum_{c,d} |r_cdmnj| (Sec. III-A, after eq.
 * (w0_wf)), from the raw images and coil maps. */
int fmo_pwls_weights(int64_t n, int32_t ncoil, int32_t L, const double *y, const double *s,
                     const double *gam, double *rho);

/* niters plain CG iterations on (2 diag(rho) + beta C^T C) f = 2 rho ftilde
 * from f = ftilde (eq. (w0_wf)). */
int fmo_pwls_cg(const fmo_problem *pb, const uint8_t *mask, const double *rho,
                const double *ftilde, int32_t niters, double *f);

/* Implicit adjoint of a converged map fhat (stationary point of Psi):
 * v = H^{-1} dL/df with the exact Hessian H = diag(h) + beta C^T C,
 * h_j = sum_{m<n} w_mn (2 pi dt_mn)^2 cos(x_mn), solved by conjugate gradients
 * preconditioned with IC(0) of the Huber model D + beta C^T C (problem
 * ordering) until ||r|| <= rtol ||dL/df|| or maxit iterations.  Then
 *   dL/dbeta = -v^T C^T C fhat,
 *   dL/dzhat_l = -v_j sum over pairs of d g_j / d zhat_l (gradient of a real
 *                function of complex values: d/dRe + i d/dIm),
 * written to dzhat [L][n] (interleaved complex).  *iters receives the CG
 * iterations used; FMO_ERR_NOT_PD if a CG curvature d^T H d is not positive. */
int fmo_adjoint(const fmo_problem *pb, const double *zhat, const uint8_t *mask, const double *fhat,
                const double *dldf, int32_t maxit, double rtol, double *v, double *dldbeta,
                double *dzhat, int32_t *iters);

/* Component images at a field map f (Sec. II-III, eq. (wf)): for every voxel
 * the least-squares solution x = A^+ y_j of A x = y_j with
 * A = (diag(e^{i 2 pi f_j t}) gamma) (x) s_j  (L*ncoil x K; reading R15 of the
 * dimensions), y_j stacked echo-major, gamma = 1 (K = 1, magnetisation m) or
 * [1, c] (K = 2, water and fat), c_l = sum_p amp_p e^{i 2 pi hz_p t_l}.  The
 * normal equations A^H A x = A^H y are formed and solved explicitly; x = 0
 * where A = 0 (no coil sensitivity) and outside the mask.
 *   y [ncoil][L][n], s [ncoil][n] or NULL (ncoil == 1), out [K][n] complex. */
int fmo_components(const fmo_problem *pb, int32_t ncoil, const double *y, const double *s,
                   const uint8_t *mask, const double *f, int32_t K, int32_t npeak, const double *fat_hz,
                   const double *fat_amp, double *out);

/* Lower offsets (dx, dy, dz) of the level-`level` fill pattern of IC in
 * natural order (z fastest) on a full grid: the positions (j, j - o) whose
 * level of fill is at most `level`, where stencil entries have level 0 and
 * eliminating voxel k gives (i, j) the level lev(i,k) + lev(k,j) + 1 (the
 * symbolic factorisation of IC(level)).  Found by that symbolic elimination on
 * a cube of side `side` (odd; the pattern of its centre row), returned in
 * descending lexicographic order of (dx, dy, dz).  offs: [FMO_ICT_MAXOFF][3]. */
int fmo_ict_offsets(int32_t level, int32_t side, int32_t *offs, int32_t *count);

/* Incomplete Cholesky with a drop tolerance, IC_t (Sec. III-B, Table 1; the
 * preconditioner of Sec. IV), of H = diag(curv) + beta C^T C over the in-mask
 * voxels in natural order: H ~ L L^T with L lower triangular.  Row by row in
 * natural order, each entry L_jk of a pattern position k < j (k = j - o, o one
 * of the fmo_ict_offsets of pb->ict_level, k inside the volume and the mask)
 * is
 *   L_jk = (H_jk - sum_{m < k} L_jm L_km) / L_kk
 * (m over the pattern positions of both rows, ascending), then set to zero if
 * |L_jk| < tol ||H(k:N, k)||_1 with tol = ict_factor * H_max and H_max the
 * largest magnitude in H (reading R21); L_jj = sqrt(H_jj - sum_k L_jk^2).
 * Reading R23: the fill is bounded to the level-`ict_level` pattern.
 *   L: [1 + noff][n]: row 0 the diagonal L_jj, row 1 + u the entry
 *   L(j, j - o_u) (0 outside the mask, the volume or the pattern).
 * FMO_ERR_NOT_PD if H_jj - sum_k L_jk^2 <= 0. */
int fmo_ict_factor(const fmo_problem *pb, const uint8_t *mask, const double *curv, double *L);

/* p = (L L^T)^{-1} g with the factor of fmo_ict_factor: forward solve
 * L y = g in natural order, then backward solve L^T p = y in reverse. */
int fmo_ict_apply(const fmo_problem *pb, const uint8_t *mask, const double *L, const double *g, double *p);

/* Threads for the loops over independent voxels when the oracle is built with
 * OpenMP (no effect otherwise); every sum over voxels stays sequential in
 * natural order, so the results do not depend on the thread count. */
int fmo_set_threads(int32_t nthreads);
int32_t fmo_threads(void);

#ifdef __cplusplus
}
#endif
#endif
