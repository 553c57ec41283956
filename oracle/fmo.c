/*
 * fmo.c -- FP64 CPU oracle for the preconditioned NCG-MLS field-map estimator
 * (Lin & Fessler, arXiv 2005.08661).  TEST INFRASTRUCTURE ONLY: used by the
 * tests, the smoke check and the benchmark's CPU baseline; the HIP product
 * path neither links nor calls it and shares no code with it.
 *
 * What is computed, and where the paper defines it:
 *   - coil combination and the pair weights r_{cdmnj}, collapsed to the
 *     coil-combined form R_mn = Gamma_mn conj(zhat_m) zhat_n
 *     (Sec. II eqs. (cost1), (r), (gamma)); the sum over coil pairs (c,d)
 *     of the paper's cost differs from the coil-combined cost by a constant
 *     in omega and has the same gradient;
 *   - per-voxel cost, gradient and Huber curvature over echo pairs m < n
 *     (the ordered-pair sum counts each unordered pair twice because Gamma
 *     is Hermitian, hence the weight 2|R_mn|) (Sec. III-B eqs. (ls_grad),
 *     (ls_huber), (inner_funs));
 *   - the first- or second-order finite-difference regulariser (Sec. II
 *     eq. (cost));
 *   - IC(0) of H = D + beta C^T C and the two triangular solves
 *     (Sec. III-B eqs. (precon_hess), (precon));
 *   - preconditioned NCG with Polak-Ribiere conjugacy and the monotone line
 *     search (Sec. III Algorithm, Sec. III-C eqs. (ls_cost), (ls_huber2),
 *     (ls_update));
 *   - initialisations of Sec. III-A (eqs. (w0), (w0_wf)).
 *
 * Readings taken where the paper is silent or garbled:
 *   R1 f in Hz, t in seconds, phase 2*pi*f*t; beta multiplies (beta/2)||Cf||^2.
 *   R3 the gradient carries (t_m - t_n), not its square (derivative of 1-cos).
 *   R4 "mod pi" is read as wrapping the phase to [-pi, pi]; sinc(0) = 1.
 *   R5 C has rows only for in-mask neighbour pairs; IC(0) in natural
 *      (lexicographic, z fastest), red-black or three-colour order (the
 *      last for the second-order C, whose stencil two colours do not split).
 *   R6 mu = (g - g_prev)^T p / (g_prev^T p_prev), mu = 0 at i = 0 or when the
 *      denominator is 0.  Pinned only in the quadratic limit (exact line
 *      search: the linear-CG coefficient); beyond it the conjugacy formula is
 *      parity unpinned.
 *   R7 z = -p + mu z_prev, reset to -p when z^T g >= 0.
 *   R8 the step size restarts from 0 at every outer iteration.
 *   R9 a fixed number nmls of line-search steps.
 *   R11 water-fat sweep over [-|df|/2, |df|/2], 100 values, first minimum.
 *   R12 PWLS by plain CG from the voxelwise estimate.
 *   R14 angle(0) = 0; zero data gives a zero data term.
 *   R20 second-order C: a row f_{j-e} - 2 f_j + f_{j+e} for every voxel j and
 *      axis e whose three voxels are inside the volume and the mask (R5 for
 *      second differences); no spatial weights.  IC(0) keeps L on the
 *      13-point stencil (in-mask voxels 1 or 2 steps along an axis), also
 *      where C^T C is 0 there.
 */
#include "fmo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
/* Loops whose iterations are independent (one voxel each, no shared sum) may
 * run on several threads; every sum over voxels stays a sequential loop in
 * natural order, so a build with OpenMP returns bit for bit what a build
 * without it returns. */
#define FMO_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define FMO_PARALLEL_FOR
#endif

#define TWO_PI 6.283185307179586476925286766559

int fmo_set_threads(int32_t nthreads) {
  if (nthreads < 1) return FMO_ERR_ARG;
#ifdef _OPENMP
  omp_set_num_threads(nthreads);
#endif
  return FMO_OK;
}

int32_t fmo_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

typedef struct {
  int32_t np;     /* number of echo pairs m < n */
  double *w;      /* [np][n] 2 |R_mn| */
  double *a;      /* [np][n] angle(R_mn) */
  double *d;      /* [np] 2 pi (t_m - t_n) */
} pairs_t;

static int64_t nvox(const fmo_problem *pb) {
  return (int64_t)pb->nx * pb->ny * pb->nz;
}

/* In-mask axis neighbours of voxel j; returns how many. */
static int neighbours(const fmo_problem *pb, const uint8_t *mask, int64_t j, int64_t nb[6]) {
  const int64_t nz = pb->nz, ny = pb->ny, nx = pb->nx;
  const int64_t sy = nz, sx = ny * nz;
  const int64_t z = j % nz, y = (j / nz) % ny, x = j / sx;
  int c = 0;
  if (x > 0 && mask[j - sx]) nb[c++] = j - sx;
  if (x < nx - 1 && mask[j + sx]) nb[c++] = j + sx;
  if (y > 0 && mask[j - sy]) nb[c++] = j - sy;
  if (y < ny - 1 && mask[j + sy]) nb[c++] = j + sy;
  if (z > 0 && mask[j - 1]) nb[c++] = j - 1;
  if (z < nz - 1 && mask[j + 1]) nb[c++] = j + 1;
  return c;
}

static int second_order(const fmo_problem *pb) { return pb->reg_order == 2; }

/* Coordinates and strides. */
static void coords(const fmo_problem *pb, int64_t j, int64_t c[3]) {
  const int64_t nz = pb->nz, ny = pb->ny;
  c[2] = j % nz;
  c[1] = (j / nz) % ny;
  c[0] = j / (ny * nz);
}

static int64_t stride(const fmo_problem *pb, int a) {
  return a == 0 ? (int64_t)pb->ny * pb->nz : (a == 1 ? (int64_t)pb->nz : 1);
}

static int64_t extent(const fmo_problem *pb, int a) { return a == 0 ? pb->nx : (a == 1 ? pb->ny : pb->nz); }

/* Second order: does the row centred at voxel j along axis a exist? */
static int row2(const fmo_problem *pb, const uint8_t *mask, int64_t j, int a) {
  int64_t c[3];
  coords(pb, j, c);
  if (c[a] < 1 || c[a] > extent(pb, a) - 2) return 0;
  const int64_t s = stride(pb, a);
  return mask[j] && mask[j - s] && mask[j + s];
}

/* Colours of the elimination order (natural order: one). */
static int ncolours(const fmo_problem *pb) {
  return (pb->ordering == FMO_ORDER_REDBLACK || pb->ordering == FMO_ORDER_BLOCKRB)
             ? 2
             : (pb->ordering == FMO_ORDER_COLOR3 ? 3 : 1);
}

/* Position of voxel j in the elimination order: its colour first ((x+y+z)
 * mod ncolours, or the tile colour of block red-black), then the natural
 * index (natural order inside a tile: a tile's voxels keep their relative
 * natural order, and tiles of one colour are not coupled). */
static int64_t rank_of(const fmo_problem *pb, int64_t j) {
  const int nc = ncolours(pb);
  if (nc == 1) return j;
  const int64_t nz = pb->nz, ny = pb->ny;
  const int64_t z = j % nz, y = (j / nz) % ny, x = j / (ny * nz);
  const int64_t colour =
      pb->ordering == FMO_ORDER_BLOCKRB ? (x / FMO_BLOCK + y / FMO_BLOCK) % 2 : (x + y + z) % nc;
  return colour * nvox(pb) + j;
}

/* Voxels in elimination order (in-mask only); returns the count. */
static int64_t build_order(const fmo_problem *pb, const uint8_t *mask, int64_t *order) {
  const int64_t n = nvox(pb);
  int64_t c = 0;
  for (int colour = 0; colour < ncolours(pb); ++colour)
    for (int64_t j = 0; j < n; ++j)
      if (mask[j] && rank_of(pb, j) / n == colour) order[c++] = j;
  return c;
}

static void cmul_conj(const double *zm, const double *zn, double *re, double *im) {
  /* conj(zm) * zn */
  *re = zm[0] * zn[0] + zm[1] * zn[1];
  *im = zm[0] * zn[1] - zm[1] * zn[0];
}

/* Precompute the coil-combined pair weights and phases (the paper's
 * "precompute r and t_m - t_n" step of the Algorithm). */
static int pairs_build(const fmo_problem *pb, const double *zhat, const uint8_t *mask,
                       pairs_t *pr) {
  const int64_t n = nvox(pb);
  const int L = pb->necho;
  pr->np = L * (L - 1) / 2;
  pr->w = (double *)calloc((size_t)pr->np * n, sizeof(double));
  pr->a = (double *)calloc((size_t)pr->np * n, sizeof(double));
  pr->d = (double *)calloc((size_t)pr->np, sizeof(double));
  if (!pr->w || !pr->a || !pr->d) return FMO_ERR_ARG;
  int q = 0;
  for (int m = 0; m < L; ++m)
    for (int k = m + 1; k < L; ++k, ++q) {
      const double gre = pb->gam[2 * (m * L + k)], gim = pb->gam[2 * (m * L + k) + 1];
      pr->d[q] = TWO_PI * (pb->te[m] - pb->te[k]);
      FMO_PARALLEL_FOR
      for (int64_t j = 0; j < n; ++j) {
        if (!mask[j]) continue;
        double cre, cim;
        cmul_conj(zhat + 2 * ((int64_t)m * n + j), zhat + 2 * ((int64_t)k * n + j), &cre, &cim);
        const double rre = gre * cre - gim * cim, rim = gre * cim + gim * cre;
        pr->w[(int64_t)q * n + j] = 2.0 * hypot(rre, rim);
        pr->a[(int64_t)q * n + j] = atan2(rim, rre);
      }
    }
  return FMO_OK;
}

static void pairs_free(pairs_t *pr) {
  free(pr->w);
  free(pr->a);
  free(pr->d);
}

static double sinc(double u) { return u == 0.0 ? 1.0 : sin(u) / u; }

/* phi_j, dphi_j/df_j and Huber curvature of voxel j at field value fj. */
static void voxel_terms(const pairs_t *pr, int64_t n, int64_t j, double fj, double *phi,
                        double *dphi, double *curv) {
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int q = 0; q < pr->np; ++q) {
    const double w = pr->w[(int64_t)q * n + j];
    const double d = pr->d[q];
    const double x = pr->a[(int64_t)q * n + j] + d * fj;
    const double u = x - TWO_PI * rint(x / TWO_PI);
    c0 += w * (1.0 - cos(x));
    c1 += w * d * sin(x);
    c2 += w * d * d * sinc(u);
  }
  *phi = c0;
  *dphi = c1;
  *curv = c2;
}

int fmo_gamma_fieldmap(int32_t L, double *gam) {
  if (L < 2 || !gam) return FMO_ERR_ARG;
  for (int i = 0; i < L * L; ++i) {
    gam[2 * i] = 1.0 / L;
    gam[2 * i + 1] = 0.0;
  }
  return FMO_OK;
}

int fmo_gamma_waterfat(int32_t L, const double *te, int32_t npeak, const double *fat_hz,
                       const double *fat_amp, double *gam) {
  if (L < 2 || !te || npeak < 1 || !fat_hz || !fat_amp || !gam) return FMO_ERR_ARG;
  /* gamma is L x 2: column 0 all ones, column 1 c_l. */
  double *cre = (double *)malloc(sizeof(double) * L), *cim = (double *)malloc(sizeof(double) * L);
  if (!cre || !cim) return FMO_ERR_ARG;
  for (int l = 0; l < L; ++l) {
    cre[l] = 0.0;
    cim[l] = 0.0;
    for (int p = 0; p < npeak; ++p) {
      cre[l] += fat_amp[p] * cos(TWO_PI * fat_hz[p] * te[l]);
      cim[l] += fat_amp[p] * sin(TWO_PI * fat_hz[p] * te[l]);
    }
  }
  /* G = gamma^H gamma = [[L, sum c], [sum conj c, sum |c|^2]]. */
  double s_re = 0, s_im = 0, cc = 0;
  for (int l = 0; l < L; ++l) {
    s_re += cre[l];
    s_im += cim[l];
    cc += cre[l] * cre[l] + cim[l] * cim[l];
  }
  const double det = L * cc - (s_re * s_re + s_im * s_im);
  if (!(det > 0)) {
    free(cre);
    free(cim);
    return FMO_ERR_NOT_PD;
  }
  /* G^{-1} = (1/det) [[cc, -sum c], [-sum conj c, L]]. */
  const double i00 = cc / det, i11 = L / det;
  const double i01re = -s_re / det, i01im = -s_im / det; /* entry (0,1) */
  const double i10re = -s_re / det, i10im = s_im / det;  /* entry (1,0) = conj */
  for (int m = 0; m < L; ++m)
    for (int k = 0; k < L; ++k) {
      /* Gamma_mk = sum_ab gamma_ma Ginv_ab conj(gamma_kb), gamma_m0 = 1, gamma_m1 = c_m */
      double re = i00, im = 0.0;
      /* a=0, b=1: Ginv_01 conj(c_k) */
      re += i01re * cre[k] + i01im * cim[k];
      im += i01im * cre[k] - i01re * cim[k];
      /* a=1, b=0: c_m Ginv_10 */
      re += cre[m] * i10re - cim[m] * i10im;
      im += cre[m] * i10im + cim[m] * i10re;
      /* a=1, b=1: c_m Ginv_11 conj(c_k) */
      re += i11 * (cre[m] * cre[k] + cim[m] * cim[k]);
      im += i11 * (cim[m] * cre[k] - cre[m] * cim[k]);
      gam[2 * (m * L + k)] = re;
      gam[2 * (m * L + k) + 1] = im;
    }
  free(cre);
  free(cim);
  return FMO_OK;
}

int fmo_combine(int64_t n, int32_t ncoil, int32_t L, const double *y, const double *s,
                double *zhat) {
  if (n < 0 || ncoil < 1 || L < 1 || !y || !zhat || (!s && ncoil != 1)) return FMO_ERR_ARG;
  FMO_PARALLEL_FOR
  for (int64_t j = 0; j < n; ++j) {
    double ss = 0.0;
    for (int c = 0; c < ncoil; ++c) {
      const double sre = s ? s[2 * ((int64_t)c * n + j)] : 1.0;
      const double sim = s ? s[2 * ((int64_t)c * n + j) + 1] : 0.0;
      ss += sre * sre + sim * sim;
    }
    for (int l = 0; l < L; ++l) {
      double re = 0.0, im = 0.0;
      for (int c = 0; c < ncoil; ++c) {
        const double sre = s ? s[2 * ((int64_t)c * n + j)] : 1.0;
        const double sim = s ? s[2 * ((int64_t)c * n + j) + 1] : 0.0;
        const double *yy = y + 2 * (((int64_t)c * L + l) * n + j);
        re += sre * yy[0] + sim * yy[1];
        im += sre * yy[1] - sim * yy[0];
      }
      const double sc = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
      zhat[2 * ((int64_t)l * n + j)] = re * sc;
      zhat[2 * ((int64_t)l * n + j) + 1] = im * sc;
    }
  }
  return FMO_OK;
}

int fmo_init_fieldmap(int64_t n, int32_t L, const double *zhat, const double *te,
                      const uint8_t *mask, double *f0) {
  if (L < 2 || !zhat || !te || !mask || !f0) return FMO_ERR_ARG;
  if (te[1] == te[0]) return FMO_ERR_ARG;
  FMO_PARALLEL_FOR
  for (int64_t j = 0; j < n; ++j) {
    if (!mask[j]) {
      f0[j] = 0.0;
      continue;
    }
    double re, im;
    cmul_conj(zhat + 2 * j, zhat + 2 * (n + j), &re, &im);
    f0[j] = atan2(im, re) / (TWO_PI * (te[1] - te[0]));
  }
  return FMO_OK;
}

static int check_pb(const fmo_problem *pb) {
  if (!pb || pb->nx < 1 || pb->ny < 1 || pb->nz < 1 || pb->necho < 2 || !pb->te || !pb->gam ||
      !(pb->beta >= 0) || pb->nmls < 1 || pb->niter < 0 || pb->ordering < FMO_ORDER_NATURAL ||
      pb->ordering > FMO_ORDER_BLOCKRB)
    return FMO_ERR_ARG;
  return FMO_OK;
}

int fmo_data_term(const fmo_problem *pb, const double *zhat, const uint8_t *mask,
                  const double *f, double *phi, double *dphi, double *curv) {
  if (check_pb(pb) || !zhat || !mask || !f) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  pairs_t pr;
  if (pairs_build(pb, zhat, mask, &pr)) return FMO_ERR_ARG;
  FMO_PARALLEL_FOR
  for (int64_t j = 0; j < n; ++j) {
    double a = 0, b = 0, c = 0;
    if (mask[j]) voxel_terms(&pr, n, j, f[j], &a, &b, &c);
    if (phi) phi[j] = a;
    if (dphi) dphi[j] = b;
    if (curv) curv[j] = c;
  }
  pairs_free(&pr);
  return FMO_OK;
}

int fmo_laplacian(const fmo_problem *pb, const uint8_t *mask, const double *f, double *out) {
  if (check_pb(pb) || !mask || !f || !out) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  if (second_order(pb)) {
    /* scatter every row's value back through its three coefficients 1, -2, 1 */
    for (int64_t j = 0; j < n; ++j) out[j] = 0.0;
    for (int64_t j = 0; j < n; ++j)
      for (int a = 0; a < 3; ++a)
        if (row2(pb, mask, j, a)) {
          const int64_t s = stride(pb, a);
          const double v = f[j - s] - 2.0 * f[j] + f[j + s];
          out[j - s] += v;
          out[j] -= 2.0 * v;
          out[j + s] += v;
        }
    return FMO_OK;
  }
  FMO_PARALLEL_FOR
  for (int64_t j = 0; j < n; ++j) {
    int64_t nb[6];
    double s = 0.0;
    if (mask[j]) {
      const int c = neighbours(pb, mask, j, nb);
      for (int k = 0; k < c; ++k) s += f[j] - f[nb[k]];
    }
    out[j] = s;
  }
  return FMO_OK;
}

/* Colours that are independent sets of the 7-point stencil (red-black and
 * three-colour orders), whose voxels a sweep may visit in any order within
 * the colour; block red-black couples the voxels of a tile, so it sweeps in
 * elimination order like natural order. */
static int independent_colours(const fmo_problem *pb) {
  return ncolours(pb) > 1 && pb->ordering != FMO_ORDER_BLOCKRB;
}

/* End of the run of colour `colour` that starts at position q0 of the
 * elimination order. */
static int64_t colour_end(const fmo_problem *pb, const int64_t *order, int64_t q0, int64_t cnt, int colour) {
  const int64_t n = nvox(pb);
  int64_t q = q0;
  while (q < cnt && rank_of(pb, order[q]) / n == colour) ++q;
  return q;
}

/* Pivot of voxel j from the pivots of its earlier neighbours. */
static double pivot_of(const fmo_problem *pb, const uint8_t *mask, const double *curv, const double *piv,
                       int64_t j) {
  const double b = pb->beta;
  int64_t nb[6];
  const int c = neighbours(pb, mask, j, nb);
  const int64_t rj = rank_of(pb, j);
  double s = 0.0;
  for (int k = 0; k < c; ++k)
    if (rank_of(pb, nb[k]) < rj) s += 1.0 / piv[nb[k]];
  return curv[j] + b * c - b * b * s;
}

int fmo_factor(const fmo_problem *pb, const uint8_t *mask, const double *curv, double *piv) {
  if (check_pb(pb) || !mask || !curv || !piv) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  if (!order) return FMO_ERR_ARG;
  const int64_t cnt = build_order(pb, mask, order);
  int st = FMO_OK;
  for (int64_t j = 0; j < n; ++j) piv[j] = 0.0;
  if (!independent_colours(pb)) {
    for (int64_t q = 0; q < cnt; ++q) {
      const int64_t j = order[q];
      piv[j] = pivot_of(pb, mask, curv, piv, j);
      if (!(piv[j] > 0.0)) {
        st = isfinite(piv[j]) ? FMO_ERR_NOT_PD : FMO_ERR_NONFINITE;
        break;
      }
    }
  } else {
    /* Each colour is an independent set of the 7-point stencil (axis
     * neighbours differ by one in x+y+z), so no pivot of a colour uses
     * another of the same colour: a colour's pivots are formed in any order,
     * then checked in elimination order as the sequential sweep would (the
     * first non-positive pivot stops the factorisation; later ones stay 0). */
    int64_t q0 = 0;
    for (int colour = 0; colour < ncolours(pb) && st == FMO_OK; ++colour) {
      const int64_t q1 = colour_end(pb, order, q0, cnt, colour);
      FMO_PARALLEL_FOR
      for (int64_t q = q0; q < q1; ++q) piv[order[q]] = pivot_of(pb, mask, curv, piv, order[q]);
      for (int64_t q = q0; q < q1; ++q) {
        const double v = piv[order[q]];
        if (st != FMO_OK)
          piv[order[q]] = 0.0;
        else if (!(v > 0.0))
          st = isfinite(v) ? FMO_ERR_NOT_PD : FMO_ERR_NONFINITE;
      }
      q0 = q1;
    }
  }
  free(order);
  return st;
}

/* Forward solve (P + E) x = g at voxel j: x_j = (g_j + beta sum_{k before j} x_k) / P_j. */
static double forward_of(const fmo_problem *pb, const uint8_t *mask, const double *piv, const double *g,
                         const double *x, int64_t j) {
  int64_t nb[6];
  const int c = neighbours(pb, mask, j, nb);
  const int64_t rj = rank_of(pb, j);
  double s = g[j];
  for (int k = 0; k < c; ++k)
    if (rank_of(pb, nb[k]) < rj) s += pb->beta * x[nb[k]];
  return s / piv[j];
}

/* Backward solve (P + E^T) p = P x at voxel j: p_j = x_j + beta sum_{k after j} p_k / P_j. */
static double backward_of(const fmo_problem *pb, const uint8_t *mask, const double *piv, const double *x,
                          const double *p, int64_t j) {
  int64_t nb[6];
  const int c = neighbours(pb, mask, j, nb);
  const int64_t rj = rank_of(pb, j);
  double s = 0.0;
  for (int k = 0; k < c; ++k)
    if (rank_of(pb, nb[k]) > rj) s += p[nb[k]];
  return x[j] + pb->beta * s / piv[j];
}

int fmo_apply(const fmo_problem *pb, const uint8_t *mask, const double *piv, const double *g,
              double *p) {
  if (check_pb(pb) || !mask || !piv || !g || !p) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  double *x = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  if (!order || !x) return FMO_ERR_ARG;
  const int64_t cnt = build_order(pb, mask, order);
  /* runs of one colour in the elimination order (natural order: one run);
   * within a run of several colours' order no voxel uses another of the run
   * (independent sets of the 7-point stencil), so its voxels may be visited
   * in any order */
  int64_t bound[4] = {0, cnt, cnt, cnt};
  const int nc = independent_colours(pb) ? ncolours(pb) : 1;
  for (int colour = 0; colour < nc && nc > 1; ++colour)
    bound[colour + 1] = colour_end(pb, order, bound[colour], cnt, colour);
  /* forward: (P + E) x = g, E = strictly lower part of H (entries -beta) */
  for (int r = 0; r < nc; ++r) {
    if (nc == 1) {
      for (int64_t q = 0; q < cnt; ++q) x[order[q]] = forward_of(pb, mask, piv, g, x, order[q]);
    } else {
      FMO_PARALLEL_FOR
      for (int64_t q = bound[r]; q < bound[r + 1]; ++q) x[order[q]] = forward_of(pb, mask, piv, g, x, order[q]);
    }
  }
  /* backward: (P + E^T) p = P x */
  for (int64_t j = 0; j < n; ++j) p[j] = 0.0;
  for (int r = nc - 1; r >= 0; --r) {
    if (nc == 1) {
      for (int64_t q = cnt - 1; q >= 0; --q) p[order[q]] = backward_of(pb, mask, piv, x, p, order[q]);
    } else {
      FMO_PARALLEL_FOR
      for (int64_t q = bound[r + 1] - 1; q >= bound[r]; --q) p[order[q]] = backward_of(pb, mask, piv, x, p, order[q]);
    }
  }
  free(order);
  free(x);
  return FMO_OK;
}

/* (C^T C)_jj: first order the in-mask neighbour count; second order the sum of
 * squared coefficients of the rows through j (4 as centre, 1 as an end). */
static double reg_diag1(const fmo_problem *pb, const uint8_t *mask, int64_t j) {
  if (!mask[j]) return 0.0;
  if (!second_order(pb)) {
    int64_t nb[6];
    return (double)neighbours(pb, mask, j, nb);
  }
  double d = 0.0;
  int64_t c[3];
  coords(pb, j, c);
  for (int a = 0; a < 3; ++a) {
    const int64_t s = stride(pb, a);
    d += 4.0 * row2(pb, mask, j, a);
    if (c[a] > 0) d += row2(pb, mask, j - s, a);
    if (c[a] < extent(pb, a) - 1) d += row2(pb, mask, j + s, a);
  }
  return d;
}

int fmo_reg_diag(const fmo_problem *pb, const uint8_t *mask, double *out) {
  if (check_pb(pb) || !mask || !out) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  for (int64_t j = 0; j < n; ++j) out[j] = reg_diag1(pb, mask, j);
  return FMO_OK;
}

/* Pattern of H: slot q < 6 is the neighbour at +-1 along axis q/2 (sign by q%2),
 * slot q >= 6 (second order only) the one at +-2.  Returns the neighbour's
 * index, or -1 if it is outside the volume or the mask. */
static int npat(const fmo_problem *pb) { return second_order(pb) ? 12 : 6; }

static int64_t pat_nb(const fmo_problem *pb, const uint8_t *mask, int64_t j, int q) {
  const int a = (q % 6) / 2, dist = q < 6 ? 1 : 2, sgn = (q % 2) ? 1 : -1;
  int64_t c[3];
  coords(pb, j, c);
  const int64_t t = c[a] + sgn * dist;
  if (t < 0 || t >= extent(pb, a)) return -1;
  const int64_t k = j + sgn * dist * stride(pb, a);
  return mask[k] ? k : -1;
}

/* The slot of neighbour k in j's pattern, or -1. */
static int pat_slot(const fmo_problem *pb, const uint8_t *mask, int64_t j, int64_t k) {
  for (int q = 0; q < npat(pb); ++q)
    if (pat_nb(pb, mask, j, q) == k) return q;
  return -1;
}

/* (C^T C)_jk for a pattern neighbour k = j +- dist along axis a. */
static double reg_off(const fmo_problem *pb, const uint8_t *mask, int64_t j, int q) {
  if (!second_order(pb)) return -1.0;
  const int a = (q % 6) / 2, sgn = (q % 2) ? 1 : -1;
  const int64_t s = stride(pb, a);
  if (q < 6) /* rows centred at j and at the neighbour each give (-2)(1) */
    return -2.0 * row2(pb, mask, j, a) - 2.0 * row2(pb, mask, j + sgn * s, a);
  return (double)row2(pb, mask, j + sgn * s, a); /* the row centred between them: (1)(1) */
}

int fmo_ic_general(const fmo_problem *pb, const uint8_t *mask, const double *curv, const double *g,
                   double *p, double *piv) {
  if (check_pb(pb) || !mask || !curv || !g || !p) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  const int np = npat(pb);
  const double b = pb->beta;
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  double *D = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *L = (double *)calloc((size_t)(n ? n : 1) * 12, sizeof(double)); /* L[j][slot of k], k earlier */
  double *y = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  if (!order || !D || !L || !y) return FMO_ERR_ARG;
  const int64_t cnt = build_order(pb, mask, order);
  int st = FMO_OK;
  for (int64_t t = 0; t < cnt && st == FMO_OK; ++t) {
    const int64_t j = order[t];
    const int64_t rj = rank_of(pb, j);
    /* earlier pattern neighbours of j, in elimination order */
    int64_t lk[12];
    int lq[12], m = 0;
    for (int q = 0; q < np; ++q) {
      const int64_t k = pat_nb(pb, mask, j, q);
      if (k >= 0 && rank_of(pb, k) < rj) {
        int i = m++;
        while (i > 0 && rank_of(pb, lk[i - 1]) > rank_of(pb, k)) {
          lk[i] = lk[i - 1];
          lq[i] = lq[i - 1];
          --i;
        }
        lk[i] = k;
        lq[i] = q;
      }
    }
    double dj = curv[j] + b * reg_diag1(pb, mask, j);
    for (int u = 0; u < m; ++u) {
      const int64_t k = lk[u];
      double s = b * reg_off(pb, mask, j, lq[u]);
      for (int w = 0; w < u; ++w) { /* m = lk[w] precedes k: is it also in k's pattern? */
        const int qk = pat_slot(pb, mask, k, lk[w]);
        if (qk >= 0) s -= L[j * 12 + lq[w]] * L[k * 12 + qk] * D[lk[w]];
      }
      const double ljk = s / D[k];
      L[j * 12 + lq[u]] = ljk;
      dj -= ljk * ljk * D[k];
    }
    D[j] = dj;
    if (!(dj > 0.0)) st = isfinite(dj) ? FMO_ERR_NOT_PD : FMO_ERR_NONFINITE;
  }
  if (st == FMO_OK) {
    /* forward L y = g, then backward L^T p = D^{-1} y */
    for (int64_t t = 0; t < cnt; ++t) {
      const int64_t j = order[t];
      const int64_t rj = rank_of(pb, j);
      double s = g[j];
      for (int q = 0; q < np; ++q) {
        const int64_t k = pat_nb(pb, mask, j, q);
        if (k >= 0 && rank_of(pb, k) < rj) s -= L[j * 12 + q] * y[k];
      }
      y[j] = s;
    }
    for (int64_t j = 0; j < n; ++j) p[j] = 0.0;
    for (int64_t t = cnt - 1; t >= 0; --t) {
      const int64_t j = order[t];
      const int64_t rj = rank_of(pb, j);
      double s = y[j] / D[j];
      for (int q = 0; q < np; ++q) {
        const int64_t k = pat_nb(pb, mask, j, q);
        if (k >= 0 && rank_of(pb, k) > rj) s -= L[k * 12 + pat_slot(pb, mask, k, j)] * p[k];
      }
      p[j] = s;
    }
  }
  if (piv)
    for (int64_t j = 0; j < n; ++j) piv[j] = D[j];
  free(order);
  free(D);
  free(L);
  free(y);
  return st;
}

static double dot_mask(const uint8_t *mask, int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j)
    if (mask[j]) s += a[j] * b[j];
  return s;
}

/* Psi at f + alpha z using precomputed pairs (z may be NULL). */
static double cost_at(const fmo_problem *pb, const pairs_t *pr, const uint8_t *mask,
                      const double *f, const double *z, double alpha, double *tmp, double *lap) {
  const int64_t n = nvox(pb);
  FMO_PARALLEL_FOR
  for (int64_t j = 0; j < n; ++j) tmp[j] = mask[j] ? f[j] + (z ? alpha * z[j] : 0.0) : 0.0;
  /* per-voxel costs into lap, then their sum in natural order */
  FMO_PARALLEL_FOR
  for (int64_t j = 0; j < n; ++j) {
    double a = 0.0, b, c;
    if (mask[j]) voxel_terms(pr, n, j, tmp[j], &a, &b, &c);
    lap[j] = a;
  }
  double phi_sum = 0.0;
  for (int64_t j = 0; j < n; ++j)
    if (mask[j]) phi_sum += lap[j];
  fmo_laplacian(pb, mask, tmp, lap);
  return phi_sum + 0.5 * pb->beta * dot_mask(mask, n, tmp, lap);
}

int fmo_cost(const fmo_problem *pb, const double *zhat, const uint8_t *mask, const double *f,
             double *psi) {
  if (check_pb(pb) || !zhat || !mask || !f || !psi) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  pairs_t pr;
  if (pairs_build(pb, zhat, mask, &pr)) return FMO_ERR_ARG;
  double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
  double *lap = (double *)malloc(sizeof(double) * (size_t)n);
  *psi = cost_at(pb, &pr, mask, f, NULL, 0.0, tmp, lap);
  free(tmp);
  free(lap);
  pairs_free(&pr);
  return FMO_OK;
}

int fmo_solve(const fmo_problem *pb, const double *zhat, const uint8_t *mask, const double *f0,
              double *f, double *trace, double *mls) {
  if (check_pb(pb) || !zhat || !mask || !f0 || !f) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  const double beta = pb->beta;
  pairs_t pr;
  if (pairs_build(pb, zhat, mask, &pr)) return FMO_ERR_ARG;
  const size_t nb = sizeof(double) * (size_t)(n ? n : 1);
  double *dphi = (double *)malloc(nb), *curv = (double *)malloc(nb), *g = (double *)malloc(nb);
  double *gprev = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *zprev = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *p = (double *)malloc(nb), *z = (double *)malloc(nb), *piv = (double *)malloc(nb);
  double *lap = (double *)malloc(nb), *lapz = (double *)malloc(nb), *tmp = (double *)malloc(nb);
  double *tmp2 = (double *)malloc(nb);
  int st = FMO_OK;
  /* IC_t factor: the diagonal and one row per offset of its pattern */
  double *lict = NULL;
  if (pb->precond == FMO_PRECOND_ICT) {
    int32_t offs[3 * FMO_ICT_MAXOFF], noff = 0;
    if (second_order(pb) || fmo_ict_offsets(pb->ict_level, 9, offs, &noff)) st = FMO_ERR_ARG;
    else lict = (double *)malloc(nb * (size_t)(1 + noff));
  }
  for (int64_t j = 0; j < n; ++j) f[j] = mask[j] ? f0[j] : 0.0;
  double gtp_prev = 0.0;

  for (int it = 0; it < pb->niter && st == FMO_OK; ++it) {
    /* gradient g = grad Phi + beta C^T C f, and the Huber curvature D
     * (per-voxel costs into tmp, summed in natural order below) */
    FMO_PARALLEL_FOR
    for (int64_t j = 0; j < n; ++j) {
      double a = 0, b = 0, c = 0;
      if (mask[j]) voxel_terms(&pr, n, j, f[j], &a, &b, &c);
      tmp[j] = a;
      dphi[j] = b;
      curv[j] = c;
    }
    double phi_sum = 0.0;
    for (int64_t j = 0; j < n; ++j) phi_sum += tmp[j];
    fmo_laplacian(pb, mask, f, lap);
    FMO_PARALLEL_FOR
    for (int64_t j = 0; j < n; ++j) g[j] = mask[j] ? dphi[j] + beta * lap[j] : 0.0;
    const double cost = phi_sum + 0.5 * beta * dot_mask(mask, n, f, lap);

    /* precondition p = P^{-1} g */
    if (pb->precond == FMO_PRECOND_IC0 && second_order(pb)) {
      st = fmo_ic_general(pb, mask, curv, g, p, NULL);
      if (st) break;
    } else if (pb->precond == FMO_PRECOND_IC0) {
      st = fmo_factor(pb, mask, curv, piv);
      if (st) break;
      fmo_apply(pb, mask, piv, g, p);
    } else if (pb->precond == FMO_PRECOND_ICT) {
      st = fmo_ict_factor(pb, mask, curv, lict);
      if (st) break;
      fmo_ict_apply(pb, mask, lict, g, p);
    } else if (pb->precond == FMO_PRECOND_DIAG) {
      for (int64_t j = 0; j < n; ++j) {
        if (!mask[j]) {
          p[j] = 0.0;
          continue;
        }
        const double h = curv[j] + beta * reg_diag1(pb, mask, j);
        if (!(h > 0.0)) {
          st = FMO_ERR_NOT_PD;
          break;
        }
        p[j] = g[j] / h;
      }
      if (st) break;
    } else {
      for (int64_t j = 0; j < n; ++j) p[j] = g[j];
    }

    /* Polak-Ribiere conjugacy and the search direction */
    const double gtp = dot_mask(mask, n, g, p);
    double mu = 0.0;
    if (it > 0 && gtp_prev != 0.0) mu = (gtp - dot_mask(mask, n, gprev, p)) / gtp_prev;
    double ztg = -gtp + mu * dot_mask(mask, n, zprev, g);
    int restart = 0;
    if (ztg >= 0.0) {
      mu = 0.0;
      ztg = -gtp;
      restart = 1;
    }
    FMO_PARALLEL_FOR
    for (int64_t j = 0; j < n; ++j) z[j] = mask[j] ? -p[j] + mu * zprev[j] : 0.0;

    /* monotone line search on f(alpha) = Psi(f + alpha z) */
    fmo_laplacian(pb, mask, z, lapz);
    const double A = dot_mask(mask, n, z, lap);   /* z^T C^T C f */
    const double B = dot_mask(mask, n, z, lapz);  /* ||C z||^2   */
    double alpha = 0.0;
    if (mls) mls[(int64_t)it * (pb->nmls + 1)] = cost;
    for (int k = 0; k < pb->nmls; ++k) {
      double s1 = 0.0, s2 = 0.0;
      if (k == 0) {
        for (int64_t j = 0; j < n; ++j)
          if (mask[j]) {
            s1 += z[j] * dphi[j];
            s2 += z[j] * z[j] * curv[j];
          }
      } else {
        /* derivative and curvature at f + alpha z into tmp, tmp2; sums in natural order */
        FMO_PARALLEL_FOR
        for (int64_t j = 0; j < n; ++j)
          if (mask[j]) {
            double a, b, c;
            voxel_terms(&pr, n, j, f[j] + alpha * z[j], &a, &b, &c);
            tmp[j] = b;
            tmp2[j] = c;
          }
        for (int64_t j = 0; j < n; ++j)
          if (mask[j]) {
            s1 += z[j] * tmp[j];
            s2 += z[j] * z[j] * tmp2[j];
          }
      }
      const double den = s2 + beta * B;
      if (!(den > 0.0)) {
        if (mls)
          for (int kk = k; kk < pb->nmls; ++kk)
            mls[(int64_t)it * (pb->nmls + 1) + kk + 1] =
                mls[(int64_t)it * (pb->nmls + 1) + kk];
        break;
      }
      alpha = alpha - (s1 + beta * A + alpha * beta * B) / den;
      if (mls) mls[(int64_t)it * (pb->nmls + 1) + k + 1] = cost_at(pb, &pr, mask, f, z, alpha, tmp, tmp2);
    }
    if (!isfinite(alpha)) {
      st = FMO_ERR_NONFINITE;
      break;
    }
    if (trace) {
      double *t = trace + (int64_t)it * FMO_TR_W;
      t[FMO_TR_COST] = cost;
      t[FMO_TR_GTP] = gtp;
      t[FMO_TR_MU] = mu;
      t[FMO_TR_RESTART] = restart;
      t[FMO_TR_ALPHA] = alpha;
      t[FMO_TR_ZTG] = ztg;
      t[FMO_TR_B] = B;
      t[FMO_TR_GNORM2] = dot_mask(mask, n, g, g);
    }
    FMO_PARALLEL_FOR
    for (int64_t j = 0; j < n; ++j) {
      if (mask[j]) f[j] += alpha * z[j];
      gprev[j] = g[j];
      zprev[j] = z[j];
    }
    gtp_prev = gtp;
  }
  if (trace && st == FMO_OK) {
    double *t = trace + (int64_t)pb->niter * FMO_TR_W;
    for (int c = 0; c < FMO_TR_W; ++c) t[c] = 0.0;
    t[FMO_TR_COST] = cost_at(pb, &pr, mask, f, NULL, 0.0, tmp, tmp2);
  }
  free(dphi);
  free(curv);
  free(g);
  free(gprev);
  free(zprev);
  free(p);
  free(z);
  free(piv);
  free(lap);
  free(lapz);
  free(tmp);
  free(tmp2);
  free(lict);
  pairs_free(&pr);
  return st;
}

int fmo_init_waterfat_sweep(const fmo_problem *pb, const double *zhat, const uint8_t *mask,
                            double dfat_hz, int32_t nsweep, double *ftilde) {
  if (check_pb(pb) || !zhat || !mask || !ftilde || nsweep < 2) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  pairs_t pr;
  if (pairs_build(pb, zhat, mask, &pr)) return FMO_ERR_ARG;
  const double h = fabs(dfat_hz) / 2.0;
  for (int64_t j = 0; j < n; ++j) {
    if (!mask[j]) {
      ftilde[j] = 0.0;
      continue;
    }
    double best = INFINITY, bestf = 0.0;
    for (int s = 0; s < nsweep; ++s) {
      const double fs = -h + 2.0 * h * s / (nsweep - 1);
      double a, b, c;
      voxel_terms(&pr, n, j, fs, &a, &b, &c);
      if (a < best) {
        best = a;
        bestf = fs;
      }
    }
    ftilde[j] = bestf;
  }
  pairs_free(&pr);
  return FMO_OK;
}

int fmo_pwls_weights(int64_t n, int32_t ncoil, int32_t L, const double *y, const double *s,
                     const double *gam, double *rho) {
  if (n < 0 || ncoil < 1 || L < 2 || !y || !gam || !rho || (!s && ncoil != 1))
    return FMO_ERR_ARG;
  double *a = (double *)malloc(sizeof(double) * L);
  if (!a) return FMO_ERR_ARG;
  for (int64_t j = 0; j < n; ++j) {
    double ss = 0.0;
    for (int c = 0; c < ncoil; ++c) {
      const double sre = s ? s[2 * ((int64_t)c * n + j)] : 1.0;
      const double sim = s ? s[2 * ((int64_t)c * n + j) + 1] : 0.0;
      ss += sre * sre + sim * sim;
    }
    for (int l = 0; l < L; ++l) {
      a[l] = 0.0;
      for (int c = 0; c < ncoil; ++c) {
        const double sm = s ? hypot(s[2 * ((int64_t)c * n + j)], s[2 * ((int64_t)c * n + j) + 1])
                            : 1.0;
        const double *yy = y + 2 * (((int64_t)c * L + l) * n + j);
        a[l] += sm * hypot(yy[0], yy[1]);
      }
    }
    double r = 0.0;
    for (int m = 0; m < L; ++m)
      for (int k = 0; k < L; ++k)
        r += hypot(gam[2 * (m * L + k)], gam[2 * (m * L + k) + 1]) * a[m] * a[k];
    rho[j] = ss > 0.0 ? r / ss : 0.0;
  }
  free(a);
  return FMO_OK;
}

/* out = (2 diag(rho) + beta L) v over the mask */
static void pwls_apply(const fmo_problem *pb, const uint8_t *mask, const double *rho,
                       const double *v, double *lap, double *out) {
  const int64_t n = nvox(pb);
  fmo_laplacian(pb, mask, v, lap);
  for (int64_t j = 0; j < n; ++j) out[j] = mask[j] ? 2.0 * rho[j] * v[j] + pb->beta * lap[j] : 0.0;
}

int fmo_pwls_cg(const fmo_problem *pb, const uint8_t *mask, const double *rho,
                const double *ftilde, int32_t niters, double *f) {
  if (check_pb(pb) || !mask || !rho || !ftilde || !f || niters < 0) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  const size_t nb = sizeof(double) * (size_t)(n ? n : 1);
  double *r = (double *)malloc(nb), *d = (double *)malloc(nb), *ad = (double *)malloc(nb);
  double *lap = (double *)malloc(nb);
  for (int64_t j = 0; j < n; ++j) f[j] = mask[j] ? ftilde[j] : 0.0;
  pwls_apply(pb, mask, rho, f, lap, ad);
  for (int64_t j = 0; j < n; ++j) {
    r[j] = mask[j] ? 2.0 * rho[j] * ftilde[j] - ad[j] : 0.0;
    d[j] = r[j];
  }
  double rs = dot_mask(mask, n, r, r);
  for (int it = 0; it < niters; ++it) {
    pwls_apply(pb, mask, rho, d, lap, ad);
    const double dad = dot_mask(mask, n, d, ad);
    if (!(dad > 0.0)) break;
    const double a = rs / dad;
    for (int64_t j = 0; j < n; ++j) {
      f[j] += a * d[j];
      r[j] -= a * ad[j];
    }
    const double rs2 = dot_mask(mask, n, r, r);
    const double bb = rs2 / rs;
    for (int64_t j = 0; j < n; ++j) d[j] = r[j] + bb * d[j];
    rs = rs2;
    if (rs == 0.0) break;
  }
  free(r);
  free(d);
  free(ad);
  free(lap);
  return FMO_OK;
}

/* Exact second derivative of the per-voxel data term at fj. */
static double voxel_hess(const pairs_t *pr, int64_t n, int64_t j, double fj) {
  double h = 0.0;
  for (int q = 0; q < pr->np; ++q) {
    const double w = pr->w[(int64_t)q * n + j];
    const double d = pr->d[q];
    const double x = pr->a[(int64_t)q * n + j] + d * fj;
    h += w * d * d * cos(x);
  }
  return h;
}

int fmo_adjoint(const fmo_problem *pb, const double *zhat, const uint8_t *mask, const double *fhat,
                const double *dldf, int32_t maxit, double rtol, double *v, double *dldbeta,
                double *dzhat, int32_t *iters) {
  if (check_pb(pb) || !zhat || !mask || !fhat || !dldf || !v || maxit < 0) return FMO_ERR_ARG;
  if (pb->precond == FMO_PRECOND_ICT) return FMO_ERR_ARG; /* adjoint CG preconditioners: IC(0), diag, none */
  const int64_t n = nvox(pb);
  const int L = pb->necho;
  const double beta = pb->beta;
  pairs_t pr;
  if (pairs_build(pb, zhat, mask, &pr)) return FMO_ERR_ARG;
  const size_t nb = sizeof(double) * (size_t)(n ? n : 1);
  double *h = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *curv = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *piv = (double *)malloc(nb), *r = (double *)malloc(nb), *z = (double *)malloc(nb);
  double *d = (double *)malloc(nb), *hd = (double *)malloc(nb), *lap = (double *)malloc(nb);
  int st = FMO_OK;
  for (int64_t j = 0; j < n; ++j) {
    if (!mask[j]) continue;
    double a, b;
    voxel_terms(&pr, n, j, fhat[j], &a, &b, &curv[j]);
    h[j] = voxel_hess(&pr, n, j, fhat[j]);
  }
  /* preconditioner: IC(0) (or the chosen variant) of the Huber model */
  if (pb->precond == FMO_PRECOND_IC0 && !second_order(pb)) st = fmo_factor(pb, mask, curv, piv);
  int it = 0;
  if (st == FMO_OK) {
    for (int64_t j = 0; j < n; ++j) {
      v[j] = 0.0;
      r[j] = mask[j] ? dldf[j] : 0.0;
      d[j] = 0.0;
    }
    const double bnorm = sqrt(dot_mask(mask, n, r, r));
    double rho_prev = 0.0;
    for (it = 0; it < maxit; ++it) {
      if (sqrt(dot_mask(mask, n, r, r)) <= rtol * bnorm) break;
      if (pb->precond == FMO_PRECOND_IC0 && second_order(pb)) {
        st = fmo_ic_general(pb, mask, curv, r, z, NULL);
        if (st) break;
      } else if (pb->precond == FMO_PRECOND_IC0) {
        fmo_apply(pb, mask, piv, r, z);
      } else {
        for (int64_t j = 0; j < n; ++j) {
          const double hh = curv[j] + beta * reg_diag1(pb, mask, j);
          z[j] = mask[j] ? (pb->precond == FMO_PRECOND_DIAG ? r[j] / hh : r[j]) : 0.0;
        }
      }
      const double rho = dot_mask(mask, n, r, z);
      const double bcg = (it > 0 && rho_prev != 0.0) ? rho / rho_prev : 0.0;
      for (int64_t j = 0; j < n; ++j) d[j] = mask[j] ? z[j] + bcg * d[j] : 0.0;
      fmo_laplacian(pb, mask, d, lap);
      for (int64_t j = 0; j < n; ++j) hd[j] = mask[j] ? h[j] * d[j] + beta * lap[j] : 0.0;
      const double dhd = dot_mask(mask, n, d, hd);
      if (!(dhd > 0.0)) {
        st = FMO_ERR_NOT_PD;
        break;
      }
      const double alpha = rho / dhd;
      for (int64_t j = 0; j < n; ++j) {
        v[j] += alpha * d[j];
        r[j] -= alpha * hd[j];
      }
      rho_prev = rho;
    }
  }
  if (iters) *iters = it;
  if (st == FMO_OK) {
    fmo_laplacian(pb, mask, fhat, lap);
    if (dldbeta) *dldbeta = -dot_mask(mask, n, v, lap);
    if (dzhat) {
      for (int64_t k = 0; k < 2 * (int64_t)L * n; ++k) dzhat[k] = 0.0;
      /* g_j = sum_{m<n} 4 pi dt Im(Gamma_mn conj(zhat_m) zhat_n e^{i 2 pi dt f_j});
       * for G = Im(u conj(z_m) z_n): dG/dz_n = i conj(u) z_m, dG/dz_m = -i u z_n */
      for (int64_t j = 0; j < n; ++j) {
        if (!mask[j] || v[j] == 0.0) continue;
        int q = 0;
        for (int m = 0; m < L; ++m)
          for (int k = m + 1; k < L; ++k, ++q) {
            const double dt = pb->te[m] - pb->te[k];
            const double th = TWO_PI * dt * fhat[j];
            const double gre = pb->gam[2 * (m * L + k)], gim = pb->gam[2 * (m * L + k) + 1];
            const double ure = gre * cos(th) - gim * sin(th), uim = gre * sin(th) + gim * cos(th);
            const double *zm = zhat + 2 * ((int64_t)m * n + j), *zn = zhat + 2 * ((int64_t)k * n + j);
            const double c = -v[j] * 2.0 * TWO_PI * dt;
            /* i conj(u) z_m */
            const double an_re = -(ure * zm[1] - uim * zm[0]), an_im = ure * zm[0] + uim * zm[1];
            /* -i u z_n */
            const double pre = ure * zn[0] - uim * zn[1], pim = ure * zn[1] + uim * zn[0];
            const double am_re = pim, am_im = -pre;
            dzhat[2 * ((int64_t)k * n + j)] += c * an_re;
            dzhat[2 * ((int64_t)k * n + j) + 1] += c * an_im;
            dzhat[2 * ((int64_t)m * n + j)] += c * am_re;
            dzhat[2 * ((int64_t)m * n + j) + 1] += c * am_im;
          }
      }
    }
  }
  free(h);
  free(curv);
  free(piv);
  free(r);
  free(z);
  free(d);
  free(hd);
  free(lap);
  pairs_free(&pr);
  return st;
}

/* ---------------------------------------------------------------------------
 * Incomplete Cholesky with a drop tolerance (IC_t), Sec. III-B.
 */

int fmo_ict_offsets(int32_t level, int32_t side, int32_t *offs, int32_t *count) {
  if (level < 0 || side < 3 || side % 2 == 0 || side > 15 || !offs || !count) return FMO_ERR_ARG;
  const int S = side, N = S * S * S, BIG = 1 << 20;
  int *lev = (int *)malloc(sizeof(int) * (size_t)N * N);
  if (!lev) return FMO_ERR_ARG;
  /* structural nonzeros of the 7-point H (level 0); z fastest */
  for (int i = 0; i < N * N; ++i) lev[i] = BIG;
  for (int i = 0; i < N; ++i) {
    const int x = i / (S * S), y = (i / S) % S, z = i % S;
    lev[i * N + i] = 0;
    const int nb[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int q = 0; q < 6; ++q) {
      const int a = x + nb[q][0], b = y + nb[q][1], c = z + nb[q][2];
      if (a < 0 || a >= S || b < 0 || b >= S || c < 0 || c >= S) continue;
      lev[i * N + (a * S + b) * S + c] = 0;
    }
  }
  /* symbolic elimination in natural order: eliminating k gives every pair
   * (i, j) of later voxels the level lev(i,k) + lev(k,j) + 1 if smaller */
  for (int k = 0; k < N; ++k)
    for (int i = k + 1; i < N; ++i) {
      const int lik = lev[i * N + k];
      if (lik > level) continue;
      for (int j = k + 1; j < N; ++j) {
        const int lkj = lev[k * N + j];
        if (lkj > level) continue;
        const int v = lik + lkj + 1;
        if (v < lev[i * N + j]) lev[i * N + j] = v;
      }
    }
  const int c0 = S / 2, centre = (c0 * S + c0) * S + c0;
  int cnt = 0;
  /* earlier voxels in the centre row's pattern, by descending (dx, dy, dz) */
  for (int dx = S; dx >= -S; --dx)
    for (int dy = S; dy >= -S; --dy)
      for (int dz = S; dz >= -S; --dz) {
        const int a = c0 - dx, b = c0 - dy, c = c0 - dz;
        if (a < 0 || a >= S || b < 0 || b >= S || c < 0 || c >= S) continue;
        const int k = (a * S + b) * S + c;
        if (k >= centre || lev[centre * N + k] > level) continue;
        if (cnt == FMO_ICT_MAXOFF) {
          free(lev);
          return FMO_ERR_ARG;
        }
        offs[3 * cnt] = dx;
        offs[3 * cnt + 1] = dy;
        offs[3 * cnt + 2] = dz;
        ++cnt;
      }
  free(lev);
  *count = cnt;
  return FMO_OK;
}

/* Voxel j - o if it lies inside the volume and the mask, else -1. */
static int64_t ict_nb(const fmo_problem *pb, const uint8_t *mask, int64_t j, const int32_t *o) {
  int64_t c[3];
  coords(pb, j, c);
  const int64_t x = c[0] - o[0], y = c[1] - o[1], z = c[2] - o[2];
  if (x < 0 || x >= pb->nx || y < 0 || y >= pb->ny || z < 0 || z >= pb->nz) return -1;
  const int64_t k = (x * pb->ny + y) * pb->nz + z;
  return mask[k] ? k : -1;
}

/* Entry H_jk of H = diag(curv) + beta C^T C. */
static double ict_h(const fmo_problem *pb, const uint8_t *mask, const double *curv, int64_t j, int64_t k) {
  int64_t nb[6];
  const int c = neighbours(pb, mask, j, nb);
  if (j == k) return curv[j] + pb->beta * c;
  for (int q = 0; q < c; ++q)
    if (nb[q] == k) return -pb->beta;
  return 0.0;
}

/* Pattern positions of row j (earlier voxels), ascending: returns how many;
 * idx[] the voxel indices, slot[] their offset number. */
static int ict_row(const fmo_problem *pb, const uint8_t *mask, const int32_t *offs, int noff, int64_t j,
                   int64_t *idx, int *slot) {
  int m = 0;
  for (int u = 0; u < noff; ++u) {
    const int64_t k = ict_nb(pb, mask, j, offs + 3 * u);
    if (k < 0) continue;
    int i = m++;
    while (i > 0 && idx[i - 1] > k) {
      idx[i] = idx[i - 1];
      slot[i] = slot[i - 1];
      --i;
    }
    idx[i] = k;
    slot[i] = u;
  }
  return m;
}

int fmo_ict_factor(const fmo_problem *pb, const uint8_t *mask, const double *curv, double *L) {
  if (check_pb(pb) || !mask || !curv || !L || second_order(pb) || !(pb->ict_factor >= 0.0)) return FMO_ERR_ARG;
  int32_t offs[3 * FMO_ICT_MAXOFF], noff = 0;
  if (fmo_ict_offsets(pb->ict_level, 9, offs, &noff)) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  for (int64_t i = 0; i < (int64_t)(1 + noff) * n; ++i) L[i] = 0.0;
  /* H_max: the largest magnitude in H (diagonal, or beta off the diagonal) */
  double hmax = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (!mask[j]) continue;
    int64_t nb[6];
    const int c = neighbours(pb, mask, j, nb);
    const double hjj = fabs(curv[j] + pb->beta * c);
    if (hjj > hmax) hmax = hjj;
    if (c > 0 && pb->beta > hmax) hmax = pb->beta;
  }
  const double tol = pb->ict_factor * hmax;
  int64_t rj[FMO_ICT_MAXOFF], rk[FMO_ICT_MAXOFF];
  int sj[FMO_ICT_MAXOFF], sk[FMO_ICT_MAXOFF];
  for (int64_t j = 0; j < n; ++j) {
    if (!mask[j]) continue;
    const int mj = ict_row(pb, mask, offs, noff, j, rj, sj);
    double diag = ict_h(pb, mask, curv, j, j);
    for (int a = 0; a < mj; ++a) {
      const int64_t k = rj[a];
      double s = ict_h(pb, mask, curv, j, k);
      /* m < k in both rows' patterns: row j's positions before k that row k also holds */
      const int mk = ict_row(pb, mask, offs, noff, k, rk, sk);
      for (int b = 0; b < a; ++b)
        for (int e = 0; e < mk; ++e)
          if (rk[e] == rj[b]) s -= L[(int64_t)(1 + sj[b]) * n + j] * L[(int64_t)(1 + sk[e]) * n + k];
      double v = s / L[k];
      /* drop test of reading R21: |L_jk| < tol ||H(k:N, k)||_1 */
      int64_t nb[6];
      const int c = neighbours(pb, mask, k, nb);
      double colnorm = fabs(curv[k] + pb->beta * c);
      for (int q = 0; q < c; ++q)
        if (nb[q] > k) colnorm += pb->beta;
      if (fabs(v) < tol * colnorm) v = 0.0;
      L[(int64_t)(1 + sj[a]) * n + j] = v;
    }
    for (int a = 0; a < mj; ++a) {
      const double v = L[(int64_t)(1 + sj[a]) * n + j];
      diag -= v * v;
    }
    if (!(diag > 0.0)) return isfinite(diag) ? FMO_ERR_NOT_PD : FMO_ERR_NONFINITE;
    L[j] = sqrt(diag);
  }
  return FMO_OK;
}

int fmo_ict_apply(const fmo_problem *pb, const uint8_t *mask, const double *L, const double *g, double *p) {
  if (check_pb(pb) || !mask || !L || !g || !p) return FMO_ERR_ARG;
  int32_t offs[3 * FMO_ICT_MAXOFF], noff = 0;
  if (fmo_ict_offsets(pb->ict_level, 9, offs, &noff)) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  double *y = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  if (!y) return FMO_ERR_ARG;
  int64_t rj[FMO_ICT_MAXOFF];
  int sj[FMO_ICT_MAXOFF];
  /* forward: L y = g, natural order */
  for (int64_t j = 0; j < n; ++j) {
    if (!mask[j]) continue;
    const int mj = ict_row(pb, mask, offs, noff, j, rj, sj);
    double s = g[j];
    for (int a = 0; a < mj; ++a) s -= L[(int64_t)(1 + sj[a]) * n + j] * y[rj[a]];
    y[j] = s / L[j];
  }
  /* backward: L^T p = y, reverse order; row j of L^T holds L_ij of the later
   * voxels i = j + o_u (ascending i) */
  for (int64_t j = 0; j < n; ++j) p[j] = 0.0;
  for (int64_t j = n - 1; j >= 0; --j) {
    if (!mask[j]) continue;
    /* later voxels i = j + o_u inside the volume and the mask, ascending */
    int64_t ri[FMO_ICT_MAXOFF];
    int si[FMO_ICT_MAXOFF], m = 0;
    for (int u = 0; u < noff; ++u) {
      const int32_t up[3] = {-offs[3 * u], -offs[3 * u + 1], -offs[3 * u + 2]};
      const int64_t i = ict_nb(pb, mask, j, up);
      if (i < 0) continue;
      int t = m++;
      while (t > 0 && ri[t - 1] > i) {
        ri[t] = ri[t - 1];
        si[t] = si[t - 1];
        --t;
      }
      ri[t] = i;
      si[t] = u;
    }
    double s = y[j];
    for (int a = 0; a < m; ++a) s -= L[(int64_t)(1 + si[a]) * n + ri[a]] * p[ri[a]];
    p[j] = s / L[j];
  }
  free(y);
  return FMO_OK;
}

int fmo_components(const fmo_problem *pb, int32_t ncoil, const double *y, const double *s,
                   const uint8_t *mask, const double *f, int32_t K, int32_t npeak, const double *fat_hz,
                   const double *fat_amp, double *out) {
  if (!pb || pb->nx < 1 || pb->ny < 1 || pb->nz < 1 || pb->necho < 1 || !pb->te || ncoil < 1 || !y ||
      (!s && ncoil != 1) || !mask || !f || !out || (K != 1 && K != 2))
    return FMO_ERR_ARG;
  if (K == 2 && (npeak < 1 || !fat_hz || !fat_amp)) return FMO_ERR_ARG;
  const int64_t n = nvox(pb);
  const int L = pb->necho;
  const int M = L * ncoil;
  /* gamma [L][K] */
  double *gre = (double *)calloc((size_t)L * K, sizeof(double));
  double *gim = (double *)calloc((size_t)L * K, sizeof(double));
  double *are = (double *)malloc(sizeof(double) * (size_t)M * K);
  double *aim = (double *)malloc(sizeof(double) * (size_t)M * K);
  if (!gre || !gim || !are || !aim) return FMO_ERR_ARG;
  for (int l = 0; l < L; ++l) {
    gre[l * K] = 1.0;
    if (K == 2)
      for (int p = 0; p < npeak; ++p) {
        gre[l * K + 1] += fat_amp[p] * cos(TWO_PI * fat_hz[p] * pb->te[l]);
        gim[l * K + 1] += fat_amp[p] * sin(TWO_PI * fat_hz[p] * pb->te[l]);
      }
  }
  for (int64_t j = 0; j < n; ++j) {
    double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};
    if (mask[j]) {
      /* A[(l, c)][k] = e^{i 2 pi f t_l} gamma_lk s_cj */
      for (int l = 0; l < L; ++l) {
        const double ph = TWO_PI * f[j] * pb->te[l];
        const double er = cos(ph), ei = sin(ph);
        for (int c = 0; c < ncoil; ++c) {
          const double sr = s ? s[2 * ((int64_t)c * n + j)] : 1.0;
          const double si = s ? s[2 * ((int64_t)c * n + j) + 1] : 0.0;
          for (int k = 0; k < K; ++k) {
            const double ur = er * gre[l * K + k] - ei * gim[l * K + k];
            const double ui = er * gim[l * K + k] + ei * gre[l * K + k];
            are[(l * ncoil + c) * K + k] = ur * sr - ui * si;
            aim[(l * ncoil + c) * K + k] = ur * si + ui * sr;
          }
        }
      }
      /* normal equations N = A^H A, b = A^H y */
      double nr[2][2] = {{0, 0}, {0, 0}}, ni[2][2] = {{0, 0}, {0, 0}}, br[2] = {0, 0}, bi[2] = {0, 0};
      for (int r = 0; r < M; ++r) {
        const int l = r / ncoil, c = r % ncoil;
        const double yr = y[2 * (((int64_t)c * L + l) * n + j)], yi = y[2 * (((int64_t)c * L + l) * n + j) + 1];
        for (int a = 0; a < K; ++a) {
          const double ar = are[r * K + a], ai = aim[r * K + a];
          br[a] += ar * yr + ai * yi;
          bi[a] += ar * yi - ai * yr;
          for (int b = 0; b < K; ++b) {
            const double cr = are[r * K + b], ci = aim[r * K + b];
            nr[a][b] += ar * cr + ai * ci;
            ni[a][b] += ar * ci - ai * cr;
          }
        }
      }
      if (K == 1) {
        if (nr[0][0] > 0.0) {
          xr[0] = br[0] / nr[0][0];
          xi[0] = bi[0] / nr[0][0];
        }
      } else {
        /* 2x2 complex inverse: N^{-1} = adj(N) / det(N) */
        const double dr = nr[0][0] * nr[1][1] - ni[0][0] * ni[1][1] - (nr[0][1] * nr[1][0] - ni[0][1] * ni[1][0]);
        const double di = nr[0][0] * ni[1][1] + ni[0][0] * nr[1][1] - (nr[0][1] * ni[1][0] + ni[0][1] * nr[1][0]);
        const double dd = dr * dr + di * di;
        if (dd > 0.0) {
          /* y0 = N11 b0 - N01 b1, y1 = -N10 b0 + N00 b1; x = y / det */
          const double y0r = nr[1][1] * br[0] - ni[1][1] * bi[0] - (nr[0][1] * br[1] - ni[0][1] * bi[1]);
          const double y0i = nr[1][1] * bi[0] + ni[1][1] * br[0] - (nr[0][1] * bi[1] + ni[0][1] * br[1]);
          const double y1r = -(nr[1][0] * br[0] - ni[1][0] * bi[0]) + nr[0][0] * br[1] - ni[0][0] * bi[1];
          const double y1i = -(nr[1][0] * bi[0] + ni[1][0] * br[0]) + nr[0][0] * bi[1] + ni[0][0] * br[1];
          xr[0] = (y0r * dr + y0i * di) / dd;
          xi[0] = (y0i * dr - y0r * di) / dd;
          xr[1] = (y1r * dr + y1i * di) / dd;
          xi[1] = (y1i * dr - y1r * di) / dd;
        }
      }
    }
    for (int k = 0; k < K; ++k) {
      out[2 * ((int64_t)k * n + j)] = xr[k];
      out[2 * ((int64_t)k * n + j) + 1] = xi[k];
    }
  }
  free(gre);
  free(gim);
  free(are);
  free(aim);
  return FMO_OK;
}
