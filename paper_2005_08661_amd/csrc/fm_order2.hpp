// Second-order finite-difference regulariser (Sec. II eq. (cost) with C the
// second-order operator): one row f_{j-e} - 2 f_j + f_{j+e} per voxel j and
// axis e whose three voxels are inside the volume and the mask.  The row
// centred at j along axis a exists exactly when both a-neighbours of j are in
// the mask, i.e. when the neighbour code has both bits of the axis, so no
// extra per-voxel array is needed.  C^T C is a 13-point stencil:
//   (C^T C f)_j = sum_a [ -2 r_j (f_{j-e} - 2 f_j + f_{j+e})
//                         + r_{j+e} (f_j - 2 f_{j+e} + f_{j+2e})
//                         + r_{j-e} (f_{j-2e} - 2 f_{j-e} + f_j) ],
//   (C^T C)_jj  = sum_a [ 4 r_j + r_{j-e} + r_{j+e} ],
// with r the row indicators.  Passes for the diagonal and identity
// preconditioners (single volumes); arrays are padded by two x-planes so that
// the +-2 neighbour addresses stay in bounds.
#pragma once

#include "fm_stream.hpp"

namespace fm {

__device__ __forceinline__ bool row2(uint32_t c, int a) { return has_nb(c, 2 * a) && has_nb(c, 2 * a + 1); }

// Row indicators of j and of its two neighbours along each axis (a neighbour
// row counts only if that neighbour is j's in-mask neighbour).
struct Rows2 {
  bool r[3], rm[3], rp[3];
  __device__ __forceinline__ Rows2(uint32_t c, const uint32_t (&cn)[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[a] = row2(c, a);
      rm[a] = has_nb(c, 2 * a) && row2(cn[2 * a], a);
      rp[a] = has_nb(c, 2 * a + 1) && row2(cn[2 * a + 1], a);
    }
  }
  __device__ __forceinline__ int diag() const {
    int d = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) d += 4 * (int)r[a] + (int)rm[a] + (int)rp[a];
    return d;
  }
};

// (C^T C f)_j from the values at j, j -+ e (v1[2a], v1[2a+1]) and j -+ 2e (v2).
template <typename T>
__device__ __forceinline__ T ctc2(const Rows2 &R, T fj, const T (&v1)[6], const T (&v2)[6]) {
  T s = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T fm1 = v1[2 * a], fp1 = v1[2 * a + 1], fm2 = v2[2 * a], fp2 = v2[2 * a + 1];
    if (R.r[a]) s += T(-2) * (fm1 - T(2) * fj + fp1);
    if (R.rp[a]) s += fj - T(2) * fp1 + fp2;
    if (R.rm[a]) s += fm2 - T(2) * fm1 + fj;
  }
  return s;
}

// Gradient pass with the second-order regulariser (as k_grad): also loads the
// +-2 neighbours of f and z and the neighbour codes.
template <typename T, int LMAX>
__global__ __launch_bounds__(kNT) void k_grad2(IterArgs<T> a0) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ fin = a.Fp;
  const T *__restrict__ zp = a.Zp;
  T *__restrict__ fo = a.Fc;
  T *__restrict__ gg = a.Gc;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V], cn[V][6];
  T f0[V], z0[V], fn[V][6], zn[V][6], fn2[V][6], zn2[V][6], rho[V][LMAX], tau[V][LMAX];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      f0[v] = fin[jj];
      z0[v] = zp[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        cn[v][k] = a.code[jj + of.o[k]];
        fn[v][k] = fin[jj + of.o[k]];
        zn[v][k] = zp[jj + of.o[k]];
        fn2[v][k] = fin[jj + 2 * of.o[k]];
        zn2[v][k] = zp[jj + 2 * of.o[k]];
      }
      load_echoes<T, LMAX>(a.dat, vw.es, jj, a.L, rho[v], tau[v]);
    }
  };
  int base = vw.bl * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 3>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const T alpha = (T)st.alpha;
  const T beta = (T)a.beta;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (; base < n; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = base + v * kNT + (int)threadIdx.x;
      if (j >= n) continue;
      const uint32_t cv = c[v];
      if (!(cv & NB_SELF)) {
        fo[j] = T(0);
        if (a.fout) a.fout[j] = 0.0;
        if (!a.final_pass) {
          gg[j] = T(0);
          a.D[j] = T(0);
        }
        continue;
      }
      const T fj = f0[v] + alpha * z0[v];
      T v1[6], v2[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        v1[k] = fn[v][k] + alpha * zn[v][k];
        v2[k] = fn2[v][k] + alpha * zn2[v][k];
      }
      const Rows2 R(cv, cn[v]);
      const T lap = ctc2(R, fj, v1, v2);
      T phi, dphi, curv;
      voxel_terms<T, LMAX>(rho[v], tau[v], a.L, a.pairs, fj, phi, dphi, curv);
      const T gj = dphi + beta * lap;
      fo[j] = fj;
      if (a.fout) a.fout[j] = (double)fj;
      if (!a.final_pass) {
        gg[j] = gj;
        a.D[j] = curv;
      }
      acc[0] += (double)phi;
      acc[1] += (double)fj * (double)lap;
      acc[2] += (double)gj * (double)gj;
      acc[3] += (double)z0[v] * (double)gj;
    }
    if (base + stride < n) load(base + stride);
  }
  store_partials<4, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_GRAD, vw.nb, vw.leader);
}

// Diagonal (P = diag H with diag(C^T C) of the second-order operator) or
// identity preconditioner (as k_diag).
template <typename T>
__global__ __launch_bounds__(kNT) void k_diag2(IterArgs<T> a0, const T *__restrict__ gsrc, int identity) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V], cn[V][6];
  T d0[V], g0[V], gp0[V];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      d0[v] = a.D[jj];
      g0[v] = gg[jj];
      gp0[v] = gp[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) cn[v][k] = a.code[jj + of.o[k]];
    }
  };
  int base = vw.bl * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (; base < n; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = base + v * kNT + (int)threadIdx.x;
      if (j >= n) continue;
      const uint32_t cv = c[v];
      if (!(cv & NB_SELF)) {
        a.ipiv[j] = 0.0;
        a.P[j] = T(0);
        continue;
      }
      T pj;
      if (identity) {
        a.ipiv[j] = 1.0;
        pj = g0[v];
      } else {
        const Rows2 R(cv, cn[v]);
        const double h = (double)d0[v] + beta * R.diag();
        double ip = 1.0 / h;
        if (!(h > 0.0)) {
          bad = 1;
          ip = 0.0;
        }
        a.ipiv[j] = ip;
        pj = (T)((double)g0[v] * ip);
      }
      a.P[j] = pj;
      acc[0] += (double)g0[v] * (double)pj;
      acc[1] += (double)gp0[v] * (double)pj;
    }
    if (base + stride < n) load(base + stride);
  }
  if (bad) set_status(a.status, 5);
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DOTS, vw.nb, vw.leader);
}

// Direction and line-search setup with the second-order regulariser (as
// k_dir): z = -p + mu z_prev, and over the rows of C (each row taken at its
// centre voxel) A = sum (Cz)(Cf) = z^T C^T C f and B = sum (Cz)^2; d0 = sum z^2 D.
template <typename T>
__global__ __launch_bounds__(kNT) void k_dir2(IterArgs<T> a0) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ zp = a.Zp;
  T *__restrict__ zo = a.Zc;
  const T *__restrict__ f = a.Fc;
  const T *__restrict__ p = a.P;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V];
  T p0[V], z0[V], f0[V], d0[V], pn[V][6], zn[V][6], fn[V][6];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      p0[v] = p[jj];
      z0[v] = zp[jj];
      f0[v] = f[jj];
      d0[v] = a.D[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        pn[v][k] = p[jj + of.o[k]];
        zn[v][k] = zp[jj + of.o[k]];
        fn[v][k] = f[jj + of.o[k]];
      }
    }
  };
  int base = vw.bl * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const T mu = (T)st.mu;
  double acc[3] = {0.0, 0.0, 0.0};
  for (; base < n; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = base + v * kNT + (int)threadIdx.x;
      if (j >= n) continue;
      const uint32_t cv = c[v];
      if (!(cv & NB_SELF)) {
        zo[j] = T(0);
        continue;
      }
      const T zj = -p0[v] + mu * z0[v];
      zo[j] = zj;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        if (row2(cv, ax)) {
          const T zm = -pn[v][2 * ax] + mu * zn[v][2 * ax], zq = -pn[v][2 * ax + 1] + mu * zn[v][2 * ax + 1];
          const double cz = (double)(zm - T(2) * zj + zq);
          const double cf = (double)(fn[v][2 * ax] - T(2) * f0[v] + fn[v][2 * ax + 1]);
          acc[0] += cz * cf;
          acc[1] += cz * cz;
        }
      acc[2] += (double)zj * (double)zj * (double)d0[v];
    }
    if (base + stride < n) load(base + stride);
  }
  store_partials<3, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DIR, vw.nb, vw.leader);
}

// ---------------------------------------------------------------------------
// IC(0) of H = diag(D) + beta C^T C in three-colour order (colour (x+y+z) mod
// 3, then natural), Sec. III-B eqs. (precon_hess), (precon).  No two voxels
// of a colour are coupled, and along an axis line through a voxel of colour c
// the voxels at -1, +2 have colour c-1 and those at +1, -2 colour c+1.  So:
//   colour 0: pivot H_jj, y_j = g_j;
//   colour 1: earlier neighbours j-e, j+2e (colour 0), no fill terms;
//   colour 2: earlier neighbours j+e, j-2e (colour 0) and j-e, j+2e
//     (colour 1); the colour-1 entries carry the fill terms of incomplete
//     L D L^T through their common colour-0 neighbours:
//       L(j,j-e)  D(j-e)  = H(j,j-e)  - H(j,j-2e) H(j-e,j-2e)/D(j-2e)
//                                     - H(j,j+e)  H(j-e,j+e)/D(j+e),
//       L(j,j+2e) D(j+2e) = H(j,j+2e) - H(j,j+e)  H(j+2e,j+e)/D(j+e).
// Forward L y = g over colours 0, 1, 2 and backward L^T p = D^{-1} y over
// colours 2, 1, 0 take four passes; g^T p = sum y^2/D and g_prev^T p =
// sum y' y / D with y' = L^{-1} g_prev come out of the forward passes.
// Off-diagonal entries along axis a (rows r at the centre voxel):
//   H(j,j+-e) = beta (-2 r_j - 2 r_{j+-e}),  H(j,j+-2e) = beta r_{j+-e}.

__device__ __forceinline__ int colour3(const Geo &g, int j) {
  const int z = j % g.nz, yx = j / g.nz, y = yx % g.ny, x = yx / g.ny;
  return (x + y + z) % 3;
}

// In-mask flags and row indicators on the axis line through voxel j (in the
// mask, code c): voxels j-e, j+e, j-2e, j+2e (the last two only reached
// through an in-mask middle voxel: a +-2 neighbour behind a hole couples to
// j through nothing) and the entries of H/beta among them.
struct Line2 {
  bool m1, p1, m2, p2;   // j-e, j+e, j-2e, j+2e in the mask
  double hm1, hp1;       // H(j,j-e), H(j,j+e)
  double hm2, hp2;       // H(j,j-2e), H(j,j+2e)
  double hm1m2, hp1p2;   // H(j-e,j-2e), H(j+e,j+2e)
  double hm1p1;          // H(j-e,j+e)
  __device__ __forceinline__ Line2(const uint8_t *__restrict__ code, uint32_t c, int j, int a, int o, double beta) {
    m1 = has_nb(c, 2 * a);
    p1 = has_nb(c, 2 * a + 1);
    const uint32_t cm1 = m1 ? code[j - o] : 0u, cp1 = p1 ? code[j + o] : 0u;
    m2 = has_nb(cm1, 2 * a);
    p2 = has_nb(cp1, 2 * a + 1);
    const uint32_t cm2 = m2 ? code[j - 2 * o] : 0u, cp2 = p2 ? code[j + 2 * o] : 0u;
    const double r0 = row2(c, a) ? 1.0 : 0.0, rm1 = row2(cm1, a) ? 1.0 : 0.0, rp1 = row2(cp1, a) ? 1.0 : 0.0;
    const double rm2 = row2(cm2, a) ? 1.0 : 0.0, rp2 = row2(cp2, a) ? 1.0 : 0.0;
    hm1 = beta * (-2.0 * r0 - 2.0 * rm1);
    hp1 = beta * (-2.0 * r0 - 2.0 * rp1);
    hm2 = beta * rm1;
    hp2 = beta * rp1;
    hm1m2 = beta * (-2.0 * rm1 - 2.0 * rm2);
    hp1p2 = beta * (-2.0 * rp1 - 2.0 * rp2);
    hm1p1 = beta * r0;
  }
};

// diag(C^T C) per voxel (0 outside the mask), once per setup.
__global__ __launch_bounds__(kBlock) void k_rdiag2(Geo g, const uint8_t *__restrict__ code, uint8_t *rdiag) {
  const Offs of(g);
  for (int j = (int)blockIdx.x * kBlock + (int)threadIdx.x; j < (int)g.n; j += (int)gridDim.x * kBlock) {
    const uint32_t c = code[j];
    uint32_t cn[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) cn[k] = has_nb(c, k) ? code[j + of.o[k]] : 0u;
    rdiag[j] = (c & NB_SELF) ? (uint8_t)Rows2(c, cn).diag() : (uint8_t)0;
  }
}

// Forward pass over colours 0 and 1: pivots (stored inverted), y and y' of
// colour 1, and their terms of the two dot products.  gsrc: standalone call.
template <typename T>
__global__ __launch_bounds__(kNT) void k_ic3_fwd1(IterArgs<T> a0, const T *__restrict__ gsrc) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const Offs of(g);
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (int j = vw.bl * kNT + (int)threadIdx.x; j < (int)g.n; j += vw.nb * kNT) {
    const int col = colour3(g, j);
    if (col == 2) continue;
    const uint32_t c = a.code[j];
    if (!(c & NB_SELF)) {
      a.ipiv[j] = 0.0;
      if (col == 1) {
        a0.X[j] = T(0);
        a0.X2[j] = T(0);
      }
      continue;
    }
    double d = (double)a.D[j] + beta * (double)a0.rdiag[j];
    double y = (double)gg[j], y2 = (double)gp[j];
    if (col == 1) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int o = of.o[2 * ax + 1];
        const Line2 l(a.code, c, j, ax, o, beta);
        if (l.m1 && l.hm1 != 0.0) {
          const int k = j - o;
          const double lk = l.hm1 / ((double)a.D[k] + beta * (double)a0.rdiag[k]);
          d -= l.hm1 * lk;
          y -= lk * (double)gg[k];
          y2 -= lk * (double)gp[k];
        }
        if (l.p2 && l.hp2 != 0.0) {
          const int k = j + 2 * o;
          const double lk = l.hp2 / ((double)a.D[k] + beta * (double)a0.rdiag[k]);
          d -= l.hp2 * lk;
          y -= lk * (double)gg[k];
          y2 -= lk * (double)gp[k];
        }
      }
    }
    double ip = 1.0 / d;
    if (!(d > 0.0)) {
      bad = 1;
      ip = 0.0;
    }
    a.ipiv[j] = ip;
    if (col == 1) {
      a0.X[j] = (T)y;
      a0.X2[j] = (T)y2;
    }
    acc[0] += y * y * ip;
    acc[1] += y2 * y * ip;
  }
  if (bad) set_status(a.status, 5);
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DOTS_A, vw.nb, vw.leader);
}

// Forward pass over colour 2 with the fill terms, its pivots, and the first
// backward step p = y / D; the rest of the dot products.
template <typename T>
__global__ __launch_bounds__(kNT) void k_ic3_fwd2(IterArgs<T> a0, const T *__restrict__ gsrc) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const Offs of(g);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (int j = vw.bl * kNT + (int)threadIdx.x; j < (int)g.n; j += vw.nb * kNT) {
    if (colour3(g, j) != 2) continue;
    const uint32_t c = a.code[j];
    if (!(c & NB_SELF)) {
      a.ipiv[j] = 0.0;
      a.P[j] = T(0);
      continue;
    }
    double d = (double)a.D[j] + beta * (double)a0.rdiag[j];
    double y = (double)gg[j], y2 = (double)gp[j];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int o = of.o[2 * ax + 1];
      const Line2 l(a.code, c, j, ax, o, beta);
      const double ipm1 = l.m1 ? a.ipiv[j - o] : 0.0, ipp1 = l.p1 ? a.ipiv[j + o] : 0.0;
      const double ipm2 = l.m2 ? a.ipiv[j - 2 * o] : 0.0, ipp2 = l.p2 ? a.ipiv[j + 2 * o] : 0.0;
      // colour 0: j+e and j-2e; colour 1: j-e and j+2e (entries times the pivot of the neighbour)
      const double np1 = l.hp1, nm2 = l.hm2;
      const double nm1 = l.hm1 - l.hm2 * l.hm1m2 * ipm2 - l.hp1 * l.hm1p1 * ipp1;
      const double np2 = l.hp2 - l.hp1 * l.hp1p2 * ipp1;
      const double lp1 = np1 * ipp1, lm2 = nm2 * ipm2, lm1 = nm1 * ipm1, lp2 = np2 * ipp2;
      d -= np1 * lp1 + nm2 * lm2 + nm1 * lm1 + np2 * lp2;
      if (l.p1) {
        y -= lp1 * (double)gg[j + o];
        y2 -= lp1 * (double)gp[j + o];
      }
      if (l.m2) {
        y -= lm2 * (double)gg[j - 2 * o];
        y2 -= lm2 * (double)gp[j - 2 * o];
      }
      if (l.m1) {
        y -= lm1 * (double)a0.X[j - o];
        y2 -= lm1 * (double)a0.X2[j - o];
      }
      if (l.p2) {
        y -= lp2 * (double)a0.X[j + 2 * o];
        y2 -= lp2 * (double)a0.X2[j + 2 * o];
      }
    }
    double ip = 1.0 / d;
    if (!(d > 0.0)) {
      bad = 1;
      ip = 0.0;
    }
    a.ipiv[j] = ip;
    a.P[j] = (T)(y * ip);
    acc[0] += y * y * ip;
    acc[1] += y2 * y * ip;
  }
  if (bad) set_status(a.status, 5);
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DOTS, vw.nb, vw.leader);
}

// Backward pass over colour 1: p_j = y_j / D_j - L(j+e,j) p_{j+e} - L(j-2e,j) p_{j-2e}
// (the colour-2 neighbours' entries, fill terms included, recomputed).
template <typename T>
__global__ __launch_bounds__(kNT) void k_ic3_bwd1(IterArgs<T> a0) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const Offs of(g);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  for (int j = vw.bl * kNT + (int)threadIdx.x; j < (int)g.n; j += vw.nb * kNT) {
    if (colour3(g, j) != 1) continue;
    const uint32_t c = a.code[j];
    if (!(c & NB_SELF)) {
      a.P[j] = T(0);
      continue;
    }
    const double ip = a.ipiv[j];
    double s = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int o = of.o[2 * ax + 1];
      const Line2 l(a.code, c, j, ax, o, beta);
      const double ipm1 = l.m1 ? a.ipiv[j - o] : 0.0, ipp2 = l.p2 ? a.ipiv[j + 2 * o] : 0.0;
      if (l.p1) {  // i = j+e: L(i,j) D_j = H(i,j) - H(i,j-e) H(j,j-e)/D(j-e) - H(i,j+2e) H(j,j+2e)/D(j+2e)
        const double n = l.hp1 - l.hm1p1 * l.hm1 * ipm1 - l.hp1p2 * l.hp2 * ipp2;
        s += n * (double)a.P[j + o];
      }
      if (l.m2) {  // i = j-2e: L(i,j) D_j = H(i,j) - H(i,j-e) H(j-e,j)/D(j-e)
        const double n = l.hm2 - l.hm1m2 * l.hm1 * ipm1;
        s += n * (double)a.P[j - 2 * o];
      }
    }
    a.P[j] = (T)(((double)a0.X[j] - s) * ip);
  }
  put_state(st, a.sout, PK_NONE, 0, vw.leader);
}

// Backward pass over colour 0: p_j = (g_j - sum_i H(j,i) p_i) / D_j over the
// stencil neighbours (colours 1 and 2).
template <typename T>
__global__ __launch_bounds__(kNT) void k_ic3_bwd0(IterArgs<T> a0, const T *__restrict__ gsrc) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const Offs of(g);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  for (int j = vw.bl * kNT + (int)threadIdx.x; j < (int)g.n; j += vw.nb * kNT) {
    if (colour3(g, j) != 0) continue;
    const uint32_t c = a.code[j];
    if (!(c & NB_SELF)) {
      a.P[j] = T(0);
      continue;
    }
    double s = (double)gg[j];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int o = of.o[2 * ax + 1];
      const Line2 l(a.code, c, j, ax, o, beta);
      if (l.m1) s -= l.hm1 * (double)a.P[j - o];
      if (l.p1) s -= l.hp1 * (double)a.P[j + o];
      if (l.m2) s -= l.hm2 * (double)a.P[j - 2 * o];
      if (l.p2) s -= l.hp2 * (double)a.P[j + 2 * o];
    }
    a.P[j] = (T)(s * a.ipiv[j]);
  }
  put_state(st, a.sout, PK_NONE, 0, vw.leader);
}

}  // namespace fm
