// Implicit adjoint of the converged field map.
//
// At a stationary point fhat of the cost of Sec. II eq. (cost), grad Psi = 0,
// so a loss L(fhat) has dL/dtheta = -v^T d(grad Psi)/dtheta with H v = dL/df,
// H = diag(h) + beta C^T C the exact Hessian, h_j = sum_{m<n} w_mn (2 pi dt)^2
// cos(x_mn) (the curvature the Huber bound of Sec. III-B eq. (ls_huber)
// replaces).  H v = dL/df is solved by conjugate gradients preconditioned with
// the IC(0) factor of the Huber model D + beta C^T C (Sec. III-B eq.
// (precon)), reusing the iteration's preconditioner passes.  One CG iteration
// is: preconditioner passes (z = M^{-1} r, leaving r^T z), direction pass
// (d = z + (rho / rho_prev) d_prev, partial d^T H d) and update pass
// (v += alpha d, r -= alpha H d, partial ||r||^2).  The direction buffer
// ping-pongs with the CG iteration parity because the Hessian stencil reads
// the previous direction at neighbours.
//
// The gradients then follow from v:
//   dL/dbeta   = -v^T C^T C fhat,
//   dL/dzhat_l = -v_j d g_j / d zhat_l, with g_j = sum_{m<n} 2 (2 pi dt_mn)
//                Im(Gamma_mn conj(zhat_m) zhat_n e^{i 2 pi dt_mn f_j}),
//   dL/dy_cl   = (s_c / sqrt(sum_c |s_c|^2)) dL/dzhat_l  (zhat is linear in y),
// complex gradients in the d/dRe + i d/dIm convention.
//
// With the second-order regulariser (R2) C^T C is the 13-point operator of
// fm_order2.hpp in the Hessian products and in dL/dbeta, and CG is
// preconditioned by diag(H) (the Huber curvature plus beta diag(C^T C)) or
// not at all: the solution v does not depend on the preconditioner, only the
// iteration count does.
#pragma once

#include "fm_stream.hpp"
#include "fm_order2.hpp"

namespace fm {

template <typename T>
struct AdjArgs {
  Geo geo;
  int32_t L;
  double beta;
  const T2<T> *dat;
  const uint8_t *code;
  const PairC<T> *pairs;
  const T *F;      // fhat
  T *R;            // residual (padded: the preconditioner reads neighbours)
  const T *Zp;     // preconditioned residual (padded)
  T *Dd[2];        // CG directions (padded), slot par written this iteration
  T *V;            // solution v
  T *H;            // exact Hessian diagonal h_j (without beta deg)
  T *Dc;           // Huber curvature (the preconditioner's D)
  double *hinv;    // 1 / (D + beta deg) for the red-black preconditioner
  int32_t par;     // CG iteration parity
  int32_t nparts_in;
  int32_t nvals_in;
  const State *sin;
  State *sout;
  const double *pin;
  double *pout;
  int32_t *status;
};

// Data-term curvatures at f: the Huber bound (as in the iteration) and the
// exact second derivative, with the same turn-based wrap as voxel_terms:
// cos(2 pi xi) = 1 - 2 s^2.
template <typename T, int LMAX>
__device__ __forceinline__ void voxel_curvatures(const T (&rho)[LMAX], const T (&tau)[LMAX], int L,
                                                 const PairC<T> *__restrict__ pc, T f, T &curv, T &hess) {
  T c2 = 0, h2 = 0;
  int q = 0;
#pragma unroll
  for (int m = 0; m < LMAX; ++m) {
#pragma unroll
    for (int n = m + 1; n < LMAX; ++n) {
      if (n < L) {
        const PairC<T> P = pc[q];
        const T w = P.w * rho[m] * rho[n];
        const T xi = P.g + (tau[n] - tau[m]) + f * P.dt;
        const T x = T(3.14159265358979323846) * (xi - rint_t(xi));
        T sx, c;
        sinx_cos(x, sx, c);
        const T s = x * sx;
        const T wdd = w * P.d2pi * P.d2pi;
        c2 += wdd * (sx * c);
        h2 += wdd * (T(1) - T(2) * s * s);
        ++q;
      }
    }
  }
  curv = c2;
  hess = h2;
}

// Set-up at fhat: curvatures, r = dL/df, v = 0, d_prev = 0; partial ||r||^2.
template <typename T, int LMAX>
__global__ __launch_bounds__(kNT) void k_adj_setup(AdjArgs<T> a, const double *__restrict__ dldf, double rtol2,
                                                   int write_hinv) {
  const Geo g = a.geo;
  const int n = (int)g.n;
  double acc[1] = {0.0};
  for (int j = (int)blockIdx.x * kNT + (int)threadIdx.x; j < n; j += (int)gridDim.x * kNT) {
    const uint32_t c = a.code[j];
    T r = T(0), curv = T(0), hess = T(0);
    double hv = 0.0;
    if (c & NB_SELF) {
      T rho[LMAX], tau[LMAX];
      load_echoes<T, LMAX>(a.dat, (int64_t)n, j, a.L, rho, tau);
      voxel_curvatures<T, LMAX>(rho, tau, a.L, a.pairs, a.F[j], curv, hess);
      r = (T)dldf[j];
      const double h = (double)curv + a.beta * nb_deg(c);
      hv = h > 0.0 ? 1.0 / h : 0.0;
      acc[0] += (double)r * (double)r;
    }
    a.R[j] = r;
    a.Dc[j] = curv;
    a.H[j] = hess;
    a.V[j] = T(0);
    a.Dd[1][j] = T(0);
    if (write_hinv) a.hinv[j] = hv;
  }
  store_partials<1, kNT>(acc, a.pout);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State s{};
    s.kind = PK_ADJ_INIT;
    s.nparts = (int32_t)gridDim.x;
    s.trace_cap = -1;
    s.cg_rtol2 = rtol2;
    *a.sout = s;
  }
}

// Direction d = z + (rho / rho_prev) d_prev and the partial d^T H d.
template <typename T, bool R2>
__global__ __launch_bounds__(kNT) void k_adj_dir(AdjArgs<T> a) {
  constexpr int V = R2 ? 1 : Vpt<T>::v, K2 = R2 ? 6 : 1;
  const Geo g = a.geo;
  const T *__restrict__ dp = a.Dd[(a.par + 1) & 1];
  T *__restrict__ dn = a.Dd[a.par & 1];
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = (int)gridDim.x * chunk;
  uint32_t c[V], cn[V][K2];
  T z0[V], d0[V], h0[V], zn[V][6], dnb[V][6], zn2[V][K2], dnb2[V][K2];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      z0[v] = a.Zp[jj];
      d0[v] = dp[jj];
      h0[v] = a.H[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        zn[v][k] = a.Zp[jj + of.o[k]];
        dnb[v][k] = dp[jj + of.o[k]];
      }
      if constexpr (R2) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          cn[v][k] = a.code[jj + of.o[k]];
          zn2[v][k] = a.Zp[jj + 2 * of.o[k]];
          dnb2[v][k] = dp[jj + 2 * of.o[k]];
        }
      }
    }
  };
  int base = (int)blockIdx.x * chunk;
  if (base < n) load(base);
  State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, nullptr, a.status);
  double acc[1] = {0.0};
  if (!st.cg_done) {
    const double rho = st.gtp;  // r^T M^{-1} r from the preconditioner passes
    const T bcg = (T)((st.cg_it > 0 && st.cg_rho_prev != 0.0) ? rho / st.cg_rho_prev : 0.0);
    const T beta = (T)a.beta;
    st.cg_rho = rho;
    for (; base < n; base += stride) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int j = base + v * kNT + (int)threadIdx.x;
        if (j >= n) continue;
        const uint32_t cv = c[v];
        if (!(cv & NB_SELF)) {
          dn[j] = T(0);
          continue;
        }
        const T dj = z0[v] + bcg * d0[v];
        T lap = T(0);
        if constexpr (R2) {
          T v1[6], v2[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            v1[k] = zn[v][k] + bcg * dnb[v][k];
            v2[k] = zn2[v][k] + bcg * dnb2[v][k];
          }
          lap = ctc2(Rows2(cv, cn[v]), dj, v1, v2);
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k)
            if (has_nb(cv, k)) lap += dj - (zn[v][k] + bcg * dnb[v][k]);
        }
        dn[j] = dj;
        const T qj = h0[v] * dj + beta * lap;
        acc[0] += (double)dj * (double)qj;
      }
      if (base + stride < n) load(base + stride);
    }
  }
  store_partials<1, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_ADJ_CURV, gridDim.x);
}

// v += alpha d, r -= alpha H d; partial ||r||^2.
template <typename T, bool R2>
__global__ __launch_bounds__(kNT) void k_adj_update(AdjArgs<T> a) {
  constexpr int V = R2 ? 1 : Vpt<T>::v, K2 = R2 ? 6 : 1;
  const Geo g = a.geo;
  const T *__restrict__ d = a.Dd[a.par & 1];
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = (int)gridDim.x * chunk;
  uint32_t c[V], cn[V][K2];
  T d0[V], h0[V], v0[V], r0[V], dnb[V][6], dnb2[V][K2];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      d0[v] = d[jj];
      h0[v] = a.H[jj];
      v0[v] = a.V[jj];
      r0[v] = a.R[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) dnb[v][k] = d[jj + of.o[k]];
      if constexpr (R2) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          cn[v][k] = a.code[jj + of.o[k]];
          dnb2[v][k] = d[jj + 2 * of.o[k]];
        }
      }
    }
  };
  int base = (int)blockIdx.x * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 1>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, nullptr, a.status);
  double acc[1] = {0.0};
  if (!st.cg_done) {
    const T alpha = (T)st.cg_alpha;
    const T beta = (T)a.beta;
    for (; base < n; base += stride) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int j = base + v * kNT + (int)threadIdx.x;
        if (j >= n) continue;
        const uint32_t cv = c[v];
        if (!(cv & NB_SELF)) continue;
        const T dj = d0[v];
        T lap = T(0);
        if constexpr (R2) {
          lap = ctc2(Rows2(cv, cn[v]), dj, dnb[v], dnb2[v]);
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k)
            if (has_nb(cv, k)) lap += dj - dnb[v][k];
        }
        const T qj = h0[v] * dj + beta * lap;
        const T rj = r0[v] - alpha * qj;
        a.V[j] = v0[v] + alpha * dj;
        a.R[j] = rj;
        acc[0] += (double)rj * (double)rj;
      }
      if (base + stride < n) load(base + stride);
    }
  }
  store_partials<1, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_ADJ_UPD, gridDim.x);
}

// Gradients from v: dL/dy (complex64, layout of y), v as float64, and the
// partial v^T C^T C fhat for dL/dbeta.
template <typename T, int LMAX, bool R2>
__global__ __launch_bounds__(kNT) void k_adj_out(AdjArgs<T> a, const float2 *__restrict__ sens, int ncoil,
                                                 float2 *__restrict__ dldy, double *__restrict__ vout) {
  const Geo g = a.geo;
  const int n = (int)g.n;
  const T kPi = T(3.14159265358979323846);
  double acc[1] = {0.0};
  for (int j = (int)blockIdx.x * kNT + (int)threadIdx.x; j < n; j += (int)gridDim.x * kNT) {
    const uint32_t c = a.code[j];
    const T vj = (c & NB_SELF) ? a.V[j] : T(0);
    if (vout) vout[j] = (double)vj;
    // zhat-gradients in the frame of each echo's own phase: dL/dzhat_l = a_l e^{i theta_l}
    T are[LMAX], aim[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) are[l] = aim[l] = T(0);
    T rho[LMAX], tau[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) rho[l] = tau[l] = T(0);
    if (c & NB_SELF) {
      const T fj = a.F[j];
      T lap = T(0);
      const int o[6] = {-(int)g.sx, (int)g.sx, -(int)g.sy, (int)g.sy, -1, 1};
      if constexpr (R2) {
        uint32_t cn[6];
        T v1[6], v2[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          cn[k] = a.code[j + o[k]];
          v1[k] = a.F[j + o[k]];
          v2[k] = a.F[j + 2 * o[k]];
        }
        lap = ctc2(Rows2(c, cn), fj, v1, v2);
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(c, k)) lap += fj - a.F[j + o[k]];
      }
      acc[0] += (double)vj * (double)lap;
      load_echoes<T, LMAX>(a.dat, (int64_t)n, j, a.L, rho, tau);
      int q = 0;
#pragma unroll
      for (int m = 0; m < LMAX; ++m) {
#pragma unroll
        for (int nn = m + 1; nn < LMAX; ++nn) {
          if (nn < a.L) {
            const PairC<T> P = a.pairs[q];
            const T xi = P.g + (tau[nn] - tau[m]) + fj * P.dt;
            const T x = kPi * (xi - rint_t(xi));
            T sx, cc;
            sinx_cos(x, sx, cc);
            const T s = x * sx;
            const T S2 = T(2) * s * cc;          // sin(2 pi xi)
            const T C2 = T(1) - T(2) * s * s;    // cos(2 pi xi)
            const T coef = -vj * P.d2pi * P.w;
            // d/dzhat_n: coef rho_m (sin + i cos); d/dzhat_m: coef rho_n (sin - i cos)
            are[nn] += coef * rho[m] * S2;
            aim[nn] += coef * rho[m] * C2;
            are[m] += coef * rho[nn] * S2;
            aim[m] -= coef * rho[nn] * C2;
            ++q;
          }
        }
      }
    }
    // rotate by e^{i theta_l}, theta_l = 2 pi tau_l
    T gre[LMAX], gim[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
      const T x = kPi * (tau[l] - rint_t(tau[l]));
      T sx, cc;
      sinx_cos(x, sx, cc);
      const T s = x * sx;
      const T sn = T(2) * s * cc, cs = T(1) - T(2) * s * s;
      gre[l] = are[l] * cs - aim[l] * sn;
      gim[l] = are[l] * sn + aim[l] * cs;
    }
    if (dldy) {
      double ss = 1.0;
      if (sens) {
        ss = 0.0;
        for (int cc = 0; cc < ncoil; ++cc) {
          const float2 sv = sens[(int64_t)cc * n + j];
          ss += (double)sv.x * sv.x + (double)sv.y * sv.y;
        }
      }
      const double scale = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
      for (int cc = 0; cc < ncoil; ++cc) {
        double sr = scale, si = 0.0;
        if (sens) {
          const float2 sv = sens[(int64_t)cc * n + j];
          sr = sv.x * scale;
          si = sv.y * scale;
        }
        for (int l = 0; l < a.L; ++l) {
          T xr = T(0), xim = T(0);
#pragma unroll
          for (int k = 0; k < LMAX; ++k)
            if (k == l) {
              xr = gre[k];
              xim = gim[k];
            }
          float2 o;
          o.x = (float)(sr * (double)xr - si * (double)xim);
          o.y = (float)(sr * (double)xim + si * (double)xr);
          dldy[((int64_t)cc * a.L + l) * n + j] = o;
        }
      }
    }
  }
  store_partials<1, kNT>(acc, a.pout);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State s = *a.sin;
    s.kind = PK_ADJ_FIN;
    s.nparts = (int32_t)gridDim.x;
    *a.sout = s;
  }
}

}  // namespace fm
