// Streaming passes of one NCG iteration (gradient, red-black / diagonal
// preconditioner, direction, line search).
//
// Launch shape: blocks of kNT threads, each thread owning V voxels of a chunk
// of kNT*V consecutive voxels (V = 2).  Every load of a
// chunk is issued before any use: neighbour slots are addressed whenever the
// index lies inside the volume and masked afterwards with the voxel's
// neighbour code, so no load waits on another.  The first chunk is loaded
// before the incoming partial sums are reduced, overlapping the two latencies.
#pragma once

#include "fm_kernels.hpp"

namespace fm {

#ifndef FM_VPT32
#define FM_VPT32 2
#endif
#ifndef FM_VPT64
#define FM_VPT64 2
#endif

#ifndef FM_NT
#define FM_NT 256
#endif
constexpr int kNT = FM_NT;  // threads per block of the streaming passes

template <typename T>
struct Vpt {
  static constexpr int v = sizeof(T) == 4 ? FM_VPT32 : FM_VPT64;
};

// Per-kernel overrides of the voxels per thread (FP32 working type).
#ifndef FM_V_GRAD
#define FM_V_GRAD FM_VPT32
#endif
// The line-search pass, with no neighbour loads, keeps more voxels in flight
// per thread (up to 4 echoes; at 8.4 M voxels 70 -> 63 us, unchanged at 1 M).
#ifndef FM_V_MLS
#define FM_V_MLS 4
#endif
template <typename T, int V32>
struct Vk {
  static constexpr int v = sizeof(T) == 4 ? V32 : FM_VPT64;
};

// Every array read at neighbour offsets is padded by one x-plane (sx
// elements) on both sides, so j + off is always a valid address; the code
// bits decide whether the value is a neighbour.  Indices are 32-bit (the
// plan checks n + 2 sx < 2^31).
struct Offs {
  int o[6];
  __device__ __forceinline__ explicit Offs(const Geo &g) {
    o[0] = -(int)g.sx;
    o[1] = (int)g.sx;
    o[2] = -(int)g.sy;
    o[3] = (int)g.sy;
    o[4] = -1;
    o[5] = 1;
  }
};

__device__ __forceinline__ bool has_nb(uint32_t c, int k) { return (c >> (k + 1)) & 1u; }

// Arguments as seen by one workgroup, with the ping-pong slots of the launch's
// iteration parity resolved (c = current, p = previous; no array members, so
// nothing is indexed at run time and everything stays in registers).  For a
// batched launch every per-voxel pointer is moved to the workgroup's volume,
// and the scalar state, incoming partial sums, trace, beta and geometry are
// that volume's.
template <typename T>
struct VArgs {
  Geo geo;
  int32_t L;
  double beta;
  const T2<T> *dat;
  const uint8_t *code;
  const PairC<T> *pairs;
  T *Fc, *Fp, *Zc, *Zp, *Gc, *Gp;
  T *D, *P;
  double *ipiv, *hinv;
  int32_t write_hinv, store_piv, nparts_in, nvals_in, final_pass;
  const State *sin;
  State *sout;
  const double *pin;
  double *pout;
  int32_t *status;
  double *trace;
  double *fout;
};

template <bool BATCH, typename T>
__device__ __forceinline__ VArgs<T> at_volume(const IterArgs<T> &a0, const VolView &vw) {
  VArgs<T> a;
  const int o = BATCH ? vw.off : 0;
  const bool odd = (a0.par & 1) != 0;
  a.geo = vw.g;
  a.L = a0.L;
  a.beta = vw.beta;
  a.dat = a0.dat + o;
  a.code = a0.code + o;
  a.pairs = a0.pairs;
  a.Fc = (odd ? a0.F[1] : a0.F[0]) + o;
  a.Fp = (odd ? a0.F[0] : a0.F[1]) + o;
  a.Zc = (odd ? a0.Z[1] : a0.Z[0]) + o;
  a.Zp = (odd ? a0.Z[0] : a0.Z[1]) + o;
  a.Gc = (odd ? a0.G[1] : a0.G[0]) + o;
  a.Gp = (odd ? a0.G[0] : a0.G[1]) + o;
  a.D = a0.D + o;
  a.P = a0.P + o;
  a.ipiv = a0.ipiv + o;
  a.hinv = a0.hinv + o;
  a.write_hinv = a0.write_hinv;
  a.store_piv = a0.store_piv;
  a.nparts_in = vw.pcount;
  a.nvals_in = a0.nvals_in;
  a.final_pass = a0.final_pass;
  a.sin = a0.sin + vw.vol;
  a.sout = a0.sout + vw.vol;
  a.pin = a0.pin + vw.pfirst;
  a.pout = a0.pout;
  a.status = a0.status;
  a.trace = a0.trace + (BATCH ? (size_t)vw.vol * a0.bt.trace_stride : 0);
  a.fout = BATCH ? (a0.bt.fouts ? a0.bt.fouts[vw.vol] : nullptr) : a0.fout;
  return a;
}

// ---------------------------------------------------------------------------
// Gradient pass of iteration i (Sec. III eq. (ls_grad)), fused with the update
// f^i = f^{i-1} + alpha z^{i-1} of the previous iteration:
//   g_j = dphi_j(f_j) + beta (C^T C f)_j,  D_j = Huber curvature (eq. (ls_huber)),
// hinv_j = 1 / (D_j + beta deg_j) for the red-black preconditioner.
// Partial sums: sum phi, f^T C^T C f, ||g||^2, z_prev^T g.
template <typename T, int LMAX, bool BATCH>
__global__ __launch_bounds__(kNT) void k_grad(IterArgs<T> a0) {
  constexpr int V = Vk<T, FM_V_GRAD>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ fin = a.Fp;
  const T *__restrict__ zp = a.Zp;
  T *__restrict__ fo = a.Fc;
  T *__restrict__ gg = a.Gc;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V];
  T f0[V], z0[V], fn[V][6], zn[V][6], rho[V][LMAX], tau[V][LMAX];
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
        fn[v][k] = fin[jj + of.o[k]];
        zn[v][k] = zp[jj + of.o[k]];
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
          if (a.write_hinv == 1) a.hinv[j] = 0.0;
        }
        continue;
      }
      const T fj = f0[v] + alpha * z0[v];
      T lap = T(0);
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) lap += fj - (fn[v][k] + alpha * zn[v][k]);
      T phi, dphi, curv;
      voxel_terms<T, LMAX>(rho[v], tau[v], a.L, a.pairs, fj, phi, dphi, curv);
      const T gj = dphi + beta * lap;
      fo[j] = fj;
      if (a.fout) a.fout[j] = (double)fj;
      if (!a.final_pass) {
        gg[j] = gj;
        a.D[j] = curv;
        if (a.write_hinv == 1 || (a.write_hinv == 2 && !(cv & NB_BLACK))) {
          const double h = (double)curv + a.beta * nb_deg(cv);
          a.hinv[a.write_hinv == 2 ? j >> 1 : j] = h > 0.0 ? 1.0 / h : 0.0;
        }
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

// ---------------------------------------------------------------------------
// IC(0) in red-black order (Sec. III-B eq. (precon) with the red voxels,
// x+y+z even, eliminated first).  Red voxels have no earlier neighbour, so
// their pivot is h_r = D_r + beta deg_r and x_r = g_r / h_r; black voxels come
// last with every neighbour earlier:
//   P_b = h_b - beta^2 sum_k 1/h_k,   x_b = (g_b + beta sum_k g_k / h_k) / P_b,
// and p_b = x_b (no later neighbour); then p_r = x_r + (beta / h_r) sum_k p_k.
// 1/h is read from hinv (written once per voxel by the gradient pass).
//
// Partial sums.  With DOTS = false (standalone preconditioner): g^T p and
// g_prev^T p over the black voxels, the red pass adds the rest.  With
// DOTS = true (the iteration): both dot products in full, from the factored
// form M = L Lam L^T of the preconditioner, u^T M^{-1} g = (L^{-1} u)^T
// Lam^{-1} (L^{-1} g).  L^{-1} g is g on red voxels and
// y_b = g_b + beta sum_k g_k / h_k on black ones, with Lam = h_r, P_b, so
//   g^T p      = sum_r g_r^2 / h_r       + sum_b y_b  y_b / P_b,
//   g_prev^T p = sum_r g'_r g_r / h_r    + sum_b y'_b y_b / P_b,
// and the direction can be formed in the red pass (k_rb_red_dir).
template <typename T, bool BATCH, bool DOTS = false>
__global__ __launch_bounds__(kNT) void k_rb_black(IterArgs<T> a0, const T *__restrict__ gsrc) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc + vw.off : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const double *__restrict__ hv = a.hinv;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  constexpr int NGP = DOTS ? 6 : 1;
  uint32_t c[V];
  T d0[V], g0[V], gp0[V], gn[V][6], gpn[V][NGP];
  double hn[V][6], h0[V];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      d0[v] = a.D[jj];
      g0[v] = gg[jj];
      gp0[v] = gp[jj];
      if (DOTS) h0[v] = hv[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        gn[v][k] = gg[jj + of.o[k]];
        hn[v][k] = hv[jj + of.o[k]];
        if (DOTS) gpn[v][k < NGP ? k : 0] = gp[jj + of.o[k]];
      }
    }
  };
  int base = vw.bl * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta, b2 = a.beta * a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (; base < n; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = base + v * kNT + (int)threadIdx.x;
      if (j >= n) continue;
      const uint32_t cv = c[v];
      if (!(cv & NB_SELF)) {
        if (a.store_piv) a.ipiv[j] = 0.0;
        a.P[j] = T(0);
        continue;
      }
      if (!(cv & NB_BLACK)) {
        if (DOTS) {
          const double gh = (double)g0[v] * h0[v];
          acc[0] += (double)g0[v] * gh;
          acc[1] += (double)gp0[v] * gh;
        }
        continue;
      }
      const double h = (double)d0[v] + beta * nb_deg(cv);
      double sp = 0.0, sxv = 0.0, syp = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) {
          sp += hn[v][k];
          sxv += (double)gn[v][k] * hn[v][k];
          if (DOTS) syp += (double)gpn[v][k < NGP ? k : 0] * hn[v][k];
        }
      const double piv = h - b2 * sp;
      double ip = 1.0 / piv;
      if (!(piv > 0.0)) {
        bad = 1;
        ip = 0.0;
      }
      if (a.store_piv) a.ipiv[j] = ip;
      const double yb = (double)g0[v] + beta * sxv;
      const T pj = (T)(yb * ip);
      a.P[j] = pj;
      if (DOTS) {
        const double x = yb * ip;
        acc[0] += yb * x;
        acc[1] += ((double)gp0[v] + beta * syp) * x;
      } else {
        acc[0] += (double)g0[v] * (double)pj;
        acc[1] += (double)gp0[v] * (double)pj;
      }
    }
    if (base + stride < n) load(base + stride);
  }
  if (bad) set_status(a.status, 5);
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, DOTS ? PK_DOTS : PK_DOTS_A, vw.nb, vw.leader);
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_rb_red(IterArgs<T> a0, const T *__restrict__ gsrc) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc + vw.off : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V];
  T g0[V], gp0[V], pn[V][6];
  double h0[V];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      g0[v] = gg[jj];
      gp0[v] = gp[jj];
      h0[v] = a.hinv[jj];
#pragma unroll
      for (int k = 0; k < 6; ++k) pn[v][k] = a.P[jj + of.o[k]];
    }
  };
  int base = vw.bl * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (; base < n; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = base + v * kNT + (int)threadIdx.x;
      if (j >= n) continue;
      const uint32_t cv = c[v];
      if (!(cv & NB_SELF) || (cv & NB_BLACK)) continue;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) s += (double)pn[v][k];
      const double ip = h0[v];  // red pivots are h_r (1/h stored as 0 when h_r <= 0)
      if (!(ip > 0.0)) bad = 1;
      if (a.store_piv) a.ipiv[j] = ip;
      const T pj = (T)((double)g0[v] * ip + beta * s * ip);
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

// Red pass of the iteration fused with the direction step (Sec. III Algorithm,
// readings R6, R7): the incoming partials are the full dot products of
// k_rb_black<DOTS = true>, so mu is known at entry, and every voxel forms
//   z = -p + mu z_prev   (p_r from the red rule above, p_b from the black pass).
// The line-search sums A = z^T C^T C f and B = ||C z||^2 are taken over the
// edges of C: the 7-point stencil joins a red and a black voxel on every edge,
// so each red voxel adds (z_r - z_k)(f_r - f_k) and (z_r - z_k)^2 over its
// in-mask neighbours k, with z_k = -p_k + mu z_prev_k formed from their
// loaded values.  d0 = sum z^2 D over all voxels.  Partial sums as k_dir.
template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_rb_red_dir(IterArgs<T> a0) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = a.Gc;
  const T *__restrict__ zp = a.Zp;
  T *__restrict__ zo = a.Zc;
  const T *__restrict__ f = a.Fc;
  const T *__restrict__ p = a.P;
  const Offs of(g);
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V];
  T g0[V], p0[V], z0[V], f0[V], d0[V], pn[V][6], zn[V][6], fn[V][6];
  double h0[V];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      g0[v] = gg[jj];
      h0[v] = a.hinv[jj];
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
  const double beta = a.beta;
  const T mu = (T)st.mu;
  double acc[3] = {0.0, 0.0, 0.0};
  int bad = 0;
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
      T pj = p0[v];
      const bool red = !(cv & NB_BLACK);
      if (red) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(cv, k)) s += (double)pn[v][k];
        const double ip = h0[v];
        if (!(ip > 0.0)) bad = 1;
        pj = (T)((double)g0[v] * ip + beta * s * ip);
      }
      const T zj = -pj + mu * z0[v];
      zo[j] = zj;
      acc[2] += (double)zj * (double)zj * (double)d0[v];
      if (red) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(cv, k)) {
            const double dz = (double)(zj - (-pn[v][k] + mu * zn[v][k]));
            acc[0] += dz * (double)(f0[v] - fn[v][k]);
            acc[1] += dz * dz;
          }
      }
    }
    if (base + stride < n) load(base + stride);
  }
  if (bad) set_status(a.status, 5);
  store_partials<3, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DIR, vw.nb, vw.leader);
}

// ---------------------------------------------------------------------------
// Pair-mapped red-black passes of the iteration (used when every column has
// an even length).  Then voxels 2q and 2q+1 lie in one column and have
// opposite colours, so one thread per pair takes the pass's heavy voxel (the
// one whose six neighbours it reads: black in the black pass, red in the red
// pass) and the light one.  Compared with a voxel per lane, no lane loads
// neighbours it then discards, which halves the neighbour loads; the pair's
// own values move as one 2-element load or store.  Same arithmetic as
// k_rb_black<DOTS = true> and k_rb_red_dir.
#ifndef FM_VPAIR_B32
#define FM_VPAIR_B32 1
#endif
#ifndef FM_VPAIR_R32
#define FM_VPAIR_R32 2
#endif
template <typename T, int V32>
struct Vpair {  // pairs per thread
  static constexpr int v = sizeof(T) == 4 ? V32 : 1;
};

template <typename T>
struct alignas(2 * sizeof(T)) Duo {
  T v0, v1;
};

template <typename T>
__device__ __forceinline__ Duo<T> ld_duo(const T *p, int j0) {
  return *reinterpret_cast<const Duo<T> *>(p + j0);
}

// Colour of the pair from whichever code is in the mask (both out: either).
__device__ __forceinline__ bool first_is_black(uint32_t cA, uint32_t cB) {
  return (cA & NB_SELF) ? (cA & NB_BLACK) != 0 : (cB & NB_BLACK) == 0;
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_rb_black_pair(IterArgs<T> a0) {
  constexpr int V = Vpair<T, FM_VPAIR_B32>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = a.Gc;
  const T *__restrict__ gp = a.Gp;
  const double *__restrict__ hv = a.hinv;
  const Offs of(g);
  const int np = (int)(g.n >> 1), chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t cb[V], cr[V];
  int jb[V];
  T d0[V], g0[V], gp0[V], gr[V], gpr[V], gn[V][6], gpn[V][6];
  double hr[V], hn[V][6];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int q = b + v * kNT + (int)threadIdx.x;
      const int j0 = 2 * (q < np ? q : np - 1);
      const uint32_t c2 = *reinterpret_cast<const uint16_t *>(a.code + j0);
      const uint32_t cA = q < np ? (c2 & 0xffu) : 0u, cB = q < np ? (c2 >> 8) : 0u;
      const bool fb = first_is_black(cA, cB);
      const int jbv = fb ? j0 : j0 + 1, jrv = fb ? j0 + 1 : j0;
      jb[v] = jbv;
      cb[v] = fb ? cA : cB;
      cr[v] = fb ? cB : cA;
      const Duo<T> g2 = ld_duo(gg, j0), gp2 = ld_duo(gp, j0);
      g0[v] = fb ? g2.v0 : g2.v1;
      gr[v] = fb ? g2.v1 : g2.v0;
      gp0[v] = fb ? gp2.v0 : gp2.v1;
      gpr[v] = fb ? gp2.v1 : gp2.v0;
      hr[v] = hv[j0 >> 1];
      d0[v] = a.D[jbv];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        gn[v][k] = gg[jbv + of.o[k]];
        gpn[v][k] = gp[jbv + of.o[k]];
        hn[v][k] = hv[(jbv + of.o[k]) >> 1];  // a red neighbour: its pair's entry
      }
    }
  };
  int base = vw.bl * chunk;
  if (base < np) load(base);
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta, b2 = a.beta * a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (; base < np; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int q = base + v * kNT + (int)threadIdx.x;
      if (q >= np) continue;
      if (cr[v] & NB_SELF) {
        const double gh = (double)gr[v] * hr[v];
        acc[0] += (double)gr[v] * gh;
        acc[1] += (double)gpr[v] * gh;
      }
      const uint32_t cv = cb[v];
      if (!(cv & NB_SELF)) continue;
      const double h = (double)d0[v] + beta * nb_deg(cv);
      double sp = 0.0, sxv = 0.0, syp = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) {
          sp += hn[v][k];
          sxv += (double)gn[v][k] * hn[v][k];
          syp += (double)gpn[v][k] * hn[v][k];
        }
      const double piv = h - b2 * sp;
      double ip = 1.0 / piv;
      if (!(piv > 0.0)) {
        bad = 1;
        ip = 0.0;
      }
      const double yb = (double)g0[v] + beta * sxv;
      const double x = yb * ip;
      a.P[jb[v] >> 1] = (T)x;
      acc[0] += yb * x;
      acc[1] += ((double)gp0[v] + beta * syp) * x;
    }
    if (base + stride < np) load(base + stride);
  }
  if (bad) set_status(a.status, 5);
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DOTS, vw.nb, vw.leader);
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_rb_red_dir_pair(IterArgs<T> a0) {
  constexpr int V = Vpair<T, FM_VPAIR_R32>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = a.Gc;
  const T *__restrict__ zp = a.Zp;
  T *__restrict__ zo = a.Zc;
  const T *__restrict__ f = a.Fc;
  const T *__restrict__ p = a.P;
  const Offs of(g);
  const int np = (int)(g.n >> 1), chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t cb[V], cr[V];
  bool fbk[V];
  T gr[V], zr[V], fr[V], dr[V], pb[V], zb[V], db[V], pn[V][6], zn[V][6], fn[V][6];
  double hr[V];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int q = b + v * kNT + (int)threadIdx.x;
      const int j0 = 2 * (q < np ? q : np - 1);
      const uint32_t c2 = *reinterpret_cast<const uint16_t *>(a.code + j0);
      const uint32_t cA = q < np ? (c2 & 0xffu) : 0u, cB = q < np ? (c2 >> 8) : 0u;
      const bool fb = first_is_black(cA, cB);
      const int jrv = fb ? j0 + 1 : j0;
      fbk[v] = fb;
      cb[v] = fb ? cA : cB;
      cr[v] = fb ? cB : cA;
      const Duo<T> z2 = ld_duo(zp, j0), d2 = ld_duo(a.D, j0);
      zr[v] = fb ? z2.v1 : z2.v0;
      zb[v] = fb ? z2.v0 : z2.v1;
      dr[v] = fb ? d2.v1 : d2.v0;
      db[v] = fb ? d2.v0 : d2.v1;
      pb[v] = p[j0 >> 1];
      gr[v] = gg[jrv];
      fr[v] = f[jrv];
      hr[v] = a.hinv[j0 >> 1];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        pn[v][k] = p[(jrv + of.o[k]) >> 1];  // a black neighbour: its pair's entry
        zn[v][k] = zp[jrv + of.o[k]];
        fn[v][k] = f[jrv + of.o[k]];
      }
    }
  };
  int base = vw.bl * chunk;
  if (base < np) load(base);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  const T mu = (T)st.mu;
  double acc[3] = {0.0, 0.0, 0.0};
  int bad = 0;
  for (; base < np; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int q = base + v * kNT + (int)threadIdx.x;
      if (q >= np) continue;
      T zrv = T(0), zbv = T(0);
      const uint32_t cv = cr[v];
      if (cv & NB_SELF) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(cv, k)) s += (double)pn[v][k];
        const double ip = hr[v];
        if (!(ip > 0.0)) bad = 1;
        const T pj = (T)((double)gr[v] * ip + beta * s * ip);
        zrv = -pj + mu * zr[v];
        acc[2] += (double)zrv * (double)zrv * (double)dr[v];
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(cv, k)) {
            const double dz = (double)(zrv - (-pn[v][k] + mu * zn[v][k]));
            acc[0] += dz * (double)(fr[v] - fn[v][k]);
            acc[1] += dz * dz;
          }
      }
      if (cb[v] & NB_SELF) {
        zbv = -pb[v] + mu * zb[v];
        acc[2] += (double)zbv * (double)zbv * (double)db[v];
      }
      Duo<T> out;
      out.v0 = fbk[v] ? zbv : zrv;
      out.v1 = fbk[v] ? zrv : zbv;
      *reinterpret_cast<Duo<T> *>(zo + 2 * q) = out;
    }
    if (base + stride < np) load(base + stride);
  }
  if (bad) set_status(a.status, 5);
  store_partials<3, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DIR, vw.nb, vw.leader);
}

// Diagonal (P = diag H) or identity preconditioner.
template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_diag(IterArgs<T> a0, const T *__restrict__ gsrc, int identity) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ gg = gsrc ? gsrc + vw.off : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V];
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
        const double h = (double)d0[v] + beta * nb_deg(cv);
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

// ---------------------------------------------------------------------------
// Direction and line-search setup (Sec. III Algorithm and Sec. III-C).  The
// incoming dot products give the Polak-Ribiere mu (readings R6, R7); then
// z = -p + mu z_prev, A = z^T C^T C f, B = ||C z||^2 (once per outer
// iteration) and d0 = sum z^2 D, from which the next kernel takes the first
// step alpha = -z^T g / (d0 + beta B).
template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_dir(IterArgs<T> a0) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
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
      T lz = T(0), lf = T(0);
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) {
          lz += zj - (-pn[v][k] + mu * zn[v][k]);
          lf += f0[v] - fn[v][k];
        }
      zo[j] = zj;
      acc[0] += (double)zj * (double)lf;
      acc[1] += (double)zj * (double)lz;
      acc[2] += (double)zj * (double)zj * (double)d0[v];
    }
    if (base + stride < n) load(base + stride);
  }
  store_partials<3, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DIR, vw.nb, vw.leader);
}

// One further line-search pass (Sec. III-C eq. (ls_update)) at the current
// alpha: S1 = z^T grad Phi(f + alpha z), S2 = sum z^2 d(f + alpha z); the next
// kernel applies alpha <- alpha - (S1 + beta A + alpha beta B) / (S2 + beta B).
template <typename T, int LMAX, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mls(IterArgs<T> a0) {
  constexpr int V = Vk<T, LMAX <= 4 ? FM_V_MLS : FM_VPT32>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ f = a.Fc;
  const T *__restrict__ z = a.Zc;
  const int n = (int)g.n, chunk = kNT * V, stride = vw.nb * chunk;
  uint32_t c[V];
  T f0[V], z0[V], rho[V][LMAX], tau[V][LMAX];
  auto load = [&](int b) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = b + v * kNT + (int)threadIdx.x;
      const int jj = j < n ? j : n - 1;
      c[v] = j < n ? a.code[jj] : 0u;
      f0[v] = f[jj];
      z0[v] = z[jj];
      load_echoes<T, LMAX>(a.dat, vw.es, jj, a.L, rho[v], tau[v]);
    }
  };
  int base = vw.bl * chunk;
  if (base < n) load(base);
  const State st = take_state<kNT, 3>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const T alpha = (T)st.alpha;
  double acc[2] = {0.0, 0.0};
  for (; base < n; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = base + v * kNT + (int)threadIdx.x;
      if (j >= n || !(c[v] & NB_SELF)) continue;
      T phi, dphi, curv;
      voxel_terms<T, LMAX>(rho[v], tau[v], a.L, a.pairs, f0[v] + alpha * z0[v], phi, dphi, curv);
      acc[0] += (double)z0[v] * (double)dphi;
      acc[1] += (double)z0[v] * (double)z0[v] * (double)curv;
    }
    if (base + stride < n) load(base + stride);
  }
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_MLS, vw.nb, vw.leader);
}

// Mark loaded values as used where they were loaded: the compiler would
// otherwise sink a load whose value a masked voxel does not need into that
// voxel's branch, issuing it late and waiting for it alone.
__device__ __forceinline__ void keep(float4 v) { asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w)); }
__device__ __forceinline__ void keep(float v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep(uint32_t v) { asm volatile("" ::"v"(v)); }

// An echo-pair constant read by every lane alike, moved to scalar registers
// (the vector registers are the scarce ones in the four-voxel passes).
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ PairC<float> uniform_pair(const PairC<float> &p) {
  PairC<float> q = p;
  q.w = uniform_f(p.w);
  q.g = uniform_f(p.g);
  q.dt = uniform_f(p.dt);
  q.d2pi = uniform_f(p.d2pi);
  return q;
}

// The line-search pass of k_mls with four consecutive voxels per thread
// (FP32, NE = L echoes fixed at compile time so that no load is conditional,
// n a multiple of 4): the codes in one 4-byte load, f, z and each echo's data
// in 16-byte loads, so a wave's load moves 1 KiB of one array (k_mls's
// per-voxel loads move 256 B, and 64 B for the codes).  Same arithmetic per
// voxel; only the order of the partial sums differs.
template <int NE, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mls_q(IterArgs<float> a0) {
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<float> a = at_volume<BATCH>(a0, vw);
  const int nq = (int)(a.geo.n >> 2), stride = vw.nb * kNT;
  const int64_t es = vw.es;
  uint32_t c4;
  float4 f4, z4, d4[NE][2];
  auto load = [&](int q) {
    const int j = 4 * q;
    c4 = *reinterpret_cast<const uint32_t *>(a.code + j);
    f4 = *reinterpret_cast<const float4 *>(a.Fc + j);
    z4 = *reinterpret_cast<const float4 *>(a.Zc + j);
#pragma unroll
    for (int l = 0; l < NE; ++l) {
      const float4 *d = reinterpret_cast<const float4 *>(a.dat + (size_t)l * (size_t)es + j);
      d4[l][0] = d[0];
      d4[l][1] = d[1];
    }
  };
  int q = vw.bl * kNT + (int)threadIdx.x;
  const State st = take_state<kNT, 3>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow,
                                      vw.leader);
  const float alpha = (float)st.alpha;
  constexpr int NP = NE * (NE - 1) / 2;
  PairC<float> pc[NP];  // the echo-pair constants, read once into scalar registers
#pragma unroll
  for (int k = 0; k < NP; ++k) pc[k] = uniform_pair(a.pairs[k]);
  double acc[2] = {0.0, 0.0};
  for (; q < nq; q += stride) {
    load(q);
    keep(c4);
    keep(f4);
    keep(z4);
#pragma unroll
    for (int l = 0; l < NE; ++l) {
      keep(d4[l][0]);
      keep(d4[l][1]);
    }
    const float fv[4] = {f4.x, f4.y, f4.z, f4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool in = (c4 >> (8 * i)) & NB_SELF;
      float rho[NE], tau[NE];
#pragma unroll
      for (int l = 0; l < NE; ++l) {
        const float4 &d = d4[l][i >> 1];
        rho[l] = (i & 1) ? d.z : d.x;
        tau[l] = (i & 1) ? d.w : d.y;
      }
      float phi, dphi, curv;
      voxel_terms<float, NE>(rho, tau, NE, pc, fv[i] + alpha * zv[i], phi, dphi, curv);
      acc[0] += in ? (double)zv[i] * (double)dphi : 0.0;
      acc[1] += in ? (double)zv[i] * (double)zv[i] * (double)curv : 0.0;
    }
  }
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_MLS, vw.nb, vw.leader);
}

// The gradient pass of k_grad (iteration only: no final pass, no user
// output) with four consecutive voxels of a column per thread (FP32, at most
// four echoes, nz a multiple of 4): codes in one 4-byte load; f, z, the echo
// data and the +-x, +-y neighbours' f and z in 16-byte loads; the -z / +z
// neighbours inside the four from registers; f, g, D stored 16 bytes at a time
// (NE = L echoes fixed at compile time, as k_mls_q).  Every neighbour's updated
// f is formed with the expression k_grad uses, so f, g, D and 1/h are the same
// bits; only the order of the partial sums differs.
template <int NE, bool BATCH>
__global__ __launch_bounds__(kNT) void k_grad_q(IterArgs<float> a0) {
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<float> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const int nq = (int)(g.n >> 2), stride = vw.nb * kNT, sx = (int)g.sx, sy = (int)g.sy;
  const int64_t es = vw.es;
  const float *__restrict__ fin = a.Fp;
  const float *__restrict__ zin = a.Zp;
  uint32_t c4;
  float4 f4, z4, fx[2], zx[2], fy[2], zy[2], d4[NE][2];
  float fzm, zzm, fzp, zzp;  // f, z of the voxels below and above the four
  auto load = [&](int q) {
    const int j = 4 * q;
    c4 = *reinterpret_cast<const uint32_t *>(a.code + j);
    f4 = *reinterpret_cast<const float4 *>(fin + j);
    z4 = *reinterpret_cast<const float4 *>(zin + j);
    fx[0] = *reinterpret_cast<const float4 *>(fin + j - sx);
    fx[1] = *reinterpret_cast<const float4 *>(fin + j + sx);
    zx[0] = *reinterpret_cast<const float4 *>(zin + j - sx);
    zx[1] = *reinterpret_cast<const float4 *>(zin + j + sx);
    fy[0] = *reinterpret_cast<const float4 *>(fin + j - sy);
    fy[1] = *reinterpret_cast<const float4 *>(fin + j + sy);
    zy[0] = *reinterpret_cast<const float4 *>(zin + j - sy);
    zy[1] = *reinterpret_cast<const float4 *>(zin + j + sy);
    fzm = fin[j - 1];
    zzm = zin[j - 1];
    fzp = fin[j + 4];
    zzp = zin[j + 4];
#pragma unroll
    for (int l = 0; l < NE; ++l) {
      const float4 *d = reinterpret_cast<const float4 *>(a.dat + (size_t)l * (size_t)es + j);
      d4[l][0] = d[0];
      d4[l][1] = d[1];
    }
  };
  int q = vw.bl * kNT + (int)threadIdx.x;
  const State st = take_state<kNT, 3>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow,
                                      vw.leader);
  const float alpha = (float)st.alpha;
  const float beta = (float)a.beta;
  constexpr int NP = NE * (NE - 1) / 2;
  PairC<float> pc[NP];  // the echo-pair constants, read once into scalar registers
#pragma unroll
  for (int k = 0; k < NP; ++k) pc[k] = uniform_pair(a.pairs[k]);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (; q < nq; q += stride) {
    load(q);
    keep(c4);
    keep(f4);
    keep(z4);
#pragma unroll
    for (int l = 0; l < NE; ++l) {
      keep(d4[l][0]);
      keep(d4[l][1]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      keep(fx[k]);
      keep(zx[k]);
      keep(fy[k]);
      keep(zy[k]);
    }
    keep(fzm);
    keep(zzm);
    keep(fzp);
    keep(zzp);
    const int j = 4 * q;
    const float fv[4] = {f4.x, f4.y, f4.z, f4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
    const float fxm[4] = {fx[0].x, fx[0].y, fx[0].z, fx[0].w}, fxp[4] = {fx[1].x, fx[1].y, fx[1].z, fx[1].w};
    const float zxm[4] = {zx[0].x, zx[0].y, zx[0].z, zx[0].w}, zxp[4] = {zx[1].x, zx[1].y, zx[1].z, zx[1].w};
    const float fym[4] = {fy[0].x, fy[0].y, fy[0].z, fy[0].w}, fyp[4] = {fy[1].x, fy[1].y, fy[1].z, fy[1].w};
    const float zym[4] = {zy[0].x, zy[0].y, zy[0].z, zy[0].w}, zyp[4] = {zy[1].x, zy[1].y, zy[1].z, zy[1].w};
    float fo[4], go[4], dout[4];
    double hv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t cv = (c4 >> (8 * i)) & 0xffu;
      const bool in = cv & NB_SELF;
      const float fj = fv[i] + alpha * zv[i];
      const float fn[6] = {fxm[i] + alpha * zxm[i], fxp[i] + alpha * zxp[i], fym[i] + alpha * zym[i],
                           fyp[i] + alpha * zyp[i], i > 0 ? fv[i - 1] + alpha * zv[i - 1] : fzm + alpha * zzm,
                           i < 3 ? fv[i + 1] + alpha * zv[i + 1] : fzp + alpha * zzp};
      float lap = 0.f;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) lap += fj - fn[k];
      float rho[NE], tau[NE];
#pragma unroll
      for (int l = 0; l < NE; ++l) {
        const float4 &d = d4[l][i >> 1];
        rho[l] = (i & 1) ? d.z : d.x;
        tau[l] = (i & 1) ? d.w : d.y;
      }
      float phi, dphi, curv;
      voxel_terms<float, NE>(rho, tau, NE, pc, fj, phi, dphi, curv);
      const float gj = dphi + beta * lap;
      fo[i] = in ? fj : 0.f;
      go[i] = in ? gj : 0.f;
      dout[i] = in ? curv : 0.f;
      const double h = (double)curv + a.beta * nb_deg(cv);
      hv[i] = in && h > 0.0 ? 1.0 / h : 0.0;
      acc[0] += in ? (double)phi : 0.0;
      acc[1] += in ? (double)fj * (double)lap : 0.0;
      acc[2] += in ? (double)gj * (double)gj : 0.0;
      acc[3] += in ? (double)zv[i] * (double)gj : 0.0;
    }
    *reinterpret_cast<float4 *>(a.Fc + j) = make_float4(fo[0], fo[1], fo[2], fo[3]);
    *reinterpret_cast<float4 *>(a.Gc + j) = make_float4(go[0], go[1], go[2], go[3]);
    *reinterpret_cast<float4 *>(a.D + j) = make_float4(dout[0], dout[1], dout[2], dout[3]);
    if (a.write_hinv == 1) {
      *reinterpret_cast<double2 *>(a.hinv + j) = make_double2(hv[0], hv[1]);
      *reinterpret_cast<double2 *>(a.hinv + j + 2) = make_double2(hv[2], hv[3]);
    } else if (a.write_hinv == 2) {
      // 1/h of each pair's red voxel at the pair index (x + y + z even is red)
      const int col = j / sy, x = col / g.ny, y = col - x * g.ny;
      const bool first_red = ((x + y) & 1) == 0;  // the pair's first voxel (z even) is red
      *reinterpret_cast<double2 *>(a.hinv + (j >> 1)) =
          make_double2(first_red ? hv[0] : hv[1], first_red ? hv[2] : hv[3]);
    }
  }
  store_partials<4, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_GRAD, vw.nb, vw.leader);
}

}  // namespace fm
