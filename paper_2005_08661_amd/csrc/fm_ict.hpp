// Incomplete Cholesky with a drop tolerance (IC_t) of H = diag(D) + beta C^T C
// in natural order (Sec. III-B eqs. (precon_hess), (precon); the tolerance
// H_max x factor of Table 1 and Sec. IV), with its fill bounded to the
// level-K pattern of natural-order IC (K = 0, 1, 2).
//
// Factor H ~ L L^T row by row: for each pattern position k = j - o of row j,
//   L_jk = (H_jk - sum_{m < k} L_jm L_km) / L_kk,
// then L_jk = 0 if |L_jk| < tol ||H(k:N, k)||_1 (tol = factor x H_max, the
// largest magnitude in H), and L_jj = sqrt(H_jj - sum_k L_jk^2).  The solves
// are L y = g in natural order and L^T p = y in reverse.
//
// Schedule: every offset o = (dx, dy, dz) of the pattern satisfies
// a dx + b dy + dz >= 1 for the level's weights (a, b) (level 0: 1, 1;
// level 1: 3, 2; level 2: 7, 3), so the voxels with a x + b y + z = s depend
// only on voxels of smaller s.  One launch handles one such level s (the
// factor row and the forward solve of each of its voxels, or the backward
// solve in reverse level order); the launches run back to back from a HIP
// graph.  Neither kernel takes part in the chain of scalar state: the
// conjugacy dot products come from k_ict_dots afterwards.
//
// Storage: lo[u][j] = L(j, j - o_u) in the offsets' table order (descending
// lexicographic (dx, dy, dz)), ld[j] = L_jj, y and p in FP64.  For two
// offsets that are both inside the volume for the same row, lexicographic
// order is voxel-index order, so the unrolled loops add the products in
// ascending column order, as a sequential row-by-row factorisation does.
// FP contraction is off in these kernels: every product is rounded before
// it is subtracted.
#pragma once

#include "fm_stream.hpp"

namespace fm {

constexpr int kIctMaxOff = 11;  // offsets of the level-2 pattern
// Threads per workgroup of the level kernels: half a wavefront.  A level has
// at most nx x ceil(nz / b) voxels whose neighbours lie about nz elements
// apart, so every lane's load is a cache line of its own and a compute unit's
// address processing bounds the launch; small workgroups spread a level over
// more compute units (measured per 10-iteration solve at 128x128x64: 108 ms
// with 256 threads, 78 with 128, 64 with 64, 61 with 32, 60 with 16).
constexpr int kIctNT = 32;

// Lower offsets (dx, dy, dz) of the level-K fill pattern, descending
// lexicographic order, and the level weights (a, b) of the schedule.
template <int LEVEL>
struct IctPattern;
template <>
struct IctPattern<0> {
  static constexpr int n = 3, a = 1, b = 1;
  static constexpr int off[n][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
};
template <>
struct IctPattern<1> {
  static constexpr int n = 6, a = 3, b = 2;
  static constexpr int off[n][3] = {{1, 0, 0}, {1, 0, -1}, {1, -1, 0}, {0, 1, 0}, {0, 1, -1}, {0, 0, 1}};
};
template <>
struct IctPattern<2> {
  static constexpr int n = 11, a = 7, b = 3;
  static constexpr int off[n][3] = {{1, 0, 0},  {1, 0, -1}, {1, 0, -2}, {1, -1, 1}, {1, -1, 0}, {1, -1, -1},
                                    {1, -2, 0}, {0, 1, 0},  {0, 1, -1}, {0, 1, -2}, {0, 0, 1}};
};

// For row entry u and an earlier entry v (o_v > o_u): the offset w with
// o_v = o_u + o_w, i.e. m = j - o_v is the entry w of row k = j - o_u; -1 if
// o_v - o_u is not in the pattern.
template <int LEVEL>
__host__ __device__ constexpr int ict_pair(int u, int v) {
  using P = IctPattern<LEVEL>;
  const int dx = P::off[v][0] - P::off[u][0], dy = P::off[v][1] - P::off[u][1], dz = P::off[v][2] - P::off[u][2];
  for (int w = 0; w < P::n; ++w)
    if (P::off[w][0] == dx && P::off[w][1] == dy && P::off[w][2] == dz) return w;
  return -1;
}

template <typename T>
struct IctArgs {
  Geo geo;
  double beta;
  double factor;          // tol = factor x H_max
  const double *hmax;     // H_max of this factorisation (device scalar)
  const uint8_t *code;
  const T *D;             // curvature of the Huber model
  int32_t kcol;           // threads per x column of a level: floor((nz - 1) / b) + 1
  double *lo;             // [noff][n]
  double *ld;             // [n]
  double *y;              // [n] forward-solve values
  double *pd;             // [n] p in FP64
  T *P;                   // [n] p in the working type
  int32_t *status;
};

// Voxel of level s handled by thread t (false: none).
template <int LEVEL, typename T>
__device__ __forceinline__ bool ict_voxel(const IctArgs<T> &a, int s, int t, int &x, int &y, int &z) {
  constexpr int A = IctPattern<LEVEL>::a, B = IctPattern<LEVEL>::b;
  const Geo &g = a.geo;
  x = t / a.kcol;
  const int q = t - x * a.kcol;
  if (x >= g.nx) return false;
  const int r = s - A * x;  // = b y + z
  if (r < 0) return false;
  const int ylo = r - (g.nz - 1) > 0 ? (r - (g.nz - 1) + B - 1) / B : 0;
  y = ylo + q;
  if (y >= g.ny || B * y > r) return false;
  z = r - B * y;
  return true;
}

__device__ __forceinline__ bool ict_inside(const Geo &g, int x, int y, int z) {
  return x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
}

// H_max = max over in-mask voxels of |D_j + beta deg_j| and, where a voxel has
// an in-mask neighbour, beta: one maximum per workgroup, then one overall.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ict_hmax(Geo g, const uint8_t *__restrict__ code, const T *__restrict__ D,
                                                     double beta, double *part) {
  double m = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < g.n; j += (int64_t)gridDim.x * kBlock) {
    const uint32_t c = code[j];
    if (!(c & NB_SELF)) continue;
    const int deg = nb_deg(c);
    m = fmax(m, fabs((double)D[j] + beta * deg));
    if (deg > 0) m = fmax(m, beta);
  }
  __shared__ double red[kBlock];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_ict_hmax_fin(const double *__restrict__ part, int nparts, double *hmax) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBlock) m = fmax(m, part[b]);
  __shared__ double red[kBlock];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *hmax = red[0];
}

// Level s of the factorisation and of the forward solve L y = g.
template <typename T, int LEVEL>
__global__ __launch_bounds__(kIctNT) void k_ict_fwd(IctArgs<T> a, const T *__restrict__ gsrc, int s) {
#pragma clang fp contract(off)
  using Pat = IctPattern<LEVEL>;
  constexpr int NO = Pat::n;
  int x, y, z;
  if (!ict_voxel<LEVEL>(a, s, (int)(blockIdx.x * kIctNT + threadIdx.x), x, y, z)) return;
  const Geo g = a.geo;
  const int n = (int)g.n;
  const int j = (x * g.ny + y) * g.nz + z;
  // Every load of the voxel is issued before the mask test (a level is a
  // chain of dependent memory round trips; the test must not add one).
  const uint32_t c = a.code[j];
  const double hmax = *a.hmax, dj = (double)a.D[j], gj = (double)gsrc[j];
  const double beta = a.beta;
  // the earlier voxels k = j - o_u of the pattern (-1: outside the volume or
  // the mask), their L_kk, y_k and ||H(k:N, k)||_1 = |H_kk| + beta x (in-mask
  // neighbours after k), and the entries of their rows the products use
  int kv[NO];
  double lkk[NO], yk[NO], cn[NO], lkm[NO][NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int kx = x - Pat::off[u][0], ky = y - Pat::off[u][1], kz = z - Pat::off[u][2];
    const int k0 = ict_inside(g, kx, ky, kz) ? (kx * g.ny + ky) * g.nz + kz : j;
    const uint32_t ck = a.code[k0];
    const bool ok = k0 != j && (ck & NB_SELF);
    kv[u] = ok ? k0 : -1;
    // values of a position outside the volume or the mask are selected away,
    // never multiplied by zero (the substituted slot may hold anything)
    const double ldk = a.ld[k0], ykk = a.y[k0];
    lkk[u] = ok ? ldk : 1.0;
    yk[u] = ok ? ykk : 0.0;
    double cnu = fabs((double)a.D[k0] + beta * nb_deg(ck));
    if (ck & NB_XP) cnu = cnu + beta;
    if (ck & NB_YP) cnu = cnu + beta;
    if (ck & NB_ZP) cnu = cnu + beta;
    cn[u] = cnu;
#pragma unroll
    for (int v = 0; v < NO; ++v) {
      const int w = ict_pair<LEVEL>(u, v);
      const double e = (v < u && w >= 0) ? a.lo[(size_t)w * n + k0] : 0.0;
      lkm[u][v] = ok ? e : 0.0;
    }
  }
  if (!(c & NB_SELF)) {
#pragma unroll
    for (int u = 0; u < NO; ++u) a.lo[(size_t)u * n + j] = 0.0;
    a.ld[j] = 0.0;
    a.y[j] = 0.0;
    return;
  }
  const double tol = a.factor * hmax;
  double row[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const bool stencil = Pat::off[u][0] + Pat::off[u][1] + Pat::off[u][2] == 1 && Pat::off[u][0] >= 0 &&
                         Pat::off[u][1] >= 0 && Pat::off[u][2] >= 0;
    double sum = stencil ? -beta : 0.0;  // H_jk
    // m = j - o_v over the earlier entries v of this row, ascending m
#pragma unroll
    for (int v = 0; v < u; ++v)
      if (ict_pair<LEVEL>(u, v) >= 0) sum = sum - row[v] * lkm[u][v];
    double val = sum / lkk[u];
    if (fabs(val) < tol * cn[u]) val = 0.0;
    row[u] = kv[u] >= 0 ? val : 0.0;
  }
  double diag = dj + beta * nb_deg(c);
#pragma unroll
  for (int u = 0; u < NO; ++u) diag = diag - row[u] * row[u];
  const bool bad = !(diag > 0.0);
  const double ljj = bad ? 0.0 : sqrt(diag);
  double yv = gj;
#pragma unroll
  for (int u = 0; u < NO; ++u) yv = yv - row[u] * yk[u];
#pragma unroll
  for (int u = 0; u < NO; ++u) a.lo[(size_t)u * n + j] = row[u];
  a.ld[j] = ljj;
  a.y[j] = bad ? 0.0 : yv / ljj;
  if (bad) set_status(a.status, isfinite(diag) ? 5 : 6);
}

// Level s (in reverse order) of the backward solve L^T p = y: p_j = (y_j -
// sum_i L_ij p_i) / L_jj over the later voxels i = j + o_u, ascending.
template <typename T, int LEVEL>
__global__ __launch_bounds__(kIctNT) void k_ict_bwd(IctArgs<T> a, int s) {
#pragma clang fp contract(off)
  using Pat = IctPattern<LEVEL>;
  constexpr int NO = Pat::n;
  int x, y, z;
  if (!ict_voxel<LEVEL>(a, s, (int)(blockIdx.x * kIctNT + threadIdx.x), x, y, z)) return;
  const Geo g = a.geo;
  const int n = (int)g.n;
  const int j = (x * g.ny + y) * g.nz + z;
  const uint32_t c = a.code[j];  // loaded with the rest, tested after (as in the forward sweep)
  const double yj = a.y[j], lj = a.ld[j];
  double li[NO], pi[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int ix = x + Pat::off[u][0], iy = y + Pat::off[u][1], iz = z + Pat::off[u][2];
    const int i0 = ict_inside(g, ix, iy, iz) ? (ix * g.ny + iy) * g.nz + iz : j;
    const bool ok = i0 != j && (a.code[i0] & NB_SELF);
    const double e = a.lo[(size_t)u * n + i0], pv = a.pd[i0];
    li[u] = ok ? e : 0.0;
    pi[u] = ok ? pv : 0.0;
  }
  if (!(c & NB_SELF)) {
    a.pd[j] = 0.0;
    a.P[j] = T(0);
    return;
  }
  double sum = yj;
#pragma unroll
  for (int u = NO - 1; u >= 0; --u) sum = sum - li[u] * pi[u];
  const double p = sum / lj;
  a.pd[j] = p;
  a.P[j] = (T)p;
}

// Conjugacy dot products g^T p and g_prev^T p (p from the IC_t solves, FP64),
// in the chain of scalar state like the other preconditioner passes.
template <typename T>
__global__ __launch_bounds__(kNT) void k_ict_dots(IterArgs<T> a0, const double *__restrict__ pd,
                                                  const T *__restrict__ gsrc) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow,
                                      vw.leader);
  const int n = (int)a.geo.n;
  double acc[2] = {0.0, 0.0};
  for (int j = (int)(blockIdx.x * kNT + threadIdx.x); j < n; j += (int)(gridDim.x * kNT)) {
    if (!(a.code[j] & NB_SELF)) continue;
    const double p = pd[j];
    acc[0] += (double)gg[j] * p;
    acc[1] += (double)a.Gp[j] * p;
  }
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DOTS, vw.nb, vw.leader);
}

// Pivots L_jj^2 (0 outside the mask) for fm_precondition.
__global__ __launch_bounds__(kBlock) void k_ict_piv(int64_t n, const uint8_t *__restrict__ code,
                                                    const double *__restrict__ ld, double *piv) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
    piv[j] = (code[j] & NB_SELF) ? ld[j] * ld[j] : 0.0;
}

}  // namespace fm
