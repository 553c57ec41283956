// HIP kernels of the preconditioned NCG-MLS field-map iteration for gfx950.
//
// Storage: every per-voxel array is z fastest (j = (x*ny + y)*nz + z).
// T is the per-voxel storage/arithmetic type (double for F64, float for MIX);
// pivots, reductions and scalars are always FP64.
//
// Ping-pong buffers keyed by the iteration index i held on the device:
//   F[i&1] = f^i, Z[i&1] = z^i, G[i&1] = g^i; index (i+1)&1 holds the
//   previous iterate (f^{i-1}, z^{i-1}, g^{i-1}).
#pragma once

#include "fm_common.hpp"

namespace fm {

template <typename T>
struct T2 {
  T x, y;
};

struct Geo {
  int32_t nx, ny, nz;
  int64_t n;
  int64_t sx, sy;  // strides of x and y (z stride is 1)
};

// ---------------------------------------------------------------------------
// Setup (Sec. II eq. (r), the Algorithm's precompute): coil combination into
// per-echo magnitude |zhat_l| and phase angle(zhat_l)/2pi (turns), the
// neighbour code, the in-mask count, the field-map initial value of eq. (w0)
// and, for water-fat, the PWLS weight rho_j of Sec. III-A.
template <typename T>
struct SetupArgs {
  Geo geo;
  int32_t ncoil, L;
  const float2 *y;     // [ncoil][L][n]
  const float2 *sens;  // [ncoil][n] or nullptr
  const uint8_t *mask;
  T2<T> *dat;          // [L][estride] (|zhat|, angle/2pi)
  int64_t estride;     // echo stride of dat (n, or the batch's padded total)
  uint8_t *code;
  double *f0;          // field-map init output (double) or nullptr
  double inv_2pi_dt;   // 1 / (2 pi (t_2 - t_1))
  double *rho;         // water-fat PWLS weights or nullptr
  const double *gabs;  // [L*L] |Gamma_mn| (water-fat) or nullptr
  const PairC<double> *pairs_d;  // FP64 pair table for the water-fat sweep
  int32_t npairs;
  int32_t nsweep;      // water-fat sweep values (0 = no sweep)
  double sweep_half;   // |delta_f| / 2
  double *ftilde;      // water-fat sweep output or nullptr
  double *partials;    // [kMaxK][gridDim.x] in-mask counts
};

// LMAX bounds the echo count (compile-time register arrays); WF selects the
// water-fat outputs (the sweep and the PWLS weights), so the field-map
// instantiation carries none of their registers.
template <typename T, int LMAX, bool WF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LMAX <= 3 ? 3 : 1))) void k_setup(SetupArgs<T> a) {
  const Geo g = a.geo;
  double cnt[1] = {0.0};
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < g.n; j += (int64_t)gridDim.x * kBlock) {
    const int32_t z = (int32_t)(j % g.nz);
    const int32_t yy = (int32_t)((j / g.nz) % g.ny);
    const int32_t x = (int32_t)(j / g.sx);
    const bool in = a.mask[j] != 0;
    uint32_t c = 0;
    if (in) {
      c = NB_SELF;
      if ((x + yy + z) & 1) c |= NB_BLACK;
      if (x > 0 && a.mask[j - g.sx]) c |= NB_XM;
      if (x < g.nx - 1 && a.mask[j + g.sx]) c |= NB_XP;
      if (yy > 0 && a.mask[j - g.sy]) c |= NB_YM;
      if (yy < g.ny - 1 && a.mask[j + g.sy]) c |= NB_YP;
      if (z > 0 && a.mask[j - 1]) c |= NB_ZM;
      if (z < g.nz - 1 && a.mask[j + 1]) c |= NB_ZP;
      cnt[0] += 1.0;
    }
    a.code[j] = (uint8_t)c;
    // coil sums, a chunk of CU coils at a time with all of the chunk's loads
    // issued together (the coil map of a coil is loaded once for all echoes);
    // each sum still runs over the coils in order
    constexpr int CU = LMAX <= 4 ? 8 : (LMAX <= 8 ? 4 : 2);
    double ss = a.sens ? 0.0 : 1.0;
    double sre[LMAX], sim[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) sre[l] = sim[l] = 0.0;
    for (int c0 = 0; c0 < a.ncoil; c0 += CU) {
      float2 sv[CU], yv[CU][LMAX];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const int cc = c0 + u < a.ncoil ? c0 + u : c0;
        sv[u] = a.sens ? a.sens[(int64_t)cc * g.n + j] : make_float2(1.f, 0.f);
#pragma unroll
        for (int l = 0; l < LMAX; ++l) yv[u][l] = a.y[((int64_t)cc * a.L + (l < a.L ? l : 0)) * g.n + j];
      }
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        if (c0 + u >= a.ncoil) break;
        const float2 sc = sv[u];
        if (a.sens) ss += (double)sc.x * sc.x + (double)sc.y * sc.y;
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
          const float2 yl = yv[u][l];
          if (a.sens) {
            sre[l] += (double)sc.x * yl.x + (double)sc.y * yl.y;
            sim[l] += (double)sc.x * yl.y - (double)sc.y * yl.x;
          } else {
            sre[l] += yl.x;
            sim[l] += yl.y;
          }
        }
      }
    }
    const double scale = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    double z1r = 0, z1i = 0, z2r = 0, z2i = 0;
    double mag[LMAX], ph[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
      mag[l] = ph[l] = 0.0;
      if (l >= a.L) continue;
      const double re = sre[l] * scale, im = sim[l] * scale;
      if (l == 0) { z1r = re; z1i = im; }
      if (l == 1) { z2r = re; z2i = im; }
      mag[l] = sqrt(re * re + im * im);
      ph[l] = atan2(im, re) * 0.15915494309189533577;
      T2<T> d;
      d.x = (T)mag[l];
      d.y = (T)ph[l];
      a.dat[(int64_t)l * a.estride + j] = d;
    }
    if (WF && a.ftilde) {
      // Sec. III-A water-fat start: the sweep value of least per-voxel cost
      // (first one on ties), evaluated in FP64 in every precision mode.  Per
      // pair, 1 - cos(2 pi xi) = 2 sin^2(pi h) with h the wrap of xi; sin(pi h)
      // from the FP64 Taylor form of sinx_cos (|pi h| <= pi/2).
      double best = 1.0 / 0.0, bestf = 0.0;
      if (in) {
        constexpr int NPM = LMAX * (LMAX - 1) / 2;
        constexpr bool HOIST = LMAX <= 6;  // the per-voxel pair parts fit in registers
        // the per-pair parts that do not depend on the sweep value, formed once
        // with the expressions of the per-value form (same bits); slot k of the
        // unrolled (m, n) loops, pair pq of the table (slots with n >= L skipped)
        double pa[HOIST ? NPM : 1], pw[HOIST ? NPM : 1];
        if constexpr (HOIST) {
          int k = 0, pq = 0;
#pragma unroll
          for (int m = 0; m < LMAX; ++m) {
#pragma unroll
            for (int n2 = m + 1; n2 < LMAX; ++n2, ++k) {
              pa[k] = pw[k] = 0.0;
              if (n2 < a.L) {
                const PairC<double> P = a.pairs_d[pq];
                pa[k] = P.g + (ph[n2] - ph[m]);
                pw[k] = P.w * mag[m] * mag[n2];
                ++pq;
              }
            }
          }
        }
        for (int q = 0; q < a.nsweep; ++q) {
          const double fs = -a.sweep_half + 2.0 * a.sweep_half * q / (a.nsweep - 1);
          double c0 = 0.0;
          int k = 0, pq = 0;
#pragma unroll
          for (int m = 0; m < LMAX; ++m) {
#pragma unroll
            for (int n2 = m + 1; n2 < LMAX; ++n2, ++k) {
              if (n2 < a.L) {
                const PairC<double> P = a.pairs_d[pq];
                double xi, w;
                if constexpr (HOIST) {
                  xi = pa[k] + fs * P.dt;
                  w = pw[k];
                } else {
                  xi = P.g + (ph[n2] - ph[m]) + fs * P.dt;
                  w = P.w * mag[m] * mag[n2];
                }
                const double x = 3.14159265358979323846 * (xi - rint(xi));
                double sx, cs;
                sinx_cos(x, sx, cs);
                const double sn = x * sx;
                c0 += w * (2.0 * sn * sn);
                ++pq;
              }
            }
          }
          if (c0 < best) {
            best = c0;
            bestf = fs;
          }
        }
      }
      a.ftilde[j] = in ? bestf : 0.0;
    }
    if (a.f0) {
      // eq. (w0): angle(conj(z_1) z_2) / (2 pi (t_2 - t_1))
      const double pr = z1r * z2r + z1i * z2i, pi = z1r * z2i - z1i * z2r;
      a.f0[j] = in ? atan2(pi, pr) * a.inv_2pi_dt : 0.0;
    }
    if (WF && a.rho) {
      // rho_j = (1/S_j) sum_{m,n} |Gamma_mn| a_m a_n, a_m = sum_c |s_c| |y_cm|
      double av[LMAX];
#pragma unroll
      for (int m = 0; m < LMAX; ++m) {
        av[m] = 0.0;
        if (m >= a.L) continue;
        double am = 0.0;
        for (int cc = 0; cc < a.ncoil; ++cc) {
          const float2 yv = a.y[((int64_t)cc * a.L + m) * g.n + j];
          double sm = 1.0;
          if (a.sens) {
            const float2 s = a.sens[(int64_t)cc * g.n + j];
            sm = sqrt((double)s.x * s.x + (double)s.y * s.y);
          }
          am += sm * sqrt((double)yv.x * yv.x + (double)yv.y * yv.y);
        }
        av[m] = am;
      }
      double r = 0.0;
#pragma unroll
      for (int m = 0; m < LMAX; ++m)
#pragma unroll
        for (int n2 = 0; n2 < LMAX; ++n2)
          if (m < a.L && n2 < a.L) r += a.gabs[m * a.L + n2] * av[m] * av[n2];
      a.rho[j] = (in && ss > 0.0) ? r / ss : 0.0;
    }
  }
  store_partials<1>(cnt, a.partials);
}

// In-mask count from the setup partials (one block).
__global__ __launch_bounds__(kBlock) void k_count(const double *__restrict__ partials, int nparts, double *nmask) {
  double t[kMaxK];
  sum_partials<1>(partials, nparts, 1, t, nparts);
  if (threadIdx.x == 0) *nmask = t[0];
}

// Fresh scalar state (block 0 writes it).
__device__ __forceinline__ void init_state(State *sout, int trace_cap, int nmls, const double *nmask) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State s{};
    s.iter = 0;
    s.kind = PK_NONE;
    s.nparts = 0;
    s.nmls = nmls;
    s.trace_cap = trace_cap;
    s.nmask = nmask ? *nmask : 0.0;
    *sout = s;
  }
}

// Start of a solve: fresh state and the initial map in F[1] (the slot read as
// the previous iterate by the first gradient pass), zero previous direction
// and gradient.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_start(Geo g, const double *__restrict__ f0,
                                                   const uint8_t *__restrict__ code, T *Fprev,
                                                   T *Zprev, T *Gprev, int64_t gcount, State *sout, int trace_cap,
                                                   int nmls, const double *nmask) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < g.n; j += (int64_t)gridDim.x * kBlock) {
    Fprev[j] = (code[j] & NB_SELF) ? (T)f0[j] : T(0);
    Zprev[j] = T(0);
  }
  // gcount elements of the gradient (more than n in the colour-major layout)
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < gcount; j += (int64_t)gridDim.x * kBlock)
    Gprev[j] = T(0);
  init_state(sout, trace_cap, nmls, nmask);
}

__global__ void k_state_init(State *sout, int trace_cap, int nmls) { init_state(sout, trace_cap, nmls, nullptr); }

// ---------------------------------------------------------------------------
// Gradient pass of iteration i (Sec. III eq. (ls_grad), fused with the update
// f^i = f^{i-1} + alpha z^{i-1} of the previous iteration):
//   g_j = dphi_j(f_j) + beta (C^T C f)_j,  D_j = Huber curvature (eq. (ls_huber)).
// Grid totals: sum phi, f^T C^T C f, ||g||^2, z_prev^T g.
// Batches: many volumes advance together, one launch per pass.  The
// per-voxel arrays of all volumes are concatenated (each volume padded by its
// own x-plane on both sides); the launch's workgroups are partitioned among
// the volumes, and each volume keeps its own scalar state and partial sums.
struct VolDesc {
  Geo geo;
  int64_t off;     // global index of the volume's voxel 0
  int32_t b0, nb;  // its workgroups [b0, b0 + nb) of a streaming launch
  double beta;
  int32_t tty, txc, tnyt;  // plane-march tiles of the red-black passes: strip width, run length, strips
};

struct Batch {
  const VolDesc *vol;        // [nvol]
  const int32_t *blockvol;   // [grid] volume of each workgroup
  int64_t estride;           // echo stride of the echo data (all padded voxels)
  int64_t trace_stride;      // doubles per volume trace
  double *const *fouts;      // final pass: output map of each volume
};

template <typename T>
struct IterArgs {
  Geo geo;
  int32_t L;
  double beta;
  const T2<T> *dat;
  const uint8_t *code;
  const PairC<T> *pairs;
  T *F[2];
  T *Z[2];
  T *G[2];
  T *D;
  T *X;
  T *X2;         // second forward-solve vector (three-colour IC(0))
  T *P;
  const uint8_t *rdiag;  // diag(C^T C) of the second-order operator (three-colour IC(0), colour-major)
  const uint8_t *ccode;  // neighbour codes in the colour-major layout (three-colour IC(0))
  int32_t cm;            // G, D, P, ipiv, X, X2 are colour-major (three-colour IC(0) plans)
  T *Pv, *Dv;            // voxel-order copies of p and D (three-colour IC(0) plans)
  double *ipiv;  // 1 / pivot
  double *hinv;  // 1 / (D + beta deg), written by the gradient pass when needed
  int32_t write_hinv;  // gradient pass also writes hinv (red-black IC(0)): 1 for every voxel at j;
                       // 2 for the pair-mapped passes: of red voxels only, at their pair j >> 1
  int32_t store_piv;   // preconditioner passes also store every pivot
  int32_t par;         // parity of the iteration this launch belongs to
  int32_t nparts_in;   // partial sums left by the previous launch (blocks)
  int32_t nvals_in;    // values per block in them
  const State *sin;    // incoming scalar state
  State *sout;         // outgoing scalar state (block 0)
  const double *pin;   // incoming partial sums
  double *pout;        // outgoing partial sums
  int32_t *status;     // sticky device status word
  double *trace;       // [trace_cap + 1][8]
  double *fout;        // final pass: user output (double) or nullptr
  int32_t final_pass;
  int32_t reg2;        // second-order regulariser (fm_eval only; the passes have their own kernels)
  Batch bt;            // batched launches only
};

// A workgroup's view of its volume: geometry, offset of the volume in the
// concatenated arrays, position among the volume's workgroups, and where its
// state and incoming partial sums are.
struct VolView {
  Geo g;
  int off;
  int vol;
  int bl, nb;       // workgroup index within the volume, workgroups of the volume
  int pfirst;       // first incoming partial of the volume
  int pcount;       // incoming partials of the volume
  int prow;         // row stride of the incoming partials
  int64_t es;       // echo stride
  double beta;
  bool leader;
};

template <bool BATCH, typename A>
__device__ __forceinline__ VolView vol_view(const A &a) {
  VolView w;
  if (!BATCH) {
    w.g = a.geo;
    w.off = 0;
    w.vol = 0;
    w.bl = (int)blockIdx.x;
    w.nb = (int)gridDim.x;
    w.pfirst = 0;
    w.pcount = a.nparts_in;
    w.prow = a.nparts_in;
    w.es = a.geo.n;
    w.beta = a.beta;
  } else {
    const int v = a.bt.blockvol[blockIdx.x];
    const VolDesc d = a.bt.vol[v];
    w.g = d.geo;
    w.off = (int)d.off;
    w.vol = v;
    w.bl = (int)blockIdx.x - d.b0;
    w.nb = d.nb;
    w.pfirst = d.b0;
    w.pcount = a.nparts_in ? d.nb : 0;  // the predecessor used the same partition
    w.prow = (int)gridDim.x;
    w.es = a.bt.estride;
    w.beta = d.beta;
  }
  w.leader = (w.bl == 0);
  return w;
}

template <typename T, int LMAX>
__device__ __forceinline__ void load_echoes(const T2<T> *__restrict__ dat, int64_t n, int j, int L,
                                            T (&rho)[LMAX], T (&tau)[LMAX]) {
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    if (l < L) {
      const T2<T> *__restrict__ dl = dat + (size_t)l * (size_t)n;  // uniform per echo
      const T2<T> d = dl[j];
      rho[l] = d.x;
      tau[l] = d.y;
    } else {
      rho[l] = T(0);
      tau[l] = T(0);
    }
  }
}

// End of a solve (one block): consume the final gradient pass (the cost of
// the final map) and leave a state from which the iteration can continue.
__global__ __launch_bounds__(kBlock) void k_finish(const State *sin, State *sout, const double *pin, int nparts_in,
                                                    int nvals_in, double beta, double *trace, int32_t *status) {
  const State st = take_state<kBlock, 4>(sin, pin, nparts_in, nvals_in, beta, trace, status);
  put_state(st, sout, PK_NONE, 0);
}

// End of a batched solve: workgroup v consumes volume v's partial sums.
__global__ __launch_bounds__(kBlock) void k_finish_batch(Batch bt, const State *sin, State *sout, const double *pin,
                                                          int nparts_in, int rowstride, int nvals_in, double *trace,
                                                          int32_t *status) {
  const int v = (int)blockIdx.x;
  const VolDesc d = bt.vol[v];
  const State st = take_state<kBlock, 4>(sin + v, pin + (nparts_in ? d.b0 : 0), nparts_in ? d.nb : 0, nvals_in,
                                         d.beta, trace + (size_t)v * bt.trace_stride, status, rowstride, true);
  put_state(st, sout + v, PK_NONE, 0, true);
}

// hinv_j = 1 / (D_j + beta deg_j) for the standalone preconditioner call.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_hinv(Geo g, double beta, const uint8_t *__restrict__ code,
                                                  const T *__restrict__ D, double *hinv, int32_t *status) {
  int bad = 0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < g.n; j += (int64_t)gridDim.x * kBlock) {
    const uint32_t c = code[j];
    double v = 0.0;
    if (c & NB_SELF) {
      const double h = (double)D[j] + beta * nb_deg(c);
      if (h > 0.0) v = 1.0 / h; else bad = 1;
    }
    hinv[j] = v;
  }
  if (bad) set_status(status, 5);
}

// ---------------------------------------------------------------------------
// Evaluation at a user-supplied map (row-level checks and the adjoint).
// The second-difference row centred at a voxel along axis ax exists when both
// of its ax-neighbours are in the mask (both code bits set).
__device__ __forceinline__ bool row2_code(uint32_t c, int ax) { return ((c >> (2 * ax + 1)) & 3u) == 3u; }

template <typename T, int LMAX>
__global__ __launch_bounds__(kBlock) void k_eval(IterArgs<T> a, const double *__restrict__ fu,
                                                  double *phi_o, double *dphi_o, double *curv_o,
                                                  double *lap_o) {
  const Geo g = a.geo;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < g.n; j += (int64_t)gridDim.x * kBlock) {
    const uint32_t c = a.code[j];
    if (!(c & NB_SELF)) {
      if (phi_o) phi_o[j] = 0.0;
      if (dphi_o) dphi_o[j] = 0.0;
      if (curv_o) curv_o[j] = 0.0;
      if (lap_o) lap_o[j] = 0.0;
      continue;
    }
    const T fj = (T)fu[j];
    T lap = T(0);
    if (a.reg2) {
      // second-order C^T C (13-point): rows centred at j and at its axis neighbours
      const int64_t s3[3] = {g.sx, g.sy, 1};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int64_t s = s3[ax];
        const bool hm = (c >> (2 * ax + 1)) & 1u, hp = (c >> (2 * ax + 2)) & 1u;
        const bool r = hm && hp;
        const bool rm = hm && row2_code(a.code[j - s], ax), rp = hp && row2_code(a.code[j + s], ax);
        if (r) lap += T(-2) * ((T)fu[j - s] - T(2) * fj + (T)fu[j + s]);
        if (rp) lap += fj - T(2) * (T)fu[j + s] + (T)fu[j + 2 * s];
        if (rm) lap += (T)fu[j - 2 * s] - T(2) * (T)fu[j - s] + fj;
      }
    } else {
      if (c & NB_XM) lap += fj - (T)fu[j - g.sx];
      if (c & NB_XP) lap += fj - (T)fu[j + g.sx];
      if (c & NB_YM) lap += fj - (T)fu[j - g.sy];
      if (c & NB_YP) lap += fj - (T)fu[j + g.sy];
      if (c & NB_ZM) lap += fj - (T)fu[j - 1];
      if (c & NB_ZP) lap += fj - (T)fu[j + 1];
    }
    T rho[LMAX], tau[LMAX];
    load_echoes<T, LMAX>(a.dat, g.n, (int)j, a.L, rho, tau);
    T phi, dphi, curv;
    voxel_terms<T, LMAX>(rho, tau, a.L, a.pairs, fj, phi, dphi, curv);
    if (phi_o) phi_o[j] = (double)phi;
    if (dphi_o) dphi_o[j] = (double)dphi;
    if (curv_o) curv_o[j] = (double)curv;
    if (lap_o) lap_o[j] = (double)lap;
  }
}

// Component images at a field map (eq. (wf)): with A = (diag(e^{i 2 pi f t})
// gamma) (x) s_j, A^H A = (gamma^H gamma) sum_c |s_c|^2 and A^H y = gamma^H
// diag(e^{-i 2 pi f t}) z, z_l = sum_c conj(s_c) y_cl, so
//   x = B diag(e^{-i 2 pi f t}) z / sum_c |s_c|^2,  B = (gamma^H gamma)^{-1} gamma^H
// (K x L, from the host).  FP64 in every precision mode; 0 outside the mask or
// where the coil maps vanish.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_components(Geo g, int ncoil, int L, int K, const float2 *__restrict__ y,
                                                        const float2 *__restrict__ sens,
                                                        const uint8_t *__restrict__ code, const double *__restrict__ fu,
                                                        const T *__restrict__ fw, const double *__restrict__ te,
                                                        const double2 *__restrict__ B, float2 *__restrict__ out) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < g.n; j += (int64_t)gridDim.x * kBlock) {
    double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};
    if (code[j] & NB_SELF) {
      double ss = 1.0;
      if (sens) {
        ss = 0.0;
        for (int c = 0; c < ncoil; ++c) {
          const float2 sv = sens[(int64_t)c * g.n + j];
          ss += (double)sv.x * sv.x + (double)sv.y * sv.y;
        }
      }
      if (ss > 0.0) {
        const double fj = fu ? fu[j] : (double)fw[j];
        for (int l = 0; l < L; ++l) {
          double zr = 0.0, zi = 0.0;
          for (int c = 0; c < ncoil; ++c) {
            const float2 yv = y[((int64_t)c * L + l) * g.n + j];
            if (sens) {
              const float2 sv = sens[(int64_t)c * g.n + j];
              zr += (double)sv.x * yv.x + (double)sv.y * yv.y;
              zi += (double)sv.x * yv.y - (double)sv.y * yv.x;
            } else {
              zr += yv.x;
              zi += yv.y;
            }
          }
          // e^{-i 2 pi f t_l} z_l
          double sn, cs;
          sincospi(2.0 * fj * te[l], &sn, &cs);
          const double wr = cs * zr + sn * zi, wi = cs * zi - sn * zr;
          for (int k = 0; k < K; ++k) {
            const double2 b = B[k * L + l];
            xr[k] += b.x * wr - b.y * wi;
            xi[k] += b.x * wi + b.y * wr;
          }
        }
        for (int k = 0; k < K; ++k) {
          xr[k] /= ss;
          xi[k] /= ss;
        }
      }
    }
    for (int k = 0; k < K; ++k) {
      float2 o;
      o.x = (float)xr[k];
      o.y = (float)xi[k];
      out[(int64_t)k * g.n + j] = o;
    }
  }
}

// Conversions between user float64 arrays and the working type.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_work(int64_t n, const double *__restrict__ src, T *dst) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
    dst[j] = (T)src[j];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_work(int64_t n, const T *__restrict__ src, double *dst) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
    dst[j] = (double)src[j];
}

__global__ __launch_bounds__(kBlock) void k_pivots(int64_t n, const double *__restrict__ ipiv, double *piv) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
    piv[j] = ipiv[j] > 0.0 ? 1.0 / ipiv[j] : 0.0;
}

}  // namespace fm
