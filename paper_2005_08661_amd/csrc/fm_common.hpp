// Device-side building blocks shared by the field-map kernels: the scalar
// state carried from kernel to kernel, the mask/neighbour code, deterministic
// FP64 reductions and the per-voxel echo-pair data term.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

constexpr int kBlock = 256;      // threads per block of the streaming kernels
constexpr int kWave = 64;        // CDNA wavefront
#ifndef FM_MAXGRID
#define FM_MAXGRID 1024
#endif
constexpr int kMaxGrid = FM_MAXGRID;  // blocks (hence partial sums) of a streaming pass
constexpr int kMaxK = 4;         // values reduced per kernel

// Neighbour code of a voxel: bit 0 = inside the mask; bits 1..6 = the
// -x, +x, -y, +y, -z, +z neighbour is inside the volume and the mask (only set
// for in-mask voxels).  deg = number of in-mask neighbours.
// Bit 7 marks the black voxels (x+y+z odd) of the red-black ordering.
enum : uint32_t { NB_SELF = 1u, NB_XM = 2u, NB_XP = 4u, NB_YM = 8u, NB_YP = 16u, NB_ZM = 32u, NB_ZP = 64u,
                  NB_BLACK = 128u };

__device__ __forceinline__ int nb_deg(uint32_t c) { return __popc((c >> 1) & 63u); }

// What the partial sums handed from one kernel to the next contain.
enum PartKind : int32_t {
  PK_NONE = 0,   // nothing to consume
  PK_GRAD = 1,   // sum phi, f^T C^T C f, ||g||^2, z_prev^T g
  PK_DOTS_A = 2, // first half of g^T p, g_prev^T p (red-black: black voxels)
  PK_DOTS = 3,   // (rest of) g^T p, g_prev^T p
  PK_DIR = 4,    // z^T C^T C f, ||C z||^2, sum z^2 D
  PK_MLS = 5,    // S1 = z^T dphi(f + alpha z), S2 = sum z^2 d(f + alpha z)
  PK_COUNT = 6,  // in-mask voxel count
  PK_ADJ_INIT = 7, // adjoint CG: ||b||^2 of the right-hand side dL/df
  PK_ADJ_CURV = 8, // adjoint CG: d^T H d
  PK_ADJ_UPD = 9,  // adjoint CG: ||r||^2 after the update
  PK_ADJ_FIN = 10, // adjoint: v^T C^T C fhat
};

// Scalar state of one solve.  Two copies ping-pong along the kernel chain:
// a kernel reads copy q&1 (and the partial sums its predecessor wrote), every
// block derives the same updated scalars, and block 0 writes copy (q+1)&1.
struct State {
  double alpha;     // line-search step
  double mu;        // Polak-Ribiere coefficient
  double gtp;       // g^T p
  double gtp_prev;  // g^T p of the previous iteration
  double gpp;       // g_prev^T p
  double acc0, acc1;// first halves of g^T p, g_prev^T p (red-black)
  double zpg;       // z_prev^T g
  double ztg;       // z^T g
  double A;         // z^T C^T C f
  double B;         // ||C z||^2
  double cost;      // Psi at the start of the iteration
  double gnorm2;    // ||g||^2
  double nmask;     // in-mask voxels
  int32_t iter;     // current iteration
  int32_t restart;  // direction reset in the current iteration
  int32_t ls_left;  // line-search steps still to apply in this iteration
  int32_t kind;     // PartKind of the incoming partial sums
  int32_t nparts;   // number of incoming partial blocks
  int32_t nmls;     // line-search steps per iteration
  int32_t trace_cap;// rows of the trace (iterations recorded)
  int32_t ls_done;  // line search of this iteration stopped (zero curvature)
  // conjugate gradients of the implicit adjoint (H v = dL/df); the
  // preconditioner passes leave r^T M^{-1} r in gtp
  double cg_rho;      // r^T z of the current CG iteration
  double cg_rho_prev; // r^T z of the previous one
  double cg_alpha;    // CG step
  double cg_b2;       // ||dL/df||^2
  double cg_r2;       // ||r||^2
  double cg_rtol2;    // squared relative tolerance
  double cg_dbeta;    // dL/dbeta = -v^T C^T C fhat
  int32_t cg_it;      // CG updates applied
  int32_t cg_done;    // converged (or broken down): later passes are no-ops
};

// Per echo-pair constants (m < n): weight factor 2|Gamma_mn|, phase of
// Gamma_mn in turns, dt = t_m - t_n and 2*pi*dt.
template <typename T>
struct PairC {
  T w;
  T g;
  T dt;
  T d2pi;
  int32_t m, n;
  int32_t pad[2];
};

// ---------------------------------------------------------------------------
// sin(x)/x and cos(x) for |x| <= pi/2 as polynomials in x^2 with constant
// term 1.  FP32: least-squares fits over Chebyshev nodes of [-pi/2, pi/2],
// through x^8 (sin) and x^10 (cos), one term fewer each than the Taylor forms
// of the same accuracy (errors 2e-8 and 3e-9 with the coefficients rounded to
// FP32, below the evaluation's own rounding).  FP64: the Taylor series through
// x^20 (remainder <= 2e-17), coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!.
// No division and no special case at x = 0.
__device__ __forceinline__ void sinx_cos(float x, float &sx, float &c) {
  const float x2 = x * x;
  sx = 1.f + x2 * (-1.666665971e-01f + x2 * (8.333084174e-03f + x2 * (-1.981087116e-04f + x2 * 2.608453997e-06f)));
  c = 1.f + x2 * (-0.5f + x2 * (4.166664183e-02f + x2 * (-1.388839795e-03f + x2 * (2.476165537e-05f +
      x2 * -2.607347938e-07f))));
}

__device__ __forceinline__ void sinx_cos(double x, double &sx, double &c) {
  const double x2 = x * x;
  sx = 1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 + x2 * (1.0 / 362880.0 +
       x2 * (-1.0 / 39916800.0 + x2 * (1.0 / 6227020800.0 + x2 * (-1.0 / 1307674368000.0 +
       x2 * (1.0 / 355687428096000.0 + x2 * (-1.0 / 121645100408832000.0 +
       x2 * (1.0 / 51090942171709440000.0))))))))));
  c = 1.0 + x2 * (-0.5 + x2 * (1.0 / 24.0 + x2 * (-1.0 / 720.0 + x2 * (1.0 / 40320.0 +
      x2 * (-1.0 / 3628800.0 + x2 * (1.0 / 479001600.0 + x2 * (-1.0 / 87178291200.0 +
      x2 * (1.0 / 20922789888000.0 + x2 * (-1.0 / 6402373705728000.0 +
      x2 * (1.0 / 2432902008176640000.0))))))))));
}

__device__ __forceinline__ float rint_t(float x) { return rintf(x); }
__device__ __forceinline__ double rint_t(double x) { return rint(x); }

// Per-voxel data term at field value f (Hz) over the echo pairs.  The phase
// of pair (m,n) is 2 pi xi with xi = angle(Gamma_mn)/2pi + tau_n - tau_m + f dt
// (turns).  With h = xi - rint(xi) in [-1/2, 1/2] (the wrap of reading R4),
// x = pi h, sx = sin(x)/x, s = x sx and c = cos(x):
//   1 - cos(2 pi xi) = 2 s^2,   sin(2 pi xi) = 2 s c,   sinc(2 pi h) = sx c.
template <typename T, int LMAX>
__device__ __forceinline__ void voxel_terms(const T (&rho)[LMAX], const T (&tau)[LMAX], int L,
                                            const PairC<T> *__restrict__ pc, T f, T &phi, T &dphi,
                                            T &curv) {
  T c0 = 0, c1 = 0, c2 = 0;
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
        const T wd = w * P.d2pi;
        c0 += w * (T(2) * s * s);
        c1 += wd * (T(2) * s * c);
        c2 += wd * P.d2pi * (sx * c);
        ++q;
      }
    }
  }
  phi = c0;
  dphi = c1;
  curv = c2;
}

// The same terms from per-pair values that do not change during a solve: the
// weight w_q = 2|Gamma_mn| rho_m rho_n and the phase offset
// xg_q = angle(Gamma_mn)/2pi + tau_n - tau_m (turns), formed once with the
// expressions voxel_terms uses (pair_consts), so the results are the same bits.
template <typename T, int L>
__device__ __forceinline__ void pair_consts(const T (&rho)[L], const T (&tau)[L], const PairC<T> *__restrict__ pc,
                                            T (&w)[L * (L - 1) / 2], T (&xg)[L * (L - 1) / 2]) {
  int q = 0;
#pragma unroll
  for (int m = 0; m < L; ++m) {
#pragma unroll
    for (int n = m + 1; n < L; ++n, ++q) {
      const PairC<T> P = pc[q];
      w[q] = P.w * rho[m] * rho[n];
      xg[q] = P.g + (tau[n] - tau[m]);
    }
  }
}

template <typename T, int NP>
__device__ __forceinline__ void voxel_terms_pc(const T (&w)[NP], const T (&xg)[NP], const PairC<T> *__restrict__ pc,
                                               T f, T &phi, T &dphi, T &curv) {
  T c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const PairC<T> P = pc[q];
    const T xi = xg[q] + f * P.dt;
    const T x = T(3.14159265358979323846) * (xi - rint_t(xi));
    T sx, c;
    sinx_cos(x, sx, c);
    const T s = x * sx;
    const T wd = w[q] * P.d2pi;
    c0 += w[q] * (T(2) * s * s);
    c1 += wd * (T(2) * s * c);
    c2 += wd * P.d2pi * (sx * c);
  }
  phi = c0;
  dphi = c1;
  curv = c2;
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions without atomics.  A kernel reduces its K
// values per block and stores one partial per block; the next kernel in the
// stream has every block sum all partials in the same fixed order, so every
// block obtains bit-identical totals (kernel boundaries order the accesses).
// DPP move of a double (both halves) with the given control; lanes whose
// source is outside the row, or that the masks disable, read 0.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, BANK_MASK, true);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, BANK_MASK, true);
  return __hiloint2double(hi2, lo2);
}

// Wavefront sum with DPP row shifts and row broadcasts: lane 15 of each row
// collects its row, the broadcasts fold rows 0..3 into lane 63, which is then
// read by every lane.  Fixed order, hence deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  double t = v + dpp_d<0x111>(v);    // row_shr:1
  t = t + dpp_d<0x112>(v);           // row_shr:2
  t = t + dpp_d<0x113>(v);           // row_shr:3
  t = t + dpp_d<0x114, 0xf, 0xe>(t); // row_shr:4, banks 1-3
  t = t + dpp_d<0x118, 0xf, 0xc>(t); // row_shr:8, banks 2-3
  t = t + dpp_d<0x142, 0xa, 0xf>(t); // row_bcast:15 into rows 1 and 3
  t = t + dpp_d<0x143, 0xc, 0xf>(t); // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(t), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(t), 63);
  return __hiloint2double(hi, lo);
}

template <int K>
__device__ __forceinline__ void wave_reduce(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
}

// Block-wide sum (blockDim.x == NT); result valid in every thread.
template <int K, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
  __shared__ double red[K][NT / kWave];
  wave_reduce<K>(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) s += red[k][w];
    v[k] = s;
  }
  __syncthreads();
}

// Agent-coherent loads and stores (data exchanged between workgroups of one
// kernel, possibly on different XCDs).
template <typename T>
__device__ __forceinline__ T ld_coh(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Store the K partial sums of unit idx (of count units; a unit is a
// workgroup, or a tile of the wavefront sweep).  Layout: value k of unit u at
// pout[k * count + u] (one row per value), so a consumer reads only the rows
// that the producer wrote.
template <int K, int NT = kBlock>
__device__ __forceinline__ void store_partials_at(double (&v)[K], int idx, int count, double *__restrict__ pout) {
  static_assert(K <= kMaxK, "too many reduced values");
  block_sum<K, NT>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) pout[(size_t)k * count + idx] = v[k];
  }
}

template <int K, int NT = kBlock>
__device__ __forceinline__ void store_partials(double (&v)[K], double *__restrict__ pout) {
  store_partials_at<K, NT>(v, (int)blockIdx.x, (int)gridDim.x, pout);
}

// Sum the first nvals rows of the predecessor's nparts partials; every thread
// gets the totals.  KR (>= nvals) rows are loaded unconditionally (every row
// index is inside the buffer) and masked afterwards, and the block loop is
// unrolled over the usual partial count, so all loads are in flight at once.
template <int KR, int NT = kBlock>
__device__ __forceinline__ void sum_partials(const double *__restrict__ pin, int nparts, int nvals,
                                             double (&tot)[kMaxK], int rowstride) {
  static_assert(KR <= kMaxK, "too many reduced values");
  constexpr int U = (kMaxGrid + NT - 1) / NT < 4 ? (kMaxGrid + NT - 1) / NT : 4;
  double acc[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) acc[k] = 0.0;
  for (int b0 = 0; b0 < nparts; b0 += U * NT) {
    double x[U][KR];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * NT + (int)threadIdx.x;
      const int bb = b < nparts ? b : 0;
#pragma unroll
      for (int k = 0; k < KR; ++k) x[u][k] = pin[(size_t)k * rowstride + bb];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = b0 + u * NT + (int)threadIdx.x < nparts;
#pragma unroll
      for (int k = 0; k < KR; ++k) acc[k] += (ok && k < nvals) ? x[u][k] : 0.0;
    }
  }
  block_sum<KR, NT>(acc);
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) tot[k] = k < KR ? acc[k < KR ? k : 0] : 0.0;
}

__device__ __forceinline__ void set_status(int32_t *status, int code) { atomicCAS(status, 0, code); }

// Line-search setup from A = z^T C^T C f, B = ||C z||^2 and d0 = sum z^2 D:
// the first step from alpha = 0 is alpha = -z^T g / (d0 + beta B).
__device__ __forceinline__ void start_line_search(State &s, double A, double B, double d0, double beta,
                                                  double *trace, bool leader) {
  const bool w = (leader && threadIdx.x == 0);
  s.A = A;
  s.B = B;
  const double den = d0 + beta * B;
  s.ls_left = s.nmls - 1;  // line-search passes still to consume
  s.ls_done = 0;
  if (den > 0.0) {
    s.alpha = -s.ztg / den;
  } else {
    s.alpha = 0.0;
    s.ls_done = 1;
  }
  if (w && s.iter < s.trace_cap) trace[(size_t)s.iter * 8 + 6] = B;
}

// Apply the incoming partial sums to the scalar state (identically in every
// block).  trace (row-major [trace_cap+1][8]) is written by block 0 only.
__device__ __forceinline__ void consume(State &s, const double (&t)[kMaxK], double beta, double *trace,
                                        int32_t *status, bool leader) {
  const bool w = (leader && threadIdx.x == 0);
  switch (s.kind) {
    case PK_GRAD: {
      s.cost = t[0] + 0.5 * beta * t[1];
      s.gnorm2 = t[2];
      s.zpg = t[3];
      if (w && s.iter <= s.trace_cap) trace[(size_t)s.iter * 8 + 0] = s.cost;
      if (w && !(isfinite(s.cost) && isfinite(s.gnorm2))) set_status(status, 6);
      break;
    }
    case PK_DOTS_A: {
      s.acc0 = t[0];
      s.acc1 = t[1];
      break;
    }
    case PK_DOTS: {
      // Polak-Ribiere conjugacy with restart (readings R6, R7)
      const double gtp = s.acc0 + t[0];
      const double gpp = s.acc1 + t[1];
      double mu = (s.gtp_prev != 0.0) ? (gtp - gpp) / s.gtp_prev : 0.0;
      double ztg = -gtp + mu * s.zpg;
      int restart = 0;
      if (ztg >= 0.0) {
        mu = 0.0;
        ztg = -gtp;
        restart = 1;
      }
      s.gtp = gtp;
      s.gpp = gpp;
      s.mu = mu;
      s.ztg = ztg;
      s.restart = restart;
      s.acc0 = 0.0;
      s.acc1 = 0.0;
      if (w && s.iter < s.trace_cap) {
        double *r = trace + (size_t)s.iter * 8;
        r[1] = gtp;
        r[2] = mu;
        r[3] = (double)restart;
        r[5] = ztg;
        r[7] = s.gnorm2;
      }
      break;
    }
    case PK_DIR: {
      start_line_search(s, t[0], t[1], t[2], beta, trace, leader);
      break;
    }
    case PK_MLS: {
      // eq. (ls_update): alpha <- alpha - (S1 + beta A + alpha beta B) / (S2 + beta B)
      if (!s.ls_done) {
        const double den = t[1] + beta * s.B;
        if (den > 0.0) {
          s.alpha = s.alpha - (t[0] + beta * s.A + s.alpha * beta * s.B) / den;
        } else {
          s.ls_done = 1;
        }
      }
      s.ls_left -= 1;
      break;
    }
    case PK_ADJ_INIT:
    case PK_ADJ_UPD: {
      if (s.kind == PK_ADJ_INIT) s.cg_b2 = t[0];
      if (!s.cg_done) {
        s.cg_r2 = t[0];
        if (!isfinite(t[0])) {
          s.cg_done = 1;
          if (w) set_status(status, 6);
        } else if (s.cg_r2 <= s.cg_rtol2 * s.cg_b2) {
          s.cg_done = 1;
        }
      }
      break;
    }
    case PK_ADJ_CURV: {
      if (!s.cg_done) {
        if (t[0] > 0.0) {
          s.cg_alpha = s.cg_rho / t[0];
          s.cg_rho_prev = s.cg_rho;
          s.cg_it += 1;
        } else {
          // the true Hessian is not positive definite along d
          s.cg_alpha = 0.0;
          s.cg_done = 1;
          if (w) set_status(status, 5);
        }
      }
      break;
    }
    case PK_ADJ_FIN: {
      s.cg_dbeta = -t[0];
      break;
    }
    default:
      break;
  }
  // The iteration ends once its last line-search pass has been consumed.
  if ((s.kind == PK_DIR || s.kind == PK_MLS) && s.ls_left == 0) {
    if (w && s.iter < s.trace_cap) trace[(size_t)s.iter * 8 + 4] = s.alpha;
    if (w && !isfinite(s.alpha)) set_status(status, 6);
    s.gtp_prev = s.gtp;
    s.iter += 1;
  }
  s.kind = PK_NONE;
  s.nparts = 0;
}

// Iteration index after the incoming partials are consumed, known before the
// partials are summed (lets a kernel issue its loads first).
__device__ __forceinline__ int iter_after(const State &s) {
  if (s.kind == PK_DIR) return s.iter + (s.nmls == 1 ? 1 : 0);
  if (s.kind == PK_MLS) return s.iter + (s.ls_left == 1 ? 1 : 0);
  return s.iter;
}

// Common prologue: load the incoming state and sum the incoming partials
// (their count nparts_in is fixed by the launch sequence, so both loads are
// issued together), then apply them.  Returns the updated state (identical in
// every block).
// KR bounds the number of values the kernel may consume (nvals_in <= KR).
// The partials of this consumer are pin[k * rowstride + b], b < nparts_in
// (rowstride < 0: rowstride = nparts_in).  leader: the workgroup that writes
// the trace and the outgoing state (the first one of its volume).
template <int NT = kBlock, int KR = 4>
__device__ __forceinline__ State take_state(const State *__restrict__ sin, const double *__restrict__ pin,
                                            int nparts_in, int nvals_in, double beta, double *trace,
                                            int32_t *status, int rowstride = -1, bool leader = blockIdx.x == 0) {
  State s = *sin;
  double t[kMaxK];
  sum_partials<KR, NT>(pin, nparts_in, nvals_in, t, rowstride < 0 ? nparts_in : rowstride);
  if (s.kind != PK_NONE) {
    if ((s.nparts != nparts_in || nvals_in > KR) && leader && threadIdx.x == 0) set_status(status, 7);
    consume(s, t, beta, trace, status, leader);
  }
  return s;
}

// Epilogue: the leader publishes the state with the kind of partials it leaves.
__device__ __forceinline__ void put_state(State s, State *__restrict__ sout, int kind, int nparts,
                                          bool leader = blockIdx.x == 0) {
  if (leader && threadIdx.x == 0) {
    s.kind = kind;
    s.nparts = nparts;
    *sout = s;
  }
}

}  // namespace fm
