// Host side of the C ABI declared in include/fmap.h: parameter validation,
// plan and workspace management, the kernel chain of one NCG iteration and
// the HIP graph that replays the whole iteration loop.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <type_traits>
#include <vector>

#include "../../include/fmap.h"
#include "fm_kernels.hpp"
#include "fm_stream.hpp"
#include "fm_natural.hpp"
#include "fm_adjoint.hpp"
#include "fm_resident.hpp"
#include "fm_order2.hpp"
#include "fm_ict.hpp"
#include "fm_tile.hpp"

using fm::kBlock;
using fm::kMaxGrid;
using fm::kMaxK;

namespace {

thread_local std::string g_last_error;

fm_status fail(fm_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

#define FM_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(FM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define FM_LAUNCH_CHECK()                                                                 \
  do {                                                                                    \
    hipError_t e_ = hipGetLastError();                                                    \
    if (e_ != hipSuccess) return fail(FM_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct fm_plan {
  fm_params prm;
  int device = 0;
  int64_t n = 0;
  fm::Geo geo{};
  bool mix = false;
  int lmax = 4;
  int npairs = 0;
  int grid = 1;   // blocks of the kBlock-thread kernels
  int sgrid = 1;  // blocks of the streaming iteration passes (kNT threads)
  size_t tsize = 8;  // bytes of the working type
  // device workspace
  void *dat = nullptr;
  uint8_t *code = nullptr;
  void *F[2] = {nullptr, nullptr};
  void *Z[2] = {nullptr, nullptr};
  void *G[2] = {nullptr, nullptr};
  void *D = nullptr, *X = nullptr, *P = nullptr;
  void *X2 = nullptr;          // three-colour IC(0): y' = L^{-1} g_prev of colour 1
  uint8_t *rdiag = nullptr;    // three-colour IC(0): diag(C^T C) of the second-order operator
  // three-colour IC(0): G, D, P, ipiv, X, X2, rdiag and a copy of the codes (ccode) are kept
  // colour-major, cm_elems elements each (three colour blocks with two padding x-planes)
  bool cm = false;
  uint8_t *ccode = nullptr;
  int64_t cm_elems = 0;
  void *Pv = nullptr, *Dv = nullptr;  // voxel-order copies of p and D for the direction pass
  double *ipiv = nullptr;
  double *hinv = nullptr;
  fm::State *S = nullptr;      // two ping-pong state copies
  double *part = nullptr;      // two ping-pong partial-sum buffers [part_rows][kMaxK]
  size_t part_rows = kMaxGrid;
  fm::Wavefront wf{};          // natural-order sweep: tiles, tickets, progress
  double *setup_part = nullptr;
  double *nmask = nullptr;
  int32_t *status = nullptr;
  double *trace = nullptr;
  void *pairs = nullptr;
  void *pairs_d = nullptr;
  double *comp_tab = nullptr;  // eq. (wf): te [L], then B = (gamma^H gamma)^{-1} gamma^H [K][L] complex
  int ncomp = 1;
  double *gabs = nullptr;
  double *rho = nullptr;
  double *f0buf = nullptr;
  double *wf_tmp = nullptr;  // water-fat init: swept map and 3 CG vectors
  bool setup_done = false;
  bool solved = false;
  // position in the kernel chain: launch q reads S[q&1], writes S[(q+1)&1];
  // iteration index and partial-sum count at the current position
  uint64_t q = 0;
  int64_t iter_host = 0;
  int last_nparts = 0;
  int last_nvals = 0;   // values per partial block at the current position
  // device allocations (freed with the plan); stencil-read arrays are
  // padded by pad elements on both sides
  std::vector<void *> bases;
  int64_t pad = 0;
  // graphs of the iteration loop keyed by (chain parity, iterations)
  hipStream_t cap_stream = nullptr;
  std::map<std::vector<int64_t>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  // implicit adjoint workspace (allocated by the first fm_adjoint call)
  bool adj_ready = false;
  void *aR = nullptr, *aZ = nullptr, *aX = nullptr, *aDc = nullptr, *aH = nullptr, *aV = nullptr;
  void *aDd[2] = {nullptr, nullptr};
  double *a_hinv = nullptr, *a_ipiv = nullptr, *a_part = nullptr;
  fm::State *aS = nullptr;
  int32_t *a_status = nullptr;
  // resident schedule (one launch for many iterations)
  bool reg2 = false;           // second-order regulariser
  int32_t sched = FM_SCHED_AUTO;
  bool res_ok = false;         // the plan qualifies (MIX, red-black IC(0), <= 4 echoes, tiles fit)
  bool res_auto = false;       // and FM_SCHED_AUTO takes it (large enough volume)
  fm::ResTile res_tile{};
  int res_grid = 0;
  double *res_part = nullptr;  // [2][kMaxK][res_grid]
  uint32_t *res_bar = nullptr; // barrier counters
  // IC_t (incomplete Cholesky with a drop tolerance, natural order, bounded fill)
  bool ict = false;
  int ict_noff = 0, ict_nlev = 0, ict_kcol = 0, ict_blocks = 0;
  double *ict_lo = nullptr, *ict_ld = nullptr, *ict_y = nullptr, *ict_pd = nullptr;
  double *ict_hmax = nullptr, *ict_hpart = nullptr;
};

namespace {

// Gamma = gamma (gamma^H gamma)^{-1} gamma^H (Sec. II eq. (gamma)).
std::vector<std::complex<double>> make_gamma(const fm_params &p) {
  const int L = p.necho;
  std::vector<std::complex<double>> G((size_t)L * L);
  if (p.model == FM_FIELDMAP) {
    for (auto &v : G) v = 1.0 / L;
    return G;
  }
  const double two_pi = 6.283185307179586476925286766559;
  std::vector<std::complex<double>> c(L);
  for (int l = 0; l < L; ++l) {
    std::complex<double> s = 0.0;
    for (int q = 0; q < p.npeak; ++q) s += p.fat_amp[q] * std::polar(1.0, two_pi * p.fat_hz[q] * p.te[l]);
    c[l] = s;
  }
  // normal matrix N = [[L, sum c], [sum conj c, sum |c|^2]] and its inverse
  std::complex<double> sc = 0.0;
  double cc = 0.0;
  for (int l = 0; l < L; ++l) {
    sc += c[l];
    cc += std::norm(c[l]);
  }
  const double det = L * cc - std::norm(sc);
  const std::complex<double> i00 = cc / det, i01 = -sc / det, i10 = -std::conj(sc) / det, i11 = (double)L / det;
  for (int m = 0; m < L; ++m)
    for (int n = 0; n < L; ++n)
      G[(size_t)m * L + n] = i00 + i01 * std::conj(c[n]) + c[m] * i10 + c[m] * i11 * std::conj(c[n]);
  return G;
}

// B = (gamma^H gamma)^{-1} gamma^H (K x L, row-major, interleaved complex):
// gamma = 1 (field map, K = 1) or [1, c] (water-fat, K = 2).
std::vector<double> make_component_matrix(const fm_params &p, int *K) {
  const int L = p.necho;
  const double two_pi = 6.283185307179586476925286766559;
  std::vector<double> out;
  if (p.model == FM_FIELDMAP) {
    *K = 1;
    for (int l = 0; l < L; ++l) {
      out.push_back(1.0 / L);
      out.push_back(0.0);
    }
    return out;
  }
  *K = 2;
  std::vector<std::complex<double>> c(L);
  for (int l = 0; l < L; ++l) {
    std::complex<double> v = 0.0;
    for (int q = 0; q < p.npeak; ++q) v += p.fat_amp[q] * std::polar(1.0, two_pi * p.fat_hz[q] * p.te[l]);
    c[l] = v;
  }
  std::complex<double> sc = 0.0;
  double cc = 0.0;
  for (int l = 0; l < L; ++l) {
    sc += c[l];
    cc += std::norm(c[l]);
  }
  const double det = L * cc - std::norm(sc);
  // N^{-1} = [[cc, -sc], [-conj(sc), L]] / det;  B = N^{-1} [1 ... 1; conj(c)]
  const std::complex<double> i00 = cc / det, i01 = -sc / det, i10 = -std::conj(sc) / det, i11 = (double)L / det;
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l < L; ++l) {
      const std::complex<double> v = (k == 0) ? i00 + i01 * std::conj(c[l]) : i10 + i11 * std::conj(c[l]);
      out.push_back(v.real());
      out.push_back(v.imag());
    }
  return out;
}

// The setup kernel for an echo bucket and model.
template <typename T>
using SetupKernel = void (*)(fm::SetupArgs<T>);
template <typename T>
SetupKernel<T> setup_kernel(int lmax, bool wf, int necho) {
  if (wf && necho == 6) return fm::k_setup<T, 6, true>;  // the water-fat echo count of the paper's experiments
  if (wf) return lmax <= 4 ? fm::k_setup<T, 4, true> : (lmax <= 8 ? fm::k_setup<T, 8, true> : fm::k_setup<T, 16, true>);
  // the field-map model with 2-4 echoes: the exact echo count, so no echo slot is loaded or summed for nothing
  if (necho == 2) return fm::k_setup<T, 2, false>;
  if (necho == 3) return fm::k_setup<T, 3, false>;
  return lmax <= 4 ? fm::k_setup<T, 4, false> : (lmax <= 8 ? fm::k_setup<T, 8, false> : fm::k_setup<T, 16, false>);
}

template <typename T>
std::vector<fm::PairC<T>> make_pairs(const fm_params &p, const std::vector<std::complex<double>> &G) {
  std::vector<fm::PairC<T>> out;
  const double two_pi = 6.283185307179586476925286766559;
  for (int m = 0; m < p.necho; ++m)
    for (int n = m + 1; n < p.necho; ++n) {
      fm::PairC<T> q{};
      const auto g = G[(size_t)m * p.necho + n];
      q.w = (T)(2.0 * std::abs(g));
      q.g = (T)(std::arg(g) / two_pi);
      q.dt = (T)(p.te[m] - p.te[n]);
      q.d2pi = (T)(two_pi * (p.te[m] - p.te[n]));
      q.m = m;
      q.n = n;
      out.push_back(q);
    }
  return out;
}

// Arguments of chain launch number q (state and partial-sum slots by parity).
template <typename T>
fm::IterArgs<T> iter_args(fm_plan *p, uint64_t q) {
  fm::IterArgs<T> a{};
  a.geo = p->geo;
  a.L = p->prm.necho;
  a.beta = p->prm.beta;
  a.dat = (const fm::T2<T> *)p->dat;
  a.code = p->code;
  a.pairs = (const fm::PairC<T> *)p->pairs;
  for (int i = 0; i < 2; ++i) {
    a.F[i] = (T *)p->F[i];
    a.Z[i] = (T *)p->Z[i];
    a.G[i] = (T *)p->G[i];
  }
  a.D = (T *)p->D;
  a.X = (T *)p->X;
  a.X2 = (T *)p->X2;
  a.P = (T *)p->P;
  a.rdiag = p->rdiag;
  a.ccode = p->ccode;
  a.cm = p->cm ? 1 : 0;
  a.Pv = (T *)p->Pv;
  a.Dv = (T *)p->Dv;
  a.ipiv = p->ipiv;
  a.hinv = p->hinv;
  // the pair-mapped passes (even column length) keep 1/h of red and p of black voxels at the pair's index
  a.write_hinv = (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_REDBLACK) ? (p->geo.nz % 2 ? 1 : 2) : 0;
  a.store_piv = 0;
  a.par = (int32_t)(p->iter_host & 1);
  a.nparts_in = p->last_nparts;
  a.nvals_in = p->last_nvals;
  a.sin = p->S + (q & 1);
  a.sout = p->S + ((q + 1) & 1);
  a.pin = p->part + (size_t)(q & 1) * p->part_rows * kMaxK;
  a.pout = p->part + (size_t)((q + 1) & 1) * p->part_rows * kMaxK;
  a.status = p->status;
  a.trace = p->trace;
  a.fout = nullptr;
  a.final_pass = 0;
  a.reg2 = p->reg2 ? 1 : 0;
  return a;
}

// Optional per-launch event recorder (measurement path only): the events are
// attached to the dispatch itself (hipExtLaunchKernelGGL), so they bracket the
// kernel's execution without extra packets in between.
struct Recorder {
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
  hipError_t err = hipSuccess;
  void pair(int c, hipEvent_t *e0, hipEvent_t *e1) {
    *e0 = *e1 = nullptr;
    if (err == hipSuccess) err = hipEventCreate(e0);
    if (err == hipSuccess) err = hipEventCreate(e1);
    ev.push_back(*e0);
    ev.push_back(*e1);
    cls.push_back(c);
  }
  ~Recorder() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

#define FM_LAUNCH(cls, kernel, grid, block, s, ...)                                   \
  do {                                                                                \
    if (rec) {                                                                        \
      hipEvent_t e0_, e1_;                                                            \
      rec->pair(cls, &e0_, &e1_);                                                     \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0_, e1_, 0, __VA_ARGS__);     \
    } else {                                                                          \
      hipLaunchKernelGGL(kernel, grid, block, 0, s, __VA_ARGS__);                     \
    }                                                                                 \
  } while (0)

// Preconditioner step p = P^{-1} g (g from gsrc, or G[iter&1] if null),
// leaving the dot products g^T p and g_prev^T p as partial sums.
void set_parts(fm_plan *p, int nparts, int nvals) {
  p->last_nparts = nparts;
  p->last_nvals = nvals;
}

// IC_t: H_max, then the factorisation with the forward solve level by level,
// then the backward solve in reverse level order (outside the state chain).
template <typename T, int LEVEL>
fm_status enqueue_ict(fm_plan *p, const T *g, hipStream_t s, Recorder *rec) {
  fm::IctArgs<T> a{};
  a.geo = p->geo;
  a.beta = p->prm.beta;
  a.factor = p->prm.ict_factor;
  a.hmax = p->ict_hmax;
  a.code = p->code;
  a.D = (const T *)p->D;
  a.kcol = p->ict_kcol;
  a.lo = p->ict_lo;
  a.ld = p->ict_ld;
  a.y = p->ict_y;
  a.pd = p->ict_pd;
  a.P = (T *)p->P;
  a.status = p->status;
  FM_LAUNCH(FM_K_PRECOND_A, fm::k_ict_hmax<T>, dim3(p->grid), dim3(kBlock), s, p->geo, (const uint8_t *)p->code,
            (const T *)p->D, p->prm.beta, p->ict_hpart);
  FM_LAUNCH_CHECK();
  FM_LAUNCH(FM_K_PRECOND_A, fm::k_ict_hmax_fin, dim3(1), dim3(kBlock), s, (const double *)p->ict_hpart, p->grid,
            p->ict_hmax);
  FM_LAUNCH_CHECK();
  for (int lv = 0; lv < p->ict_nlev; ++lv)
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_ict_fwd<T, LEVEL>), dim3(p->ict_blocks), dim3(fm::kIctNT), s, a, g, lv);
  FM_LAUNCH_CHECK();
  for (int lv = p->ict_nlev - 1; lv >= 0; --lv)
    FM_LAUNCH(FM_K_PRECOND_B, (fm::k_ict_bwd<T, LEVEL>), dim3(p->ict_blocks), dim3(fm::kIctNT), s, a, lv);
  FM_LAUNCH_CHECK();
  return FM_OK;
}

template <typename T>
fm_status enqueue_precond(fm_plan *p, const T *gsrc, hipStream_t s, Recorder *rec = nullptr) {
  auto pargs = [&](fm_plan *pp, uint64_t q) {
    fm::IterArgs<T> a = iter_args<T>(pp, q);
    a.store_piv = gsrc ? 1 : 0;  // the standalone call reports the pivots
    return a;
  };
  if (p->prm.precond == FM_PRECOND_ICT) {
    const T *g = gsrc ? gsrc : (const T *)p->G[p->iter_host & 1];
    fm_status st = p->prm.ict_level == 0 ? enqueue_ict<T, 0>(p, g, s, rec)
                   : (p->prm.ict_level == 1 ? enqueue_ict<T, 1>(p, g, s, rec) : enqueue_ict<T, 2>(p, g, s, rec));
    if (st) return st;
    FM_LAUNCH(FM_K_DOTS, fm::k_ict_dots<T>, dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++),
              (const double *)p->ict_pd, gsrc);
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
  } else if (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_COLOR3) {
    // second-order C: forward colours 0-1, forward colour 2 (+ its p), backward colours 1, 0
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_ic3_fwd1<T>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc);
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_ic3_fwd2<T>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc);
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
    FM_LAUNCH(FM_K_PRECOND_B, (fm::k_ic3_bwd1<T>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++));
    FM_LAUNCH_CHECK();
    set_parts(p, 0, 0);
    FM_LAUNCH(FM_K_PRECOND_B, (fm::k_ic3_bwd0<T>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc);
    FM_LAUNCH_CHECK();
    set_parts(p, 0, 0);
  } else if (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_BLOCKRB) {
    // block red-black: forward colour 0, colour 1; backward colour 1, colour 0 (a volume of one
    // tile column and row has no colour-1 tile)
    const fm::Wavefront &w = p->wf;
    FM_LAUNCH(FM_K_PRECOND_A, fm::k_icb_fwd<T>, dim3(w.nblk[0]), dim3(64), s, pargs(p, p->q++), w, gsrc, 0);
    FM_LAUNCH_CHECK();
    set_parts(p, 0, 0);
    if (w.nblk[1] > 0) {
      FM_LAUNCH(FM_K_PRECOND_A, fm::k_icb_fwd<T>, dim3(w.nblk[1]), dim3(64), s, pargs(p, p->q++), w, gsrc, 1);
      FM_LAUNCH_CHECK();
      FM_LAUNCH(FM_K_PRECOND_B, fm::k_icb_bwd<T>, dim3(w.nblk[1]), dim3(64), s, pargs(p, p->q++), w, gsrc, 1);
      FM_LAUNCH_CHECK();
      set_parts(p, w.nblk[1], 2);
    }
    FM_LAUNCH(FM_K_PRECOND_B, fm::k_icb_bwd<T>, dim3(w.nblk[0]), dim3(64), s, pargs(p, p->q++), w, gsrc, 0);
    FM_LAUNCH_CHECK();
    set_parts(p, w.nblk[0], 2);
  } else if (p->prm.precond == FM_PRECOND_IC0) {
    if (p->prm.ordering == FM_ORDER_NATURAL) {
      FM_LAUNCH(FM_K_PRECOND_A, fm::k_ic_fwd_wave<T>, dim3(p->wf.ntiles), dim3(64), s, pargs(p, p->q++), p->wf, gsrc);
      FM_LAUNCH_CHECK();
      set_parts(p, 0, 0);
      FM_LAUNCH(FM_K_PRECOND_B, fm::k_ic_bwd_wave<T>, dim3(p->wf.ntiles), dim3(64), s, pargs(p, p->q++), p->wf, gsrc);
      FM_LAUNCH_CHECK();
      set_parts(p, p->wf.ntiles, 2);
    } else {
      FM_LAUNCH(FM_K_PRECOND_A, (fm::k_rb_black<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc);
      FM_LAUNCH_CHECK();
      set_parts(p, p->sgrid, 2);
      FM_LAUNCH(FM_K_PRECOND_B, (fm::k_rb_red<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc);
      FM_LAUNCH_CHECK();
      set_parts(p, p->sgrid, 2);
    }
  } else if (p->reg2) {
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_diag2<T>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc,
              p->prm.precond == FM_PRECOND_NONE ? 1 : 0);
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
  } else {
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_diag<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, pargs(p, p->q++), gsrc,
                       p->prm.precond == FM_PRECOND_NONE ? 1 : 0);
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
  }
  return FM_OK;
}

// Launches per iteration (must match enqueue_iteration).
uint64_t launches_per_iteration(const fm_plan *p) {
  // preconditioner passes + direction; red-black IC(0) forms the direction in its red pass
  uint64_t precond_dir = 2;
  if (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_NATURAL) precond_dir = 3;
  if (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_COLOR3) precond_dir = 5;
  if (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_BLOCKRB) precond_dir = p->wf.nblk[1] > 0 ? 5 : 3;
  return 1 + precond_dir + (uint64_t)(p->prm.nmls - 1);
}

bool fused_red_dir(const fm_plan *p) {
  return p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_REDBLACK;
}

// Values per partial block left by the last pass of an iteration.
int tail_nvals(const fm_plan *p) { return p->prm.nmls > 1 ? 2 : 3; }

#ifndef FM_TILE_XCMIN
#define FM_TILE_XCMIN 4
#endif

// Plane-march shape of the tiled red-black passes: strips of ty columns (all
// pair slots of a workgroup on one plane), runs of at least FM_TILE_XCMIN
// planes, lengthened until the grid fits the partial-sum rows.  grid 0 where
// the tile does not apply (odd or long columns).
fm::TileShape tile_shape(const fm::Geo &g) {
  fm::TileShape t{};
  if (g.nz % 2 != 0 || g.nz > fm::kTileMaxNz) return t;
  const int nzp = g.nz / 2;
  t.ty = std::min(fm::kTileSlots / nzp, g.ny);
  t.nyt = (g.ny + t.ty - 1) / t.ty;
  if (t.nyt > kMaxGrid) return fm::TileShape{};
  t.xc = std::max<int>(FM_TILE_XCMIN, (int)(((int64_t)t.nyt * g.nx + kMaxGrid - 1) / kMaxGrid));
  while ((int64_t)t.nyt * ((g.nx + t.xc - 1) / t.xc) > kMaxGrid) ++t.xc;
  t.grid = t.nyt * ((g.nx + t.xc - 1) / t.xc);
  return t;
}

// Workgroups (hence partial sums) of the last pass of an iteration: a line-search
// pass, or the direction step's last pass (tiled or not) when there is none.
int tail_nparts(const fm_plan *p) {
  if (p->prm.nmls > 1) return p->sgrid;
  const fm::TileShape ts = fused_red_dir(p) ? tile_shape(p->geo) : fm::TileShape{};
  return ts.grid > 0 ? ts.grid : p->sgrid;
}

// One NCG iteration: gradient, preconditioner (+ dots), direction, and the
// remaining line-search passes; the last pass is consumed by the next
// iteration's gradient pass (or by the final pass).
template <typename T, int LMAX>
fm_status enqueue_iteration(fm_plan *p, hipStream_t s, Recorder *rec = nullptr) {
  // FP32, 2-6 echoes, columns a multiple of 4: the 16-byte-load passes (gradient
  // passes of either stencil; the line-search passes have none)
  const int quad = std::is_same<T, float>::value && p->prm.necho <= 6 && p->geo.nz % 4 == 0 ? p->prm.necho : 0;
  if (p->reg2) {
    if (quad == 2)
      FM_LAUNCH(FM_K_GRAD, (fm::k_grad2_q<2>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    else if (quad == 3)
      FM_LAUNCH(FM_K_GRAD, (fm::k_grad2_q<3>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    else if (quad == 4)
      FM_LAUNCH(FM_K_GRAD, (fm::k_grad2_q<4>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    else if (quad == 5)
      FM_LAUNCH(FM_K_GRAD, (fm::k_grad2_q<5>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    else if (quad == 6)
      FM_LAUNCH(FM_K_GRAD, (fm::k_grad2_q<6>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    else
      FM_LAUNCH(FM_K_GRAD, (fm::k_grad2<T, LMAX>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
  } else if (quad == 2) {
    FM_LAUNCH(FM_K_GRAD, (fm::k_grad_q<2, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
  } else if (quad == 3) {
    FM_LAUNCH(FM_K_GRAD, (fm::k_grad_q<3, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
  } else if (quad == 4) {
    FM_LAUNCH(FM_K_GRAD, (fm::k_grad_q<4, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
  } else if (quad == 5) {
    FM_LAUNCH(FM_K_GRAD, (fm::k_grad_q<5, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
  } else if (quad == 6) {
    FM_LAUNCH(FM_K_GRAD, (fm::k_grad_q<6, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
  } else {
    FM_LAUNCH(FM_K_GRAD, (fm::k_grad<T, LMAX, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
  }
  FM_LAUNCH_CHECK();
  set_parts(p, p->sgrid, 4);
  const fm::TileShape ts = fused_red_dir(p) ? tile_shape(p->geo) : fm::TileShape{};
  int dir_parts = p->sgrid;  // workgroups of the pass that ends the direction step
  if (ts.grid > 0) {
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_rb_black_tile<T, false>), dim3(ts.grid), dim3(fm::kNT), s, iter_args<T>(p, p->q++), ts);
    FM_LAUNCH_CHECK();
    set_parts(p, ts.grid, 2);
    FM_LAUNCH(FM_K_PRECOND_B, (fm::k_rb_red_dir_tile<T, false>), dim3(ts.grid), dim3(fm::kNT), s, iter_args<T>(p, p->q++),
              ts);
    FM_LAUNCH_CHECK();
    dir_parts = ts.grid;
  } else if (fused_red_dir(p) && p->geo.nz % 2 == 0) {
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_rb_black_pair<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
    FM_LAUNCH(FM_K_PRECOND_B, (fm::k_rb_red_dir_pair<T, false>), dim3(p->sgrid), dim3(fm::kNT), s,
              iter_args<T>(p, p->q++));
    FM_LAUNCH_CHECK();
  } else if (fused_red_dir(p)) {
    FM_LAUNCH(FM_K_PRECOND_A, (fm::k_rb_black<T, false, true>), dim3(p->sgrid), dim3(fm::kNT), s,
              iter_args<T>(p, p->q++), (const T *)nullptr);
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
    FM_LAUNCH(FM_K_PRECOND_B, (fm::k_rb_red_dir<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
    FM_LAUNCH_CHECK();
  } else {
    fm_status st = enqueue_precond<T>(p, nullptr, s, rec);
    if (st) return st;
    if (p->cm) {  // the direction pass reads the voxel-order copies of p and D
      fm::IterArgs<T> a = iter_args<T>(p, p->q++);
      a.P = (T *)p->Pv;
      a.D = (T *)p->Dv;
      FM_LAUNCH(FM_K_DIR, (fm::k_dir2<T>), dim3(p->sgrid), dim3(fm::kNT), s, a);
    } else if (p->reg2) {
      FM_LAUNCH(FM_K_DIR, (fm::k_dir2<T>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
    } else {
      FM_LAUNCH(FM_K_DIR, (fm::k_dir<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
    }
    FM_LAUNCH_CHECK();
  }
  set_parts(p, dir_parts, 3);
  for (int k = 1; k < p->prm.nmls; ++k) {
    if (quad == 2) {
      FM_LAUNCH(FM_K_MLS, (fm::k_mls_q<2, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    } else if (quad == 3) {
      FM_LAUNCH(FM_K_MLS, (fm::k_mls_q<3, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    } else if (quad == 4) {
      FM_LAUNCH(FM_K_MLS, (fm::k_mls_q<4, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    } else if (quad == 5) {
      FM_LAUNCH(FM_K_MLS, (fm::k_mls_q<5, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    } else if (quad == 6) {
      FM_LAUNCH(FM_K_MLS, (fm::k_mls_q<6, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<float>(p, p->q++));
    } else {
      FM_LAUNCH(FM_K_MLS, (fm::k_mls<T, LMAX, false>), dim3(p->sgrid), dim3(fm::kNT), s, iter_args<T>(p, p->q++));
    }
    FM_LAUNCH_CHECK();
    set_parts(p, p->sgrid, 2);
  }
  p->iter_host += 1;
  return FM_OK;
}

// Final pass: apply the last step, write the map, and record its cost.
template <typename T, int LMAX>
fm_status enqueue_final(fm_plan *p, double *f_out, hipStream_t s) {
  fm::IterArgs<T> a = iter_args<T>(p, p->q++);
  a.final_pass = 1;
  a.fout = f_out;
  if (p->reg2)
    hipLaunchKernelGGL((fm::k_grad2<T, LMAX>), dim3(p->sgrid), dim3(fm::kNT), 0, s, a);
  else
    hipLaunchKernelGGL((fm::k_grad<T, LMAX, false>), dim3(p->sgrid), dim3(fm::kNT), 0, s, a);
  FM_LAUNCH_CHECK();
  set_parts(p, p->sgrid, 4);
  const uint64_t q = p->q++;
  hipLaunchKernelGGL(fm::k_finish, dim3(1), dim3(kBlock), 0, s, (const fm::State *)(p->S + (q & 1)),
                     p->S + ((q + 1) & 1), (const double *)(p->part + (size_t)(q & 1) * p->part_rows * kMaxK),
                     p->last_nparts, p->last_nvals, p->prm.beta, p->trace, p->status);
  FM_LAUNCH_CHECK();
  set_parts(p, 0, 0);
  return FM_OK;
}

template <typename T, int LMAX>
fm_status enqueue_eval(fm_plan *p, const double *f, double *phi, double *dphi, double *curv, double *lap,
                       hipStream_t s) {
  fm::IterArgs<T> a = iter_args<T>(p, 0);
  hipLaunchKernelGGL((fm::k_eval<T, LMAX>), dim3(p->grid), dim3(kBlock), 0, s, a, f, phi, dphi, curv, lap);
  FM_LAUNCH_CHECK();
  return FM_OK;
}

// Dispatch on the working type and the echo-count bucket.
template <template <typename, int> class Op, typename... Args>
fm_status dispatch(fm_plan *p, Args... args) {
  if (p->mix) {
    switch (p->lmax) {
      case 4: return Op<float, 4>::run(p, args...);
      case 8: return Op<float, 8>::run(p, args...);
      default: return Op<float, 16>::run(p, args...);
    }
  }
  switch (p->lmax) {
    case 4: return Op<double, 4>::run(p, args...);
    case 8: return Op<double, 8>::run(p, args...);
    default: return Op<double, 16>::run(p, args...);
  }
}

template <typename T, int LMAX>
struct OpLoop {
  static fm_status run(fm_plan *p, int niter, hipStream_t s) {
    for (int i = 0; i < niter; ++i) {
      fm_status st = enqueue_iteration<T, LMAX>(p, s);
      if (st) return st;
    }
    return FM_OK;
  }
};
template <typename T, int LMAX>
struct OpIterationTimed {
  static fm_status run(fm_plan *p, hipStream_t s, Recorder *rec) { return enqueue_iteration<T, LMAX>(p, s, rec); }
};
template <typename T, int LMAX>
struct OpFinal {
  static fm_status run(fm_plan *p, double *f, hipStream_t s) { return enqueue_final<T, LMAX>(p, f, s); }
};
template <typename T, int LMAX>
struct OpEval {
  static fm_status run(fm_plan *p, const double *f, double *a, double *b, double *c, double *d, hipStream_t s) {
    return enqueue_eval<T, LMAX>(p, f, a, b, c, d, s);
  }
};

fm_status validate(const fm_params *p) {
  if (!p) return fail(FM_ERR_ARG, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(FM_ERR_SHAPE, "grid sizes must be >= 1");
  if (p->ncoil < 1) return fail(FM_ERR_SHAPE, "ncoil must be >= 1");
  if (p->necho < 2 || p->necho > FM_MAX_ECHO) return fail(FM_ERR_SHAPE, "necho must be in [2, 16]");
  for (int l = 0; l < p->necho; ++l)
    if (!std::isfinite(p->te[l])) return fail(FM_ERR_ARG, "echo times must be finite");
  if (!(p->beta >= 0.0) || !std::isfinite(p->beta)) return fail(FM_ERR_ARG, "beta must be finite and >= 0");
  if (p->niter < 0) return fail(FM_ERR_ARG, "niter must be >= 0");
  if (p->nmls < 1) return fail(FM_ERR_ARG, "nmls must be >= 1");
  if (p->model != FM_FIELDMAP && p->model != FM_WATERFAT) return fail(FM_ERR_ARG, "bad model");
  if (p->precision != FM_PREC_F64 && p->precision != FM_PREC_MIX) return fail(FM_ERR_ARG, "bad precision");
  if (p->ordering != FM_ORDER_NATURAL && p->ordering != FM_ORDER_REDBLACK && p->ordering != FM_ORDER_COLOR3 &&
      p->ordering != FM_ORDER_BLOCKRB)
    return fail(FM_ERR_ARG, "bad ordering");
  if (p->precond < FM_PRECOND_IC0 || p->precond > FM_PRECOND_ICT) return fail(FM_ERR_ARG, "bad preconditioner");
  if (p->reg_order < 0 || p->reg_order > 2) return fail(FM_ERR_ARG, "reg_order must be 1 or 2");
  if (p->reg_order == 2 && p->precond == FM_PRECOND_IC0 && p->ordering != FM_ORDER_COLOR3)
    return fail(FM_ERR_ARG, "IC(0) with second-order differences is built in three-colour order (FM_ORDER_COLOR3)");
  if (p->ordering == FM_ORDER_BLOCKRB && (int64_t)p->ny * p->nz * 80 >= ((int64_t)1 << 30))
    return fail(FM_ERR_SHAPE, "block red-black order needs ny * nz * 80 below 2^30 (its per-tile views use 32-bit offsets)");
  if (p->ordering == FM_ORDER_COLOR3 && (p->reg_order != 2 || p->precond != FM_PRECOND_IC0))
    return fail(FM_ERR_ARG, "three-colour order is built for IC(0) with second-order differences only");
  if (p->precond == FM_PRECOND_ICT) {
    if (p->ordering != FM_ORDER_NATURAL) return fail(FM_ERR_ARG, "IC_t is built in natural order");
    if (p->reg_order == 2) return fail(FM_ERR_ARG, "IC_t is built for first-order differences");
    if (p->ict_level < 0 || p->ict_level > 2) return fail(FM_ERR_ARG, "ict_level must be 0, 1 or 2");
    if (!(p->ict_factor >= 0.0) || !std::isfinite(p->ict_factor)) return fail(FM_ERR_ARG, "ict_factor must be finite, >= 0");
  }
  if (p->model == FM_FIELDMAP && p->te[1] == p->te[0])
    return fail(FM_ERR_ARG, "field-map initialisation needs t_2 != t_1");
  if (p->model == FM_WATERFAT) {
    if (p->npeak < 1 || p->npeak > FM_MAX_PEAK) return fail(FM_ERR_ARG, "water-fat needs 1..16 fat peaks");
    if (p->nsweep < 2) return fail(FM_ERR_ARG, "water-fat sweep needs >= 2 values");
    if (p->pwls_iters < 0) return fail(FM_ERR_ARG, "pwls_iters must be >= 0");
  }
  const int64_t n = (int64_t)p->nx * p->ny * p->nz;
  if (n > (int64_t)1 << 34) return fail(FM_ERR_SHAPE, "volume too large");
  return FM_OK;
}

bool plan_alloc(fm_plan *p, void **ptr, size_t bytes) {
  void *b = nullptr;
  if (hipMalloc(&b, bytes ? bytes : 1) != hipSuccess) return false;
  p->bases.push_back(b);
  *ptr = b;
  return true;
}

// Per-voxel array of elems entries of esize bytes with p->pad guard entries
// on each side (readable neighbour slots outside the volume).
bool plan_alloc_padded(fm_plan *p, void **ptr, size_t elems, size_t esize) {
  void *b = nullptr;
  if (!plan_alloc(p, &b, (elems + 2 * (size_t)p->pad) * esize)) return false;
  *ptr = (char *)b + (size_t)p->pad * esize;
  return true;
}

template <typename T>
fm_status upload_pairs(fm_plan *p, const std::vector<std::complex<double>> &G, void **dst) {
  auto pr = make_pairs<T>(p->prm, G);
  p->npairs = (int)pr.size();
  if (!plan_alloc(p, dst, sizeof(fm::PairC<T>) * pr.size())) return fail(FM_ERR_ALLOC, "hipMalloc of pairs failed");
  FM_HIP(hipMemcpy(*dst, pr.data(), sizeof(fm::PairC<T>) * pr.size(), hipMemcpyHostToDevice));
  return FM_OK;
}

fm_status wf_init(fm_plan *p, double *f0, hipStream_t s);  // fm_waterfat.inc

void free_plan(fm_plan *p) {
  if (!p) return;
  for (auto &kv : p->graphs) {
    if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
    if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
  }
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (void *b : p->bases)
    if (b) (void)hipFree(b);
  delete p;
}

// Run niter iterations as one graph launch.  The graph for the current chain
// parity and niter is captured on first use and replayed afterwards (its
// launches occupy the same chain positions modulo 2).
bool use_resident(const fm_plan *p) {
  return p->res_ok && (p->sched == FM_SCHED_RESIDENT || (p->sched == FM_SCHED_AUTO && p->res_auto));
}

size_t res_bar_bytes(const fm_plan *p) { return sizeof(uint32_t) * (fm::kResBarHead + (size_t)p->res_grid); }

template <int LR>
void *resident_kernel() {
  return (void *)fm::k_resident<LR>;
}

void *resident_kernel_for(int necho) {
  return necho <= 2 ? resident_kernel<2>() : (necho == 3 ? resident_kernel<3>() : resident_kernel<4>());
}

// An ordinary launch: the plan has checked that the whole grid fits on the
// device at once (occupancy x compute units), and every wait inside the
// kernel is bounded, so a grid that is not fully resident (another kernel
// holding compute units) ends with FM_ERR_TIMEOUT instead of hanging.  The
// events, when given, are attached to the dispatch itself.
template <int LR>
hipError_t launch_resident(const fm::ResArgs &a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (e0 && e1)
    hipExtLaunchKernelGGL(fm::k_resident<LR>, dim3(grid), dim3(fm::kResNT), 0, s, e0, e1, 0, a);
  else
    hipLaunchKernelGGL(fm::k_resident<LR>, dim3(grid), dim3(fm::kResNT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_resident_for(int necho, const fm::ResArgs &a, int grid, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
  return necho <= 2 ? launch_resident<2>(a, grid, s, e0, e1)
                    : (necho == 3 ? launch_resident<3>(a, grid, s, e0, e1) : launch_resident<4>(a, grid, s, e0, e1));
}

// niter iterations in one launch of the resident schedule.
fm_status run_resident(fm_plan *p, int niter, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  fm::ResArgs a{};
  a.geo = p->geo;
  a.tile = p->res_tile;
  a.beta = p->prm.beta;
  a.dat = (const fm::T2<float> *)p->dat;
  a.code = p->code;
  a.pairs = (const fm::PairC<float> *)p->pairs;
  for (int i = 0; i < 2; ++i) {
    a.F[i] = (float *)p->F[i];
    a.Z[i] = (float *)p->Z[i];
    a.G[i] = (float *)p->G[i];
  }
  a.Gr = (float *)p->X;  // n floats: the two parity halves of the red face voxels' g (unused otherwise in red-black order)
  a.P = (float *)p->P;
  a.hinv = p->hinv;
  a.par0 = (int32_t)(p->iter_host & 1);
  a.niter = niter;
  a.nparts_in = p->last_nparts;
  a.nvals_in = p->last_nvals;
  const uint64_t q = p->q;
  a.sin = p->S + (q & 1);
  a.sout = p->S + ((q + 1) & 1);
  a.pin = p->part + (size_t)(q & 1) * p->part_rows * kMaxK;
  a.part = p->res_part;
  a.bar = p->res_bar;
  a.status = p->status;
  a.trace = p->trace;
  FM_HIP(hipMemsetAsync(p->res_bar, 0, res_bar_bytes(p), s));
  hipError_t err = launch_resident_for(p->prm.necho, a, p->res_grid, s, e0, e1);
  if (err != hipSuccess) return fail(FM_ERR_HIP, std::string("resident launch: ") + hipGetErrorString(err));
  p->q += 1;
  p->iter_host += niter;
  set_parts(p, 0, 0);
  return FM_OK;
}

// Tiles of whole columns for the resident schedule: at most kResTile voxels
// each, all resident at once.  Every barrier waits for the most loaded CU, so
// the tiling minimises the voxels of the busiest CU (tiles per CU rounded up
// times voxels per tile), then the number of tiles, then the tile perimeter.  False if the plan does
// not qualify.  res_auto: the volume is large enough for the resident
// schedule to beat streaming (measured: below about 1024 voxels per CU the
// fixed cost of its grid barriers dominates).
bool plan_resident(fm_plan *p) {
  const fm_params &q = p->prm;
  if (!p->mix || q.precond != FM_PRECOND_IC0 || q.ordering != FM_ORDER_REDBLACK || q.necho < 2 || q.necho > 4)
    return false;
  // voxel pairs (z even, z odd) of one column: one red and one black voxel
  if (q.nz > fm::kResTile || q.nz % 2) return false;
  int ncu = 0, per = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || ncu < 1)
    return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, resident_kernel_for(q.necho), fm::kResNT, 0) != hipSuccess ||
      per < 1)
    return false;
  const long maxblocks = (long)per * ncu;
  const int C = fm::kResTile / q.nz;  // columns per tile, at most
  long best_cost = -1, best_nt = 0;
  for (int tx = 1; tx <= C && tx <= q.nx; ++tx)
    for (int ty = 1; tx * ty <= C && ty <= q.ny; ++ty) {
      // at most one neighbour across a tile face per axis: tiles at least 2 wide (or the whole axis)
      if ((tx < 2 && q.nx > 1) || (ty < 2 && q.ny > 1)) continue;
      const long nt = (long)((q.nx + tx - 1) / tx) * ((q.ny + ty - 1) / ty);
      if (nt > maxblocks) continue;
      const long cost = ((nt + ncu - 1) / ncu) * (long)tx * ty * q.nz;
      const bool squarer = tx + ty < p->res_tile.tx + p->res_tile.ty;  // shorter perimeter: less halo
      if (best_cost < 0 || cost < best_cost || (cost == best_cost && (nt < best_nt || (nt == best_nt && squarer)))) {
        best_cost = cost;
        best_nt = nt;
        p->res_tile.tx = tx;
        p->res_tile.ty = ty;
        p->res_tile.ntx = (q.nx + tx - 1) / tx;
        p->res_tile.nty = (q.ny + ty - 1) / ty;
      }
    }
  if (best_cost < 0) return false;
  p->res_grid = (int)best_nt;
  p->res_auto = p->n >= 512L * ncu;
  return true;
}

fm_status run_graph(fm_plan *p, int niter, hipStream_t s);

fm_status run_iterations(fm_plan *p, int niter, hipStream_t s) {
  if (niter <= 0) return FM_OK;
  if (use_resident(p)) return run_resident(p, niter, s);
  if (!p->ict) return run_graph(p, niter, s);
  // IC_t launches a kernel per wavefront level (thousands per iteration): one
  // graph of one iteration, replayed niter times
  for (int i = 0; i < niter; ++i) {
    fm_status st = run_graph(p, 1, s);
    if (st) return st;
  }
  return FM_OK;
}

fm_status run_graph(fm_plan *p, int niter, hipStream_t s) {
  const std::vector<int64_t> key = {(int64_t)(p->q & 1), niter, p->iter_host & 1, p->last_nparts, p->last_nvals};
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    const uint64_t q0 = p->q;
    const int64_t it0 = p->iter_host;
    const int np0 = p->last_nparts, nv0 = p->last_nvals;
    FM_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    fm_status st = dispatch<OpLoop>(p, niter, p->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      p->q = q0;
      p->iter_host = it0;
      set_parts(p, np0, nv0);
      return st;
    }
    if (e != hipSuccess) return fail(FM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(FM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    it = p->graphs.emplace(key, std::make_pair(g, ge)).first;
  } else {
    p->q += launches_per_iteration(p) * (uint64_t)niter;
    p->iter_host += niter;
    set_parts(p, tail_nparts(p), tail_nvals(p));
  }
  FM_HIP(hipGraphLaunch(it->second.second, s));
  return FM_OK;
}

template <typename T>
fm_status enqueue_start(fm_plan *p, const double *f0, hipStream_t s) {
  p->iter_host = 0;
  set_parts(p, 0, 0);
  const uint64_t q = p->q++;
  hipLaunchKernelGGL(fm::k_start<T>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, f0, (const uint8_t *)p->code,
                     (T *)p->F[1], (T *)p->Z[1], (T *)p->G[1], p->cm ? p->cm_elems : p->n, p->S + ((q + 1) & 1),
                     p->prm.niter, p->prm.nmls, (const double *)p->nmask);
  FM_LAUNCH_CHECK();
  return FM_OK;
}

fm_status check_plan(fm_plan *p) {
  if (!p) return fail(FM_ERR_ARG, "plan is NULL");
  int cur = 0;
  FM_HIP(hipGetDevice(&cur));
  if (cur != p->device) return fail(FM_ERR_STATE, "plan was created on another device");
  return FM_OK;
}

fm_status read_status(fm_plan *p, hipStream_t s, int32_t *status) {
  FM_HIP(hipMemcpyAsync(status, p->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FM_HIP(hipStreamSynchronize(s));
  return FM_OK;
}

// ---------------------------------------------------------------------------
// Implicit adjoint: CG on the exact Hessian at fhat, preconditioned like the
// iteration.  The chain has its own state/partial ping-pong (position aq).
fm_status adj_alloc(fm_plan *p) {
  if (p->adj_ready) return FM_OK;
  const size_t n = (size_t)p->n, ts = p->tsize;
  bool ok = plan_alloc_padded(p, &p->aR, n, ts) && plan_alloc_padded(p, &p->aZ, n, ts) &&
            plan_alloc_padded(p, &p->aX, n, ts) && plan_alloc_padded(p, &p->aDc, n, ts) &&
            plan_alloc_padded(p, &p->aH, n, ts) && plan_alloc_padded(p, &p->aV, n, ts) &&
            plan_alloc_padded(p, &p->aDd[0], n, ts) && plan_alloc_padded(p, &p->aDd[1], n, ts) &&
            plan_alloc_padded(p, (void **)&p->a_hinv, n, sizeof(double)) &&
            plan_alloc_padded(p, (void **)&p->a_ipiv, n, sizeof(double)) &&
            plan_alloc(p, (void **)&p->a_part, sizeof(double) * 2 * p->part_rows * kMaxK) &&
            plan_alloc(p, (void **)&p->aS, sizeof(fm::State) * 2) && plan_alloc(p, (void **)&p->a_status, sizeof(int32_t));
  if (!ok) return fail(FM_ERR_ALLOC, "hipMalloc of the adjoint workspace failed");
  if (hipMemset(p->a_part, 0, sizeof(double) * 2 * p->part_rows * kMaxK) != hipSuccess ||
      hipMemset(p->aS, 0, sizeof(fm::State) * 2) != hipSuccess)
    return fail(FM_ERR_HIP, "hipMemset of the adjoint state failed");
  p->adj_ready = true;
  return FM_OK;
}

template <typename T>
fm::AdjArgs<T> adj_args(fm_plan *p, uint64_t q, int par, int nparts_in, int nvals_in) {
  fm::AdjArgs<T> a{};
  a.geo = p->geo;
  a.L = p->prm.necho;
  a.beta = p->prm.beta;
  a.dat = (const fm::T2<T> *)p->dat;
  a.code = p->code;
  a.pairs = (const fm::PairC<T> *)p->pairs;
  a.F = (const T *)p->F[p->iter_host & 1];  // the final pass wrote fhat there
  a.R = (T *)p->aR;
  a.Zp = (const T *)p->aZ;
  a.Dd[0] = (T *)p->aDd[0];
  a.Dd[1] = (T *)p->aDd[1];
  a.V = (T *)p->aV;
  a.H = (T *)p->aH;
  a.Dc = (T *)p->aDc;
  a.hinv = p->a_hinv;
  a.par = par;
  a.nparts_in = nparts_in;
  a.nvals_in = nvals_in;
  a.sin = p->aS + (q & 1);
  a.sout = p->aS + ((q + 1) & 1);
  a.pin = p->a_part + (size_t)(q & 1) * p->part_rows * kMaxK;
  a.pout = p->a_part + (size_t)((q + 1) & 1) * p->part_rows * kMaxK;
  a.status = p->a_status;
  return a;
}

// Arguments of the iteration's preconditioner passes pointed at the adjoint
// buffers: right-hand side r, output z, curvature D of the Huber model.
template <typename T>
fm::IterArgs<T> adj_precond_args(fm_plan *p, uint64_t q, int nparts_in, int nvals_in) {
  fm::IterArgs<T> a{};
  a.geo = p->geo;
  a.L = p->prm.necho;
  a.beta = p->prm.beta;
  a.dat = (const fm::T2<T> *)p->dat;
  a.code = p->code;
  a.pairs = (const fm::PairC<T> *)p->pairs;
  for (int i = 0; i < 2; ++i) {
    a.F[i] = (T *)p->aV;
    a.Z[i] = (T *)p->aV;
    a.G[i] = (T *)p->aR;
  }
  a.D = (T *)p->aDc;
  a.X = (T *)p->aX;
  a.P = (T *)p->aZ;
  a.ipiv = p->a_ipiv;
  a.hinv = p->a_hinv;
  a.write_hinv = 0;
  a.store_piv = 0;
  a.par = 0;
  a.nparts_in = nparts_in;
  a.nvals_in = nvals_in;
  a.sin = p->aS + (q & 1);
  a.sout = p->aS + ((q + 1) & 1);
  a.pin = p->a_part + (size_t)(q & 1) * p->part_rows * kMaxK;
  a.pout = p->a_part + (size_t)((q + 1) & 1) * p->part_rows * kMaxK;
  a.status = p->a_status;
  a.trace = nullptr;
  return a;
}

template <typename T>
fm_status adj_enqueue_iteration(fm_plan *p, uint64_t &q, int &np, int &nv, int k, hipStream_t s) {
  const T *r = (const T *)p->aR;
  Recorder *rec = nullptr;
  if (p->reg2) {
    // second-order C: diag(H) with diag(C^T C) of the 13-point operator (also for IC(0) plans), or none
    FM_LAUNCH(0, fm::k_diag2<T>, dim3(p->sgrid), dim3(fm::kNT), s, adj_precond_args<T>(p, q++, np, nv), r,
              p->prm.precond == FM_PRECOND_NONE ? 1 : 0);
    FM_LAUNCH_CHECK();
    np = p->sgrid;
    nv = 2;
  } else if (p->prm.precond == FM_PRECOND_IC0) {
    // natural-order IC(0) also for block red-black plans (v does not depend on the preconditioner)
    if (p->prm.ordering == FM_ORDER_NATURAL || p->prm.ordering == FM_ORDER_BLOCKRB) {
      FM_LAUNCH(0, fm::k_ic_fwd_wave<T>, dim3(p->wf.ntiles), dim3(64), s, adj_precond_args<T>(p, q++, np, nv), p->wf, r);
      FM_LAUNCH_CHECK();
      np = 0;
      nv = 0;
      FM_LAUNCH(0, fm::k_ic_bwd_wave<T>, dim3(p->wf.ntiles), dim3(64), s, adj_precond_args<T>(p, q++, np, nv), p->wf, r);
      FM_LAUNCH_CHECK();
      np = p->wf.ntiles;
      nv = 2;
    } else {
      FM_LAUNCH(0, (fm::k_rb_black<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, adj_precond_args<T>(p, q++, np, nv), r);
      FM_LAUNCH_CHECK();
      np = p->sgrid;
      nv = 2;
      FM_LAUNCH(0, (fm::k_rb_red<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, adj_precond_args<T>(p, q++, np, nv), r);
      FM_LAUNCH_CHECK();
      np = p->sgrid;
      nv = 2;
    }
  } else {
    FM_LAUNCH(0, (fm::k_diag<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, adj_precond_args<T>(p, q++, np, nv), r,
              p->prm.precond == FM_PRECOND_NONE ? 1 : 0);
    FM_LAUNCH_CHECK();
    np = p->sgrid;
    nv = 2;
  }
  if (p->reg2)
    FM_LAUNCH(0, (fm::k_adj_dir<T, true>), dim3(p->sgrid), dim3(fm::kNT), s, adj_args<T>(p, q++, k & 1, np, nv));
  else
    FM_LAUNCH(0, (fm::k_adj_dir<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, adj_args<T>(p, q++, k & 1, np, nv));
  FM_LAUNCH_CHECK();
  np = p->sgrid;
  nv = 1;
  if (p->reg2)
    FM_LAUNCH(0, (fm::k_adj_update<T, true>), dim3(p->sgrid), dim3(fm::kNT), s, adj_args<T>(p, q++, k & 1, np, nv));
  else
    FM_LAUNCH(0, (fm::k_adj_update<T, false>), dim3(p->sgrid), dim3(fm::kNT), s, adj_args<T>(p, q++, k & 1, np, nv));
  FM_LAUNCH_CHECK();
  np = p->sgrid;
  nv = 1;
  return FM_OK;
}

fm_status adj_finish(fm_plan *p, uint64_t &q, int &np, int &nv, fm::State *host, hipStream_t s) {
  hipLaunchKernelGGL(fm::k_finish, dim3(1), dim3(kBlock), 0, s, (const fm::State *)(p->aS + (q & 1)),
                     p->aS + ((q + 1) & 1), (const double *)(p->a_part + (size_t)(q & 1) * p->part_rows * kMaxK),
                     np, nv, p->prm.beta, (double *)nullptr, p->a_status);
  FM_LAUNCH_CHECK();
  ++q;
  np = 0;
  nv = 0;
  FM_HIP(hipMemcpyAsync(host, p->aS + (q & 1), sizeof(fm::State), hipMemcpyDeviceToHost, s));
  FM_HIP(hipStreamSynchronize(s));
  return FM_OK;
}

constexpr int kAdjCheck = 8;  // CG iterations between convergence checks on the host

template <typename T, int LMAX>
struct OpAdjoint {
  static fm_status run(fm_plan *p, const double *dldf, const void *sens, void *dldy, double *vout, int maxit,
                       double rtol, fm::State *out, hipStream_t s) {
    uint64_t q = 0;
    int np = 0, nv = 0;
    const int write_hinv = (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_REDBLACK) ? 1 : 0;
    hipLaunchKernelGGL((fm::k_adj_setup<T, LMAX>), dim3(p->sgrid), dim3(fm::kNT), 0, s, adj_args<T>(p, q++, 0, 0, 0),
                       dldf, rtol * rtol, write_hinv);
    FM_LAUNCH_CHECK();
    np = p->sgrid;
    nv = 1;
    fm::State st{};
    int k = 0;
    while (k < maxit) {
      const int chunk = (maxit - k) < kAdjCheck ? (maxit - k) : kAdjCheck;
      for (int i = 0; i < chunk; ++i, ++k) {
        fm_status e = adj_enqueue_iteration<T>(p, q, np, nv, k, s);
        if (e) return e;
      }
      fm_status e = adj_finish(p, q, np, nv, &st, s);
      if (e) return e;
      if (st.cg_done) break;
    }
    if (maxit == 0) {
      fm_status e = adj_finish(p, q, np, nv, &st, s);
      if (e) return e;
    }
    if (p->reg2)
      hipLaunchKernelGGL((fm::k_adj_out<T, LMAX, true>), dim3(p->sgrid), dim3(fm::kNT), 0, s,
                         adj_args<T>(p, q++, 0, np, nv), (const float2 *)sens, p->prm.ncoil, (float2 *)dldy, vout);
    else
      hipLaunchKernelGGL((fm::k_adj_out<T, LMAX, false>), dim3(p->sgrid), dim3(fm::kNT), 0, s,
                         adj_args<T>(p, q++, 0, np, nv), (const float2 *)sens, p->prm.ncoil, (float2 *)dldy, vout);
    FM_LAUNCH_CHECK();
    np = p->sgrid;
    nv = 1;
    fm_status e = adj_finish(p, q, np, nv, &st, s);
    if (e) return e;
    *out = st;
    return FM_OK;
  }
};

}  // namespace

namespace {
fm_status setup_launch(fm_plan *p, const void *y, const void *sens, const uint8_t *mask, hipStream_t s);
}

// ---------------------------------------------------------------------------
extern "C" {

const char *fm_status_string(fm_status st) {
  switch (st) {
    case FM_OK: return "ok";
    case FM_ERR_ARG: return "invalid argument";
    case FM_ERR_SHAPE: return "invalid shape";
    case FM_ERR_ALLOC: return "device allocation failed";
    case FM_ERR_HIP: return "HIP runtime error";
    case FM_ERR_NOT_PD: return "IC(0) pivot not positive";
    case FM_ERR_NONFINITE: return "non-finite value in the iteration";
    case FM_ERR_STATE: return "call out of order";
    case FM_ERR_TIMEOUT: return "device-side wait exceeded its bound";
  }
  return "unknown status";
}

const char *fm_last_error(void) { return g_last_error.c_str(); }

fm_status fm_plan_create(const fm_params *prm, fm_plan **out) {
  if (!out) return fail(FM_ERR_ARG, "plan output pointer is NULL");
  *out = nullptr;
  fm_status vs = validate(prm);
  if (vs) return vs;
  fm_plan *p = new fm_plan();
  p->prm = *prm;
  p->n = (int64_t)prm->nx * prm->ny * prm->nz;
  p->geo.nx = prm->nx;
  p->geo.ny = prm->ny;
  p->geo.nz = prm->nz;
  p->geo.n = p->n;
  p->geo.sy = prm->nz;
  p->geo.sx = (int64_t)prm->ny * prm->nz;
  p->reg2 = prm->reg_order == 2;
  // one x-plane of guard entries on each side (two for the second-order stencil's +-2 neighbours)
  p->pad = (((p->reg2 ? 2 : 1) * p->geo.sx + 63) / 64) * 64;
  p->cm = p->reg2 && prm->precond == FM_PRECOND_IC0;
  if (p->cm) {
    const int64_t m = ((int64_t)prm->nz + 2) / 3;
    p->cm_elems = 3 * ((int64_t)prm->nx + 4) * prm->ny * m;
  }
  if (p->n + 2 * p->pad >= ((int64_t)1 << 31) || p->cm_elems >= ((int64_t)1 << 31)) {
    delete p;
    return fail(FM_ERR_SHAPE, "volume too large for 32-bit voxel indices");
  }
  p->mix = prm->precision == FM_PREC_MIX;
  p->tsize = p->mix ? sizeof(float) : sizeof(double);
  p->lmax = prm->necho <= 4 ? 4 : (prm->necho <= 8 ? 8 : 16);
  const int64_t blocks = (p->n + kBlock - 1) / kBlock;
  p->grid = (int)(blocks < kMaxGrid ? blocks : kMaxGrid);
  if (p->grid < 1) p->grid = 1;
  const int64_t chunk = (int64_t)fm::kNT * (p->mix ? fm::Vpt<float>::v : fm::Vpt<double>::v);
  const int64_t sblocks = (p->n + chunk - 1) / chunk;
  p->sgrid = (int)(sblocks < kMaxGrid ? sblocks : kMaxGrid);
  if (p->sgrid < 1) p->sgrid = 1;
  auto cleanup = [&](fm_status st) {
    free_plan(p);
    return st;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return cleanup(fail(FM_ERR_HIP, "hipGetDevice failed"));
  const size_t n = (size_t)p->n, ts = p->tsize, L = (size_t)prm->necho;
  const size_t trace_bytes = sizeof(double) * FM_TR_W * ((size_t)prm->niter + 1);
#define FM_ALLOC(ptr, bytes)                                                          \
  if (!plan_alloc(p, (void **)&(ptr), (bytes)))                                       \
    return cleanup(fail(FM_ERR_ALLOC, "hipMalloc of " #ptr " failed"));
#define FM_ALLOC_PAD(ptr, esize)                                                      \
  if (!plan_alloc_padded(p, (void **)&(ptr), n, (esize)))                             \
    return cleanup(fail(FM_ERR_ALLOC, "hipMalloc of " #ptr " failed"));
  FM_ALLOC(p->dat, 2 * ts * L * n);
  FM_ALLOC_PAD(p->code, 1);  // padded like every array a kernel may address at neighbour offsets
  for (int i = 0; i < 2; ++i) {
    FM_ALLOC_PAD(p->F[i], ts);
    FM_ALLOC_PAD(p->Z[i], ts);
  }
  if (p->cm) {
    const size_t e = (size_t)p->cm_elems;
    for (int i = 0; i < 2; ++i) FM_ALLOC(p->G[i], ts * e);
    FM_ALLOC(p->D, ts * e);
    FM_ALLOC(p->X, ts * e);
    FM_ALLOC(p->X2, ts * e);
    FM_ALLOC(p->P, ts * e);
    FM_ALLOC(p->ipiv, sizeof(double) * e);
    FM_ALLOC(p->rdiag, e);
    FM_ALLOC(p->ccode, e);
    FM_ALLOC_PAD(p->Pv, ts);
    FM_ALLOC_PAD(p->Dv, ts);
  } else {
    for (int i = 0; i < 2; ++i) FM_ALLOC_PAD(p->G[i], ts);
    FM_ALLOC_PAD(p->D, ts);
    FM_ALLOC_PAD(p->X, ts);
    FM_ALLOC_PAD(p->P, ts);
    FM_ALLOC_PAD(p->ipiv, sizeof(double));
  }
  FM_ALLOC_PAD(p->hinv, sizeof(double));
  FM_ALLOC(p->S, sizeof(fm::State) * 2);
  {
    // natural-order wavefront: 8x8 column tiles in anti-diagonal order
    fm::Wavefront &w = p->wf;
    w.ntx = (prm->nx + fm::kTile - 1) / fm::kTile;
    w.nty = (prm->ny + fm::kTile - 1) / fm::kTile;
    w.ntiles = w.ntx * w.nty;
    std::vector<int2> order;
    order.reserve((size_t)w.ntiles);
    for (int d = 0; d <= w.ntx + w.nty - 2; ++d)
      for (int ti = 0; ti < w.ntx; ++ti) {
        const int tj = d - ti;
        if (tj >= 0 && tj < w.nty) order.push_back(make_int2(ti, tj));
      }
    void *ord = nullptr, *cnt = nullptr;
    FM_ALLOC(ord, sizeof(int2) * order.size());
    FM_ALLOC(cnt, sizeof(uint32_t) * 2 + sizeof(int32_t) * 2 * (size_t)w.ntiles);
    if (hipMemcpy(ord, order.data(), sizeof(int2) * order.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(cnt, 0, sizeof(uint32_t) * 2 + sizeof(int32_t) * 2 * (size_t)w.ntiles) != hipSuccess)
      return cleanup(fail(FM_ERR_HIP, "wavefront tables upload failed"));
    w.order = (const int2 *)ord;
    // block red-black: the tiles of each colour (ti + tj) mod 2
    std::vector<int2> blk[2];
    for (int ti = 0; ti < w.ntx; ++ti)
      for (int tj = 0; tj < w.nty; ++tj) blk[(ti + tj) & 1].push_back(make_int2(ti, tj));
    for (int c = 0; c < 2; ++c) {
      w.nblk[c] = (int32_t)blk[c].size();
      w.blk[c] = nullptr;
      if (blk[c].empty()) continue;
      void *bp = nullptr;
      FM_ALLOC(bp, sizeof(int2) * blk[c].size());
      if (hipMemcpy(bp, blk[c].data(), sizeof(int2) * blk[c].size(), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(FM_ERR_HIP, "block tables upload failed"));
      w.blk[c] = (const int2 *)bp;
    }
    w.ticket_fwd = (uint32_t *)cnt;
    w.ticket_bwd = (uint32_t *)cnt + 1;
    w.prog_fwd = (int32_t *)((uint32_t *)cnt + 2);
    w.prog_bwd = w.prog_fwd + w.ntiles;
    p->part_rows = (size_t)(w.ntiles > kMaxGrid ? w.ntiles : kMaxGrid);
  }
  FM_ALLOC(p->part, sizeof(double) * 2 * p->part_rows * kMaxK);
  FM_ALLOC(p->setup_part, sizeof(double) * kMaxGrid * kMaxK);
  FM_ALLOC(p->nmask, sizeof(double));
  FM_ALLOC(p->status, sizeof(int32_t));
  FM_ALLOC(p->trace, trace_bytes);
  FM_ALLOC(p->f0buf, sizeof(double) * n);
  p->res_ok = plan_resident(p);
  if (p->res_ok) {
    FM_ALLOC(p->res_part, sizeof(double) * fm::kResSlots * kMaxK * (size_t)p->res_grid);
    FM_ALLOC(p->res_bar, res_bar_bytes(p));
  }
  if (prm->precond == FM_PRECOND_ICT) {
    int noff = 0, wa = 1, wb = 1;
    if (prm->ict_level == 0) {
      noff = fm::IctPattern<0>::n, wa = fm::IctPattern<0>::a, wb = fm::IctPattern<0>::b;
    } else if (prm->ict_level == 1) {
      noff = fm::IctPattern<1>::n, wa = fm::IctPattern<1>::a, wb = fm::IctPattern<1>::b;
    } else {
      noff = fm::IctPattern<2>::n, wa = fm::IctPattern<2>::a, wb = fm::IctPattern<2>::b;
    }
    p->ict = true;
    p->ict_noff = noff;
    p->ict_nlev = wa * (prm->nx - 1) + wb * (prm->ny - 1) + (prm->nz - 1) + 1;
    p->ict_kcol = (prm->nz - 1) / wb + 1;
    p->ict_blocks = (int)(((int64_t)prm->nx * p->ict_kcol + fm::kIctNT - 1) / fm::kIctNT);
    FM_ALLOC(p->ict_lo, sizeof(double) * n * (size_t)noff);
    FM_ALLOC(p->ict_ld, sizeof(double) * n);
    FM_ALLOC(p->ict_y, sizeof(double) * n);
    FM_ALLOC(p->ict_pd, sizeof(double) * n);
    FM_ALLOC(p->ict_hmax, sizeof(double));
    FM_ALLOC(p->ict_hpart, sizeof(double) * kMaxGrid);
    if (hipMemset(p->ict_lo, 0, sizeof(double) * n * (size_t)noff) != hipSuccess ||
        hipMemset(p->ict_ld, 0, sizeof(double) * n) != hipSuccess)
      return cleanup(fail(FM_ERR_HIP, "hipMemset of the IC_t factor failed"));
  }
  if (prm->model == FM_WATERFAT) {
    FM_ALLOC(p->rho, sizeof(double) * n);
    FM_ALLOC(p->gabs, sizeof(double) * L * L);
    FM_ALLOC(p->wf_tmp, sizeof(double) * n * 4);
  }
#undef FM_ALLOC
#undef FM_ALLOC_PAD
  if (hipMemset(p->code - p->pad, 0, (size_t)n + 2 * (size_t)p->pad) != hipSuccess ||
      hipMemset(p->S, 0, sizeof(fm::State) * 2) != hipSuccess || hipMemset(p->status, 0, sizeof(int32_t)) != hipSuccess ||
      hipMemset(p->nmask, 0, sizeof(double)) != hipSuccess || hipMemset(p->trace, 0, trace_bytes) != hipSuccess ||
      hipMemset(p->part, 0, sizeof(double) * 2 * p->part_rows * kMaxK) != hipSuccess)
    return cleanup(fail(FM_ERR_HIP, "hipMemset of the plan state failed"));
  const auto G = make_gamma(*prm);
  fm_status st = p->mix ? upload_pairs<float>(p, G, &p->pairs) : upload_pairs<double>(p, G, &p->pairs);
  if (st) return cleanup(st);
  st = upload_pairs<double>(p, G, &p->pairs_d);
  if (st) return cleanup(st);
  {
    int K = 1;
    std::vector<double> tab(prm->te, prm->te + prm->necho);
    const auto Bm = make_component_matrix(*prm, &K);
    tab.insert(tab.end(), Bm.begin(), Bm.end());
    p->ncomp = K;
    if (!plan_alloc(p, (void **)&p->comp_tab, sizeof(double) * tab.size()) ||
        hipMemcpy(p->comp_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(FM_ERR_ALLOC, "upload of the component matrix failed"));
  }
  if (p->gabs) {
    std::vector<double> ga((size_t)L * L);
    for (size_t i = 0; i < ga.size(); ++i) ga[i] = std::abs(G[i]);
    if (hipMemcpy(p->gabs, ga.data(), sizeof(double) * ga.size(), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(FM_ERR_HIP, "upload of |Gamma| failed"));
  }
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(fail(FM_ERR_HIP, "hipStreamCreate failed"));
  *out = p;
  return FM_OK;
}

fm_status fm_plan_destroy(fm_plan *p) {
  if (!p) return FM_OK;
  free_plan(p);
  return FM_OK;
}

fm_status fm_ict_offsets(int32_t level, int32_t *offsets, int32_t *count) {
  if (!offsets || !count) return fail(FM_ERR_ARG, "offsets and count must not be NULL");
  auto put = [&](auto pat) {
    using P = decltype(pat);
    for (int u = 0; u < P::n; ++u)
      for (int d = 0; d < 3; ++d) offsets[3 * u + d] = P::off[u][d];
    *count = P::n;
  };
  if (level == 0)
    put(fm::IctPattern<0>{});
  else if (level == 1)
    put(fm::IctPattern<1>{});
  else if (level == 2)
    put(fm::IctPattern<2>{});
  else
    return fail(FM_ERR_ARG, "IC_t level must be 0, 1 or 2");
  return FM_OK;
}

fm_status fm_get_factor(fm_plan *p, double *L, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!L) return fail(FM_ERR_ARG, "L must not be NULL");
  if (!p->ict) return fail(FM_ERR_ARG, "the plan's preconditioner is not IC_t");
  const size_t n = (size_t)p->n;
  FM_HIP(hipMemcpyAsync(L, p->ict_ld, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  FM_HIP(hipMemcpyAsync(L + n, p->ict_lo, sizeof(double) * n * (size_t)p->ict_noff, hipMemcpyDeviceToDevice, s));
  return FM_OK;
}

fm_status fm_setup(fm_plan *p, const void *y, const void *sens, const uint8_t *mask, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!y || !mask) return fail(FM_ERR_ARG, "y and mask must not be NULL");
  if (!sens && p->prm.ncoil != 1) return fail(FM_ERR_ARG, "sens may be NULL only when ncoil == 1");
  fm_status st = setup_launch(p, y, sens, mask, s);
  if (st) return st;
  p->setup_done = true;
  return FM_OK;
}

}  // extern "C"

namespace {
// The setup kernels of fm_setup (coil combination, codes, initial map, in-mask
// count), on the plan's arrays.
fm_status setup_launch(fm_plan *p, const void *y, const void *sens, const uint8_t *mask, hipStream_t s) {
  const double two_pi = 6.283185307179586476925286766559;
  auto launch = [&](auto tag) -> fm_status {
    using T = decltype(tag);
    fm::SetupArgs<T> a{};
    a.geo = p->geo;
    a.ncoil = p->prm.ncoil;
    a.L = p->prm.necho;
    a.y = (const float2 *)y;
    a.sens = (const float2 *)sens;
    a.mask = mask;
    a.dat = (fm::T2<T> *)p->dat;
    a.estride = p->n;
    a.code = p->code;
    a.f0 = p->f0buf;
    a.inv_2pi_dt = 1.0 / (two_pi * (p->prm.te[1] - p->prm.te[0]));
    a.rho = p->rho;
    a.gabs = p->gabs;
    a.pairs_d = (const fm::PairC<double> *)p->pairs_d;
    a.npairs = p->npairs;
    if (p->prm.model == FM_WATERFAT) {
      // sweep over [-|df|/2, |df|/2], df the offset of the largest fat peak
      int big = 0;
      for (int q = 1; q < p->prm.npeak; ++q)
        if (p->prm.fat_amp[q] > p->prm.fat_amp[big]) big = q;
      a.nsweep = p->prm.nsweep;
      a.sweep_half = std::fabs(p->prm.fat_hz[big]) / 2.0;
      a.ftilde = p->wf_tmp;
    }
    a.partials = p->setup_part;
    hipLaunchKernelGGL(setup_kernel<T>(p->lmax, p->prm.model == FM_WATERFAT, p->prm.necho), dim3(p->grid),
                       dim3(kBlock), 0, s, a);
    FM_LAUNCH_CHECK();
    hipLaunchKernelGGL(fm::k_count, dim3(1), dim3(kBlock), 0, s, (const double *)p->setup_part, p->grid, p->nmask);
    FM_LAUNCH_CHECK();
    if (p->cm) {
      const int64_t blocks = (p->cm_elems + kBlock - 1) / kBlock;
      const dim3 grid((unsigned)(blocks < kMaxGrid ? blocks : kMaxGrid));
      hipLaunchKernelGGL(fm::k_colour_major2, grid, dim3(kBlock), 0, s, p->geo, (const uint8_t *)p->code, p->ccode,
                         p->rdiag);
      FM_LAUNCH_CHECK();
    }
    return FM_OK;
  };
  return p->mix ? launch(float{}) : launch(double{});
}
}  // namespace

extern "C" {

fm_status fm_init(fm_plan *p, double *f0, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!f0) return fail(FM_ERR_ARG, "f0 must not be NULL");
  if (!p->setup_done) return fail(FM_ERR_STATE, "fm_init needs fm_setup first");
  if (p->prm.model == FM_WATERFAT) return wf_init(p, f0, s);
  FM_HIP(hipMemcpyAsync(f0, p->f0buf, sizeof(double) * p->n, hipMemcpyDeviceToDevice, s));
  return FM_OK;
}

fm_status fm_eval(fm_plan *p, const double *f, double *phi, double *dphi, double *curv, double *lap,
                  hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!f) return fail(FM_ERR_ARG, "f must not be NULL");
  if (!p->setup_done) return fail(FM_ERR_STATE, "fm_eval needs fm_setup first");
  return dispatch<OpEval>(p, f, phi, dphi, curv, lap, s);
}

fm_status fm_precondition(fm_plan *p, const double *curv, const double *g, double *piv, double *pout,
                          hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!curv || !g || !pout) return fail(FM_ERR_ARG, "curv, g and p must not be NULL");
  if (!p->setup_done) return fail(FM_ERR_STATE, "fm_precondition needs fm_setup first");
  auto run = [&](auto tag) -> fm_status {
    using T = decltype(tag);
    if (p->cm) {
      hipLaunchKernelGGL(fm::k_to_cm<T>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, curv, (T *)p->D);
      FM_LAUNCH_CHECK();
      hipLaunchKernelGGL(fm::k_to_cm<T>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, g, (T *)p->G[0]);
      FM_LAUNCH_CHECK();
    } else {
      hipLaunchKernelGGL(fm::k_to_work<T>, dim3(p->grid), dim3(kBlock), 0, s, p->n, curv, (T *)p->D);
      FM_LAUNCH_CHECK();
      hipLaunchKernelGGL(fm::k_to_work<T>, dim3(p->grid), dim3(kBlock), 0, s, p->n, g, (T *)p->G[0]);
      FM_LAUNCH_CHECK();
    }
    FM_HIP(hipMemsetAsync(p->status, 0, sizeof(int32_t), s));
    const uint64_t q = p->q++;
    hipLaunchKernelGGL(fm::k_state_init, dim3(1), dim3(1), 0, s, p->S + ((q + 1) & 1), p->prm.niter, p->prm.nmls);
    FM_LAUNCH_CHECK();
    p->iter_host = 0;
    set_parts(p, 0, 0);
    if (p->prm.precond == FM_PRECOND_IC0 && p->prm.ordering == FM_ORDER_REDBLACK) {
      hipLaunchKernelGGL(fm::k_hinv<T>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, p->prm.beta,
                         (const uint8_t *)p->code, (const T *)p->D, p->hinv, p->status);
      FM_LAUNCH_CHECK();
    }
    fm_status st = enqueue_precond<T>(p, (const T *)p->G[0], s);
    if (st) return st;
    if (p->cm) {
      hipLaunchKernelGGL(fm::k_from_cm<T>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, (const T *)p->P, pout);
      FM_LAUNCH_CHECK();
      if (piv) {
        hipLaunchKernelGGL(fm::k_pivots_cm, dim3(p->grid), dim3(kBlock), 0, s, p->geo, (const double *)p->ipiv, piv);
        FM_LAUNCH_CHECK();
      }
    } else {
      hipLaunchKernelGGL(fm::k_from_work<T>, dim3(p->grid), dim3(kBlock), 0, s, p->n, (const T *)p->P, pout);
      FM_LAUNCH_CHECK();
      if (piv && p->ict) {
        hipLaunchKernelGGL(fm::k_ict_piv, dim3(p->grid), dim3(kBlock), 0, s, p->n, (const uint8_t *)p->code,
                           (const double *)p->ict_ld, piv);
        FM_LAUNCH_CHECK();
      } else if (piv) {
        hipLaunchKernelGGL(fm::k_pivots, dim3(p->grid), dim3(kBlock), 0, s, p->n, (const double *)p->ipiv, piv);
        FM_LAUNCH_CHECK();
      }
    }
    int32_t status = 0;
    fm_status rs = read_status(p, s, &status);
    if (rs) return rs;
    if (status) return fail((fm_status)status, "preconditioner: non-positive pivot");
    return FM_OK;
  };
  p->solved = false;  // the iteration state was overwritten
  return p->mix ? run(float{}) : run(double{});
}

fm_status fm_solve(fm_plan *p, const void *y, const void *sens, const uint8_t *mask, const double *f0,
                   double *f_out, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!f_out) return fail(FM_ERR_ARG, "f_out must not be NULL");
  fm_status st = fm_setup(p, y, sens, mask, s);
  if (st) return st;
  const double *start = f0;
  if (!start) {
    if (p->prm.model == FM_WATERFAT) {
      st = wf_init(p, p->f0buf, s);
      if (st) return st;
    }
    start = p->f0buf;
  }
  FM_HIP(hipMemsetAsync(p->status, 0, sizeof(int32_t), s));
  p->q = 0;
  st = p->mix ? enqueue_start<float>(p, start, s) : enqueue_start<double>(p, start, s);
  if (st) return st;
  st = run_iterations(p, p->prm.niter, s);
  if (st) return st;
  st = dispatch<OpFinal>(p, f_out, s);
  if (st) return st;
  p->solved = true;
  return FM_OK;
}

fm_status fm_iterate(fm_plan *p, int32_t niter, double *f_out, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!p->solved) return fail(FM_ERR_STATE, "fm_iterate needs a previous fm_solve");
  if (niter < 0 || !f_out) return fail(FM_ERR_ARG, "niter must be >= 0 and f_out not NULL");
  fm_status st = run_iterations(p, niter, s);
  if (st) return st;
  return dispatch<OpFinal>(p, f_out, s);
}

fm_status fm_time_kernels(fm_plan *p, int32_t niter, double *ms, int32_t *launches, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!ms || !launches || niter < 0) return fail(FM_ERR_ARG, "bad arguments to fm_time_kernels");
  if (!p->solved) return fail(FM_ERR_STATE, "fm_time_kernels needs a previous fm_solve");
  for (int k = 0; k < FM_NK; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  Recorder rec;
  if (use_resident(p) && niter > 0) {
    hipEvent_t e0, e1;
    rec.pair(FM_K_RESIDENT, &e0, &e1);
    if (rec.err != hipSuccess) return fail(FM_ERR_HIP, std::string("event create: ") + hipGetErrorString(rec.err));
    fm_status st = run_resident(p, niter, s, e0, e1);
    if (st) return st;
  }
  for (int i = 0; i < niter && !use_resident(p); ++i) {
    fm_status st = dispatch<OpIterationTimed>(p, s, &rec);
    if (st) return st;
    if (rec.err != hipSuccess) return fail(FM_ERR_HIP, std::string("event record: ") + hipGetErrorString(rec.err));
  }
  FM_HIP(hipStreamSynchronize(s));
  for (size_t k = 0; k < rec.cls.size(); ++k) {
    float t = 0.f;
    FM_HIP(hipEventElapsedTime(&t, rec.ev[2 * k], rec.ev[2 * k + 1]));
    ms[rec.cls[k]] += t;
    launches[rec.cls[k]] += 1;
  }
  return FM_OK;
}

fm_status fm_adjoint(fm_plan *p, const double *dldf, const void *sens, void *dldy, double *v_out,
                     double *dldbeta, int32_t maxit, double rtol, int32_t *iters, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!dldf) return fail(FM_ERR_ARG, "dL/df must not be NULL");
  if (!sens && p->prm.ncoil != 1 && dldy) return fail(FM_ERR_ARG, "sens may be NULL only when ncoil == 1");
  if (maxit < 0 || !(rtol >= 0.0) || !std::isfinite(rtol)) return fail(FM_ERR_ARG, "maxit must be >= 0 and rtol finite, >= 0");
  if (!p->solved) return fail(FM_ERR_STATE, "fm_adjoint needs a converged map from fm_solve or fm_iterate");
  if (p->ict) return fail(FM_ERR_ARG, "fm_adjoint preconditions with IC(0), the diagonal or nothing, not IC_t");
  fm_status st = adj_alloc(p);
  if (st) return st;
  FM_HIP(hipMemsetAsync(p->a_status, 0, sizeof(int32_t), s));
  fm::State out{};
  st = dispatch<OpAdjoint>(p, dldf, sens, dldy, v_out, (int)maxit, rtol, &out, s);
  if (st) return st;
  int32_t status = 0;
  FM_HIP(hipMemcpyAsync(&status, p->a_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FM_HIP(hipStreamSynchronize(s));
  if (iters) *iters = out.cg_it;
  if (dldbeta) *dldbeta = out.cg_dbeta;
  if (status == FM_ERR_NOT_PD) return fail(FM_ERR_NOT_PD, "adjoint CG: the Hessian is not positive definite at the map");
  if (status) return fail((fm_status)status, "adjoint CG reported a device-side error");
  return FM_OK;
}

fm_status fm_set_beta(fm_plan *p, double beta) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(FM_ERR_ARG, "beta must be finite and >= 0");
  for (auto &kv : p->graphs) {
    if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
    if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
  }
  p->graphs.clear();
  p->prm.beta = beta;
  p->solved = false;
  return FM_OK;
}

fm_status fm_components(fm_plan *p, const void *y, const void *sens, const double *f, void *m_out,
                        hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!y || !m_out) return fail(FM_ERR_ARG, "y and m_out must not be NULL");
  if (!sens && p->prm.ncoil != 1) return fail(FM_ERR_ARG, "sens may be NULL only when ncoil == 1");
  if (!p->setup_done) return fail(FM_ERR_STATE, "fm_components needs fm_setup or fm_solve first");
  if (!f && !p->solved) return fail(FM_ERR_STATE, "f is NULL and there is no solved map");
  const double *te = p->comp_tab;
  const double2 *B = (const double2 *)(p->comp_tab + p->prm.necho);
  if (p->mix) {
    hipLaunchKernelGGL(fm::k_components<float>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, p->prm.ncoil,
                       p->prm.necho, p->ncomp, (const float2 *)y, (const float2 *)sens, (const uint8_t *)p->code, f,
                       (const float *)p->F[p->iter_host & 1], te, B, (float2 *)m_out);
  } else {
    hipLaunchKernelGGL(fm::k_components<double>, dim3(p->grid), dim3(kBlock), 0, s, p->geo, p->prm.ncoil,
                       p->prm.necho, p->ncomp, (const float2 *)y, (const float2 *)sens, (const uint8_t *)p->code, f,
                       (const double *)p->F[p->iter_host & 1], te, B, (float2 *)m_out);
  }
  FM_LAUNCH_CHECK();
  return FM_OK;
}

fm_status fm_plan_status(fm_plan *p, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  int32_t status = 0;
  fm_status rs = read_status(p, s, &status);
  if (rs) return rs;
  if (status) return fail((fm_status)status, "the last solve reported a device-side error");
  return FM_OK;
}

fm_status fm_set_schedule(fm_plan *p, int32_t sched) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (sched != FM_SCHED_AUTO && sched != FM_SCHED_STREAM && sched != FM_SCHED_RESIDENT)
    return fail(FM_ERR_ARG, "unknown schedule");
  if (sched == FM_SCHED_RESIDENT && !p->res_ok)
    return fail(FM_ERR_ARG, "the plan does not qualify for the resident schedule");
  p->sched = sched;
  return FM_OK;
}

fm_status fm_get_schedule(fm_plan *p, int32_t *sched) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!sched) return fail(FM_ERR_ARG, "sched must not be NULL");
  *sched = use_resident(p) ? FM_SCHED_RESIDENT : FM_SCHED_STREAM;
  return FM_OK;
}

fm_status fm_get_trace(fm_plan *p, double *trace, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!trace) return fail(FM_ERR_ARG, "trace must not be NULL");
  FM_HIP(hipMemcpyAsync(trace, p->trace, sizeof(double) * FM_TR_W * ((size_t)p->prm.niter + 1),
                        hipMemcpyDeviceToHost, s));
  int32_t status = 0;
  fm_status rs = read_status(p, s, &status);
  if (rs) return rs;
  if (status) return fail((fm_status)status, "the solve reported a device-side error");
  return FM_OK;
}

fm_status fm_mask_count(fm_plan *p, int64_t *count, hipStream_t s) {
  fm_status cs = check_plan(p);
  if (cs) return cs;
  if (!count) return fail(FM_ERR_ARG, "count must not be NULL");
  if (!p->setup_done) return fail(FM_ERR_STATE, "fm_mask_count needs fm_setup first");
  double v = 0.0;
  FM_HIP(hipMemcpyAsync(&v, p->nmask, sizeof(double), hipMemcpyDeviceToHost, s));
  FM_HIP(hipStreamSynchronize(s));
  *count = (int64_t)v;
  return FM_OK;
}

}  // extern "C"

// Water-fat initialisation lives with the rest of the plan internals.
#include "fm_waterfat.inc"

// Batched solves of many volumes.
#include "fm_batch.inc"

// The allocation-free solve.
#include "fm_noalloc.inc"
