// Resident schedule of the red-black NCG-MLS iteration (MIX precision).
//
// One launch runs many iterations.  Each workgroup owns a tile of
// tx x ty whole columns (at most kResNT * kResV voxels) and keeps every
// per-voxel quantity of its voxels on chip for the whole launch: the echo data
// in registers; f, z, g, g_prev, D, 1/h and p in LDS.  Per iteration the
// passes are those of the streaming schedule (gradient, black, red +
// direction, line-search steps).  The gradient pass ends with a wait on the
// four face-neighbour tiles only; each later pass ends with a grid barrier at
// which every workgroup sums all workgroups' partial sums in the same fixed
// order and applies them to its own copy of the scalar state (same consume()
// as the streaming kernels, so the scalars, the trace and the status are those
// of the streaming chain).
//
// Neighbour values inside a tile come from LDS; across tile faces they come
// from global arrays, which every workgroup publishes with agent-coherent
// stores before the barrier and reads with agent-coherent loads after it (the
// tiles of one launch may run on different XCDs, whose L2 caches are not
// coherent with each other).  Per iteration only the face columns are
// published (the columns a neighbour tile reads), each voxel pair (z even,
// z odd) of a column with one 8-byte store, so every store fills whole cache
// lines: f and z in the voxel-order arrays of the streaming schedule, and the
// values only one colour's neighbours read at the pair's index j/2: g of the
// red voxels (two parity halves of Gr), 1/h of the red voxels and p of the
// black ones.  At the end of the launch every workgroup writes f, z and g of
// all its voxels to the voxel-order arrays with the streaming schedule's
// parity convention (f_i in F[i&1], z_i in Z[i&1], g_i in G[i&1]), so the
// final pass and later streaming iterations continue from them unchanged.
//
// The grid barrier is a two-level arrival count (one counter per group of
// workgroups, then one global counter); the last arrival releases each group
// through a word of its own, so no word is polled by every workgroup.  Waits
// are bounded: one that runs out sets FM_ERR_TIMEOUT (status 8) and every
// workgroup leaves the launch.
#pragma once

#include "fm_stream.hpp"

namespace fm {

constexpr int kResNT = 512;                // threads per workgroup
constexpr int kResV = 4;                   // voxel slots per thread
constexpr int kResTile = kResNT * kResV;   // voxels per tile, at most
constexpr int kResGroups = 16;             // first level of the barrier
// barrier words before the tile flags: group counters, the global counter and
// the per-group release words, each on a 128-byte line of its own
constexpr int kResBarHead = (2 * kResGroups + 1) * 32;
constexpr int kResSpin = 1 << 20;          // polls (about 1 us each) before a wait gives up
// The gradient pass hands its results only to the four face-neighbour tiles
// (the black pass needs nothing global from it), so it ends with a wait on
// their progress flags instead of a grid barrier; its partial sums are taken
// at the next barrier.
// Partial-sum slots, one per pass kind, so that a slot is only rewritten
// after every workgroup has passed the barrier following its last read:
// gradient, dot products, direction, then two alternating line-search slots.
enum { kSlotG = 0, kSlotD = 1, kSlotR = 2, kSlotM = 3, kResSlots = 5 };

struct ResTile {
  int32_t tx, ty;    // columns of a tile along x and y
  int32_t ntx, nty;  // tiles along x and y (grid = ntx * nty workgroups)
};

struct ResArgs {
  Geo geo;
  ResTile tile;
  double beta;
  const T2<float> *dat;
  const uint8_t *code;
  const PairC<float> *pairs;
  float *F[2], *Z[2], *G[2];
  float *Gr;           // [2][n/2]: g of the red voxels of the face columns at the pair index, by parity
  float *P;            // p of the black voxels of the face columns at the pair index
  double *hinv;        // 1/h of the red voxels of the face columns at the pair index
  int32_t par0;        // parity of the first iteration of the launch
  int32_t niter;       // iterations of this launch
  int32_t nparts_in;   // incoming partial sums (previous launch)
  int32_t nvals_in;
  const State *sin;
  State *sout;
  const double *pin;
  double *part;        // [kResSlots][kMaxK][grid] partial sums of the passes
  uint32_t *bar;       // [kResBarHead + grid] counters, release words and tile flags, zeroed before the launch
  int32_t *status;
  double *trace;
};

__device__ __forceinline__ uint32_t ld_coh_u32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Agent-coherent store of two adjacent floats (p 8-byte aligned) as one 8-byte store.
__device__ __forceinline__ void st_coh2(float *p, float lo, float hi) {
  const uint64_t v = (uint64_t)__float_as_uint(lo) | ((uint64_t)__float_as_uint(hi) << 32);
  __hip_atomic_store((uint64_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier number e (1, 2, ...): all of this workgroup's coherent stores
// are complete when its thread 0 arrives.  Returns false if the wait ran out
// or another workgroup already reported a time-out.
__device__ __forceinline__ bool res_barrier(uint32_t *bar, int32_t *status, uint32_t e) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __shared__ int32_t ok_s;
  if (threadIdx.x == 0) {
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int ngroups = nb < kResGroups ? nb : kResGroups;
    const int g = b % ngroups;
    const uint32_t gsize = (uint32_t)(nb / ngroups + (g < nb % ngroups ? 1 : 0));
    uint32_t *cnt = bar + kResGroups * 32;
    const uint32_t old = __hip_atomic_fetch_add(bar + g * 32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the last arrival of the last group releases every group through its own
    // word, so each word is polled by one group only
    uint32_t *rel = bar + (kResGroups + 1) * 32;
    if (old + 1 == gsize * e) {
      const uint32_t og = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (og + 1 == (uint32_t)ngroups * e)
        for (int gg = 0; gg < ngroups; ++gg) __hip_atomic_store(rel + gg * 32, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t *poll = rel + g * 32;
    const uint32_t target = e;
    int spins = 0, ok = 1;
    while (ld_coh_u32(poll) < target) {
      if (++spins > kResSpin || __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 8) {
        ok = 0;
        atomicCAS(status, 0, 8);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

// Publish this tile's progress: all its coherent stores are complete when
// thread 0 stores the count.
__device__ __forceinline__ void res_publish(uint32_t *flags, uint32_t count) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flags + blockIdx.x, count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until the face-neighbour tiles have published the count: lanes 0-3 of
// the first wave poll the four neighbours' flags together.
__device__ __forceinline__ bool res_nbwait(uint32_t *flags, const ResTile &t, int32_t *status, uint32_t count) {
  __shared__ int32_t okn_s;
  const int b = (int)blockIdx.x;
  if (threadIdx.x < kWave) {
    const int q = (int)threadIdx.x, bx = b / t.nty, by = b % t.nty;
    int nbq = -1;
    if (q == 0 && bx > 0) nbq = b - t.nty;
    if (q == 1 && bx + 1 < t.ntx) nbq = b + t.nty;
    if (q == 2 && by > 0) nbq = b - 1;
    if (q == 3 && by + 1 < t.nty) nbq = b + 1;
    int ok = 1;
    for (int spins = 0;; ++spins) {
      const bool mine = nbq < 0 || ld_coh_u32(flags + nbq) >= count;
      if (__all(mine)) break;
      const bool bad = q == 0 && (spins > kResSpin ||
                                  __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 8);
      if (__any(bad)) {
        ok = 0;
        if (q == 0) atomicCAS(status, 0, 8);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (q == 0) okn_s = ok;
  }
  __syncthreads();
  return okn_s != 0;
}

// Block-wide sum of K values with the same rounding as block_sum (waves
// first, then the waves' sums in wave order); the totals go to thread 0 only
// (the one that publishes or applies them).  Thread k sums value k over the
// waves, so no thread holds more than the K totals (block_sum's every-thread
// loop over K x waves would).  No barrier before the wave sums are written:
// every call is separated from the one before it by at least one
// __syncthreads (a pass, a grid barrier or a neighbour wait lies between), so
// they cannot overwrite sums the previous call is still reading.
template <int K>
__device__ __forceinline__ void res_block_sum(double (&v)[K]) {
  constexpr int NW = kResNT / kWave;
  __shared__ double red[K][NW];
  __shared__ double tot[K];
  wave_reduce<K>(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[threadIdx.x][w];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = tot[k];
  }
}

template <int K>
__device__ __forceinline__ void res_put(double (&v)[K], double *part, int slot) {
  res_block_sum<K>(v);
  if (threadIdx.x == 0) {
    const int nb = (int)gridDim.x;
#pragma unroll
    for (int k = 0; k < K; ++k) st_coh(part + ((size_t)slot * kMaxK + k) * nb + blockIdx.x, v[k]);
  }
}

// Make the voxel indices opaque at the start of each pass, so that the
// compiler forms global addresses inside the pass instead of keeping 64-bit
// addresses of every array for every slot live across the whole launch.
template <int V>
__device__ __forceinline__ int res_opaque(int (&jv)[V]) {
#pragma unroll
  for (int v = 0; v < V; ++v) asm volatile("" : "+v"(jv[v]));
  int t = (int)threadIdx.x;  // LDS addresses likewise: one base register plus immediate offsets
  asm volatile("" : "+v"(t));
  return t;
}

// Global indices of a voxel's neighbours across the tile faces: at most one
// along x and one along y (tiles are at least 2 columns wide).  A voxel with
// no such neighbour gets the index dflt (one address shared by the wave, so
// the load costs one cache line), which keeps every halo load unconditional:
// all of a pass's halo loads are in flight together.
__device__ __forceinline__ void res_halo(uint32_t c, int j, int dflt, const Offs &of, int &jx, int &jy) {
  const uint32_t tin = c >> 8;
  jx = (has_nb(c, 0) && !(tin & 1u)) ? j + of.o[0] : ((has_nb(c, 1) && !(tin & 2u)) ? j + of.o[1] : dflt);
  jy = (has_nb(c, 2) && !(tin & 4u)) ? j + of.o[2] : ((has_nb(c, 3) && !(tin & 8u)) ? j + of.o[3] : dflt);
}

// A neighbour's value: from the tile's LDS vector when the neighbour is in the
// tile, else the prefetched halo value (branch-free: the LDS read goes to the
// voxel itself when it is not used).
template <typename T>
__device__ __forceinline__ T res_nb(const T *l, int li, int lo, bool in_tile, T halo) {
  const T x = l[in_tile ? li + lo : li];
  return in_tile ? x : halo;
}

template <int LR>
__global__ __launch_bounds__(kResNT, 4) void k_resident(ResArgs a) {
  // Thread t owns the voxel pairs (2q, 2q+1) of the tile's z-fastest order
  // with q = t and q = t + kResNT: with an even column length each pair is one
  // red and one black voxel of a column, so in the black and the red pass
  // every lane does the heavy work on one voxel of each of its pairs.
  constexpr int V = kResV, NPR = kResV / 2;
  const Geo g = a.geo;
  const int nz = g.nz, tx = a.tile.tx, ty = a.tile.ty;
  const int bx = (int)blockIdx.x / a.tile.nty, by = (int)blockIdx.x % a.tile.nty;
  const Offs of(g);
  const int loff[6] = {-ty * nz, ty * nz, -nz, nz, -1, 1};
  const int jdflt = (bx * tx * g.ny + by * ty) * nz;  // first voxel of the tile
  // the tile's per-voxel vectors (z-fastest tile order)
  __shared__ float lf[kResTile], lz[kResTile], lg[2][kResTile], lp[kResTile], ld[kResTile];
  __shared__ double lh[kResTile];
  __shared__ State ls;
  // echo-pair constants, read by every voxel: kept in LDS (uniform reads that
  // do not wait on the vector-memory counter)
  constexpr int NP = LR * (LR - 1) / 2;
  __shared__ PairC<float> lpc[NP];
  if (threadIdx.x < NP) lpc[threadIdx.x] = a.pairs[threadIdx.x];

  // this thread's voxels v = 2 * pair + (0, 1): global index (-1: none),
  // code | in-tile neighbour bits << 8 | (second voxel of the pair is black) << 16, echo data
  int jv[V];
  uint32_t cv[V];
  // the echo data, or with at most three echoes (no more pairs than echoes) the
  // per-pair weights and phase offsets, which do not change during the launch
  constexpr bool PCN = NP <= LR;
  constexpr int NE = PCN ? NP : LR;
  float ea[V][NE], eb[V][NE];
  {
    const int odd = a.par0 & 1;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int li = 2 * ((v >> 1) * kResNT + (int)threadIdx.x) + (v & 1);
      const int lc = li / nz, zz = li - lc * nz, lx = lc / ty, ly = lc - lx * ty;
      const int x = bx * tx + lx, y = by * ty + ly;
      const bool valid = lc < tx * ty && x < g.nx && y < g.ny;
      const int j = valid ? (x * g.ny + y) * nz + zz : 0;
      jv[v] = valid ? j : -1;
      const uint32_t tin = (lx > 0 ? 1u : 0u) | (lx < tx - 1 ? 2u : 0u) | (ly > 0 ? 4u : 0u) |
                           (ly < ty - 1 ? 8u : 0u) | (zz > 0 ? 16u : 0u) | (zz < nz - 1 ? 32u : 0u);
      const uint32_t second_black = ((x + y) & 1) ? 0u : 1u;  // pair (z even, z odd): x+y+z odd is black
      cv[v] = (valid ? (uint32_t)a.code[j] : 0u) | (tin << 8) | (second_black << 16);
      lf[li] = valid ? a.F[odd ^ 1][j] : 0.f;  // f_{i0-1}
      lz[li] = valid ? a.Z[odd ^ 1][j] : 0.f;  // z_{i0-1}
      lg[odd ^ 1][li] = valid ? a.G[odd ^ 1][j] : 0.f;  // g_{i0-1}
      lg[odd][li] = 0.f;
      lp[li] = 0.f;
      ld[li] = 0.f;
      lh[li] = 0.0;
      float rho[LR], tau[LR];
#pragma unroll
      for (int l = 0; l < LR; ++l) {
        const T2<float> d = valid ? a.dat[(size_t)l * (size_t)g.n + j] : T2<float>{0.f, 0.f};
        rho[l] = d.x;
        tau[l] = d.y;
      }
      if constexpr (PCN) {
        pair_consts<float, LR>(rho, tau, a.pairs, ea[v], eb[v]);
      } else {
#pragma unroll
        for (int l = 0; l < LR; ++l) {
          ea[v][l] = rho[l];
          eb[v][l] = tau[l];
        }
      }
    }
  }
  // pairs of face columns: a voxel of the pair has an in-mask x or y neighbour outside the tile
  uint32_t facem = 0;
#pragma unroll
  for (int q = 0; q < NPR; ++q) {
    const uint32_t c0 = cv[2 * q], c1 = cv[2 * q + 1];
    const uint32_t out0 = ((c0 >> 1) & 15u) & ~((c0 >> 8) & 15u), out1 = ((c1 >> 1) & 15u) & ~((c1 >> 8) & 15u);
    if (jv[2 * q] >= 0 && (out0 | out1)) facem |= 1u << q;
  }
  const int n2 = (int)(g.n >> 1);
  // g_{i0-1} of the red face voxels, read as g_prev by the neighbours' first black pass (after the
  // gradient pass's neighbour wait, which completes these stores first)
#pragma unroll
  for (int q = 0; q < NPR; ++q) {
    if (!(facem >> q & 1u)) continue;
    const int l0 = 2 * (q * kResNT + (int)threadIdx.x), lir = l0 + (((cv[2 * q] >> 16) & 1u) ? 0 : 1);
    st_coh(a.Gr + (size_t)((a.par0 & 1) ^ 1) * n2 + (jv[2 * q] >> 1), lg[(a.par0 & 1) ^ 1][lir]);
  }
  {
    // the incoming state and the partial sums the previous launch left (as take_state)
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < a.nparts_in; b += kResNT) {
      double x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = a.pin[(size_t)k * a.nparts_in + b];
#pragma unroll
      for (int k = 0; k < 4; ++k) t[k] += k < a.nvals_in ? x[k] : 0.0;
    }
    res_block_sum<4>(t);
    if (threadIdx.x == 0) {
      State s0 = *a.sin;
      if (s0.kind != PK_NONE) {
        if ((s0.nparts != a.nparts_in || a.nvals_in > 4) && blockIdx.x == 0) set_status(a.status, 7);
        const double tt[kMaxK] = {t[0], t[1], t[2], t[3]};
        consume(s0, tt, a.beta, a.trace, a.status, blockIdx.x == 0);
      }
      ls = s0;
    }
  }
  __syncthreads();
  const double beta = a.beta, b2 = a.beta * a.beta;
  const float betaf = (float)a.beta;
  const int nmls = ls.nmls;
  uint32_t e = 0;  // barriers passed
  int mslot = 0;   // alternating line-search slot
  uint32_t *flags = a.bar + kResBarHead;

  // sum all workgroups' K partials of slot s0 (values 0 .. K0-1) and of slot
  // s1 (the rest) in one block sum (fixed order, identical everywhere)
  auto take = [&](auto &t, int s0, int k0, int s1) {
    constexpr int K = sizeof(t) / sizeof(double);
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = 0.0;
    const int nb = (int)gridDim.x;
    for (int b = threadIdx.x; b < nb; b += kResNT) {
      // all K loads first: the compiler keeps coherent loads in program order
      // and would wait for each one before issuing the next
      double x[K];
#pragma unroll
      for (int k = 0; k < K; ++k)
        x[k] = ld_coh(a.part + ((size_t)(k < k0 ? s0 : s1) * kMaxK + (k < k0 ? k : k - k0)) * nb + b);
#pragma unroll
      for (int k = 0; k < K; ++k) t[k] += x[k];
    }
    res_block_sum<K>(t);
  };
  auto apply = [&](auto &t, int kind) {  // thread 0 updates the shared state in place
    constexpr int K = sizeof(t) / sizeof(double);
    if (threadIdx.x == 0) {
      double tt[kMaxK];
#pragma unroll
      for (int k = 0; k < kMaxK; ++k) tt[k] = k < K ? t[k < K ? k : 0] : 0.0;
      ls.kind = kind;
      consume(ls, tt, beta, a.trace, a.status, blockIdx.x == 0);
    }
  };
  // end of a pass: publish the partial sums, wait for every workgroup, apply
  // the totals (after those of a deferred gradient pass, if any)
  auto finish = [&](auto &acc, int kind, int slot, bool with_grad) -> bool {
    constexpr int K = sizeof(acc) / sizeof(double);
    res_put<K>(acc, a.part, slot);
    if (!res_barrier(a.bar, a.status, ++e)) return false;
    if (with_grad) {
      double tt[4 + K];
      take(tt, kSlotG, 4, slot);
      double tg[4], t[K];
#pragma unroll
      for (int k = 0; k < 4; ++k) tg[k] = tt[k];
#pragma unroll
      for (int k = 0; k < K; ++k) t[k] = tt[4 + k];
      apply(tg, PK_GRAD);
      apply(t, kind);
    } else {
      double t[K];
      take(t, slot, K, slot);
      apply(t, kind);
    }
    __syncthreads();
    return true;
  };

  bool live = true;
  for (int it = 0; it < a.niter && live; ++it) {
    const int par = (a.par0 + it) & 1;
    float *Fc = a.F[par], *Fp = a.F[par ^ 1], *Zc = a.Z[par], *Zp = a.Z[par ^ 1];
    float *Grc = a.Gr + (size_t)par * n2, *Grp = a.Gr + (size_t)(par ^ 1) * n2;
    float *lgc = lg[par], *lgp = lg[par ^ 1];

    // ---- gradient pass (as k_grad), every voxel: f_i = f_{i-1} + alpha z_{i-1}, g_i, D_i, 1/h_i
    {
      const int tid = res_opaque(jv);
      const float alpha = (float)ls.alpha;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      float fj[V], hfx[V], hzx[V], hfy[V], hzy[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        int jx, jy;
        res_halo(cv[v], jv[v], jdflt, of, jx, jy);
        hfx[v] = ld_coh(Fp + jx);
        hzx[v] = ld_coh(Zp + jx);
        hfy[v] = ld_coh(Fp + jy);
        hzy[v] = ld_coh(Zp + jy);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int li = 2 * ((v >> 1) * kResNT + tid) + (v & 1);
        fj[v] = (cv[v] & NB_SELF) ? lf[li] + alpha * lz[li] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) lf[2 * ((v >> 1) * kResNT + tid) + (v & 1)] = fj[v];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint32_t c = cv[v];
        const int li = 2 * ((v >> 1) * kResNT + tid) + (v & 1);
        if (!(c & NB_SELF)) {
          lgc[li] = 0.f;
          ld[li] = 0.f;
          lh[li] = 0.0;
          continue;
        }
        float lap = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(c, k)) {
            const float fn = (c >> (8 + k)) & 1u ? lf[li + loff[k]]
                                                  : (k < 2 ? hfx[v] + alpha * hzx[v] : hfy[v] + alpha * hzy[v]);
            lap += fj[v] - fn;
          }
        float phi, dphi, curv;
        if constexpr (PCN)
          voxel_terms_pc<float, NP>(ea[v], eb[v], lpc, fj[v], phi, dphi, curv);
        else
          voxel_terms<float, LR>(ea[v], eb[v], LR, lpc, fj[v], phi, dphi, curv);
        const float gj = dphi + betaf * lap;
        const double h = (double)curv + beta * nb_deg(c);
        const double hi = h > 0.0 ? 1.0 / h : 0.0;
        lgc[li] = gj;
        ld[li] = curv;
        lh[li] = hi;
        acc[0] += (double)phi;
        acc[1] += (double)fj[v] * (double)lap;
        acc[2] += (double)gj * (double)gj;
        acc[3] += (double)lz[li] * (double)gj;
      }
      // publish the face columns after the arithmetic (a store must be
      // acknowledged before any later wait on the vector-memory counter
      // completes): f of the pair, g and 1/h of its red voxel
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        if (!(facem >> q & 1u)) continue;
        const int l0 = 2 * (q * kResNT + tid), lir = l0 + (((cv[2 * q] >> 16) & 1u) ? 0 : 1), j0 = jv[2 * q];
        st_coh2(Fc + j0, lf[l0], lf[l0 + 1]);
        st_coh(Grc + (j0 >> 1), lgc[lir]);
        st_coh(a.hinv + (j0 >> 1), lh[lir]);
      }
      res_put<4>(acc, a.part, kSlotG);
      res_publish(flags, (uint32_t)it + 1);
    }

    // ---- black pass with both dot products (as k_rb_black_pair): per pair,
    // the black voxel's pivot and p, the red voxel's terms of the dot products.
    // The red terms and the black voxels whose neighbours are all in the tile
    // come first, while the face-neighbour tiles finish their gradient pass;
    // then the wait for them, the halo loads and the black voxels on the faces.
    {
      const int tid = res_opaque(jv);
      double acc[2] = {0.0, 0.0};
      bool bface[NPR];  // the black voxel has an in-mask x or y neighbour outside the tile
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        const uint32_t cb = ((cv[2 * q] >> 16) & 1u) ? cv[2 * q + 1] : cv[2 * q];
        bface[q] = (((cb >> 1) & 15u) & ~((cb >> 8) & 15u)) != 0;
      }
      auto black = [&](int q, float hgx, float hpx, double hhx, float hgy, float hpy, double hhy) {
        const bool sb = (cv[2 * q] >> 16) & 1u;
        const uint32_t cb = sb ? cv[2 * q + 1] : cv[2 * q];
        const int lib = 2 * (q * kResNT + tid) + (sb ? 1 : 0);
        if (!(cb & NB_SELF)) return;
        const float g0 = lgc[lib], gp0 = lgp[lib];
        const double h = (double)ld[lib] + beta * nb_deg(cb);
        double sp = 0.0, sxv = 0.0, syp = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const bool in = (cb >> (8 + k)) & 1u;
          const double hn = res_nb(lh, lib, loff[k], in, k < 2 ? hhx : hhy);
          const float gn = res_nb(lgc, lib, loff[k], in, k < 2 ? hgx : hgy);
          const float gpn = res_nb(lgp, lib, loff[k], in, k < 2 ? hpx : hpy);
          const bool hk = has_nb(cb, k);
          sp += hk ? hn : 0.0;
          sxv += hk ? (double)gn * hn : 0.0;
          syp += hk ? (double)gpn * hn : 0.0;
        }
        const double piv = h - b2 * sp;
        double ip = 1.0 / piv;
        if (!(piv > 0.0)) {
          set_status(a.status, 5);
          ip = 0.0;
        }
        const double yb = (double)g0 + beta * sxv;
        const double xb = yb * ip;
        lp[lib] = (float)xb;
        acc[0] += yb * xb;
        acc[1] += ((double)gp0 + beta * syp) * xb;
      };
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        const bool sb = (cv[2 * q] >> 16) & 1u;
        const uint32_t cr = sb ? cv[2 * q] : cv[2 * q + 1];
        const int lir = 2 * (q * kResNT + tid) + (sb ? 0 : 1);
        if (cr & NB_SELF) {
          const float g0 = lgc[lir];
          const double gh = (double)g0 * lh[lir];
          acc[0] += (double)g0 * gh;
          acc[1] += (double)lgp[lir] * gh;
        }
        if (!bface[q]) black(q, 0.f, 0.f, 0.0, 0.f, 0.f, 0.0);  // every neighbour it uses is in the tile
      }
      if (!(live = res_nbwait(flags, a.tile, a.status, (uint32_t)it + 1))) break;
      float hgx[NPR], hpx[NPR], hgy[NPR], hpy[NPR];
      double hhx[NPR], hhy[NPR];
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        const bool sb = (cv[2 * q] >> 16) & 1u;
        int jx, jy;
        res_halo(sb ? cv[2 * q + 1] : cv[2 * q], sb ? jv[2 * q + 1] : jv[2 * q], jdflt, of, jx, jy);
        // red neighbours across the faces: their pair's index
        hgx[q] = ld_coh(Grc + (jx >> 1));
        hpx[q] = ld_coh(Grp + (jx >> 1));
        hhx[q] = ld_coh(a.hinv + (jx >> 1));
        hgy[q] = ld_coh(Grc + (jy >> 1));
        hpy[q] = ld_coh(Grp + (jy >> 1));
        hhy[q] = ld_coh(a.hinv + (jy >> 1));
      }
#pragma unroll
      for (int q = 0; q < NPR; ++q)
        if (bface[q]) black(q, hgx[q], hpx[q], hhx[q], hgy[q], hpy[q], hhy[q]);
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        if (!(facem >> q & 1u)) continue;
        const bool sb = (cv[2 * q] >> 16) & 1u;
        st_coh(a.P + (jv[2 * q] >> 1), lp[2 * (q * kResNT + tid) + (sb ? 1 : 0)]);
      }
      if (!(live = finish(acc, PK_DOTS, kSlotD, true))) break;
    }

    // ---- red pass and direction (as k_rb_red_dir_pair): z_i = -p + mu z_{i-1};
    // per pair, the red voxel's p and edge sums, the black voxel's z
    {
      const int tid = res_opaque(jv);
      const float mu = (float)ls.mu;
      double acc[3] = {0.0, 0.0, 0.0};
      float znew[V], hpx[NPR], hzx[NPR], hfx[NPR], hpy[NPR], hzy[NPR], hfy[NPR];
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        const bool sb = (cv[2 * q] >> 16) & 1u;
        int jx, jy;
        res_halo(sb ? cv[2 * q] : cv[2 * q + 1], sb ? jv[2 * q] : jv[2 * q + 1], jdflt, of, jx, jy);
        hpx[q] = ld_coh(a.P + (jx >> 1));  // black neighbours' p at their pair's index
        hzx[q] = ld_coh(Zp + jx);
        hfx[q] = ld_coh(Fc + jx);
        hpy[q] = ld_coh(a.P + (jy >> 1));
        hzy[q] = ld_coh(Zp + jy);
        hfy[q] = ld_coh(Fc + jy);
      }
#pragma unroll
      for (int q = 0; q < NPR; ++q) {
        const bool sb = (cv[2 * q] >> 16) & 1u;
        const uint32_t cb = sb ? cv[2 * q + 1] : cv[2 * q], cr = sb ? cv[2 * q] : cv[2 * q + 1];
        const int l0 = 2 * (q * kResNT + tid), lib = l0 + (sb ? 1 : 0), lir = l0 + (sb ? 0 : 1);
        float zb = 0.f, zr = 0.f;
        if (cb & NB_SELF) {
          zb = -lp[lib] + mu * lz[lib];
          acc[2] += (double)zb * (double)zb * (double)ld[lib];
        }
        if (cr & NB_SELF) {
          const float z0 = lz[lir], f0 = lf[lir];
          float pn[6], zn[6], fn[6];
          double sum = 0.0;
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const bool in = (cr >> (8 + k)) & 1u;
            pn[k] = res_nb(lp, lir, loff[k], in, k < 2 ? hpx[q] : hpy[q]);
            zn[k] = res_nb(lz, lir, loff[k], in, k < 2 ? hzx[q] : hzy[q]);
            fn[k] = res_nb(lf, lir, loff[k], in, k < 2 ? hfx[q] : hfy[q]);
            sum += has_nb(cr, k) ? (double)pn[k] : 0.0;
          }
          const double ip = lh[lir];
          if (!(ip > 0.0)) set_status(a.status, 5);
          const float pj = (float)((double)lgc[lir] * ip + beta * sum * ip);
          zr = -pj + mu * z0;
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const double dz = (double)(zr - (-pn[k] + mu * zn[k]));
            const bool hk = has_nb(cr, k);
            acc[0] += hk ? dz * (double)(f0 - fn[k]) : 0.0;
            acc[1] += hk ? dz * dz : 0.0;
          }
          acc[2] += (double)zr * (double)zr * (double)ld[lir];
        }
        znew[2 * q] = sb ? zr : zb;
        znew[2 * q + 1] = sb ? zb : zr;
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) lz[2 * ((v >> 1) * kResNT + tid) + (v & 1)] = znew[v];
#pragma unroll
      for (int q = 0; q < NPR; ++q)
        if (facem >> q & 1u) st_coh2(Zc + jv[2 * q], znew[2 * q], znew[2 * q + 1]);
      if (!(live = finish(acc, PK_DIR, kSlotR, false))) break;
    }

    // ---- further line-search steps (as k_mls), every voxel
    for (int m = 1; m < nmls && live; ++m) {
      const int tid = res_opaque(jv);
      const float alpha = (float)ls.alpha;
      double acc[2] = {0.0, 0.0};
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (!(cv[v] & NB_SELF)) continue;
        const int li = 2 * ((v >> 1) * kResNT + tid) + (v & 1);
        const float z0 = lz[li];
        float phi, dphi, curv;
        if constexpr (PCN)
          voxel_terms_pc<float, NP>(ea[v], eb[v], lpc, lf[li] + alpha * z0, phi, dphi, curv);
        else
          voxel_terms<float, LR>(ea[v], eb[v], LR, lpc, lf[li] + alpha * z0, phi, dphi, curv);
        acc[0] += (double)z0 * (double)dphi;
        acc[1] += (double)z0 * (double)z0 * (double)curv;
      }
      live = finish(acc, PK_MLS, kSlotM + mslot, false);
      mslot ^= 1;
    }
  }
  // f, z and g of every voxel of the tile for the kernels after this launch
  // (the last iteration's parity; plain stores, ordered by the kernel boundary)
  {
    const int parl = (a.par0 + a.niter - 1) & 1;
#pragma unroll
    for (int q = 0; q < NPR; ++q) {
      const int l0 = 2 * (q * kResNT + (int)threadIdx.x), j0 = jv[2 * q];
      if (j0 < 0) continue;
      *(float2 *)(a.F[parl] + j0) = make_float2(lf[l0], lf[l0 + 1]);
      *(float2 *)(a.Z[parl] + j0) = make_float2(lz[l0], lz[l0 + 1]);
      *(float2 *)(a.G[parl] + j0) = make_float2(lg[parl][l0], lg[parl][l0 + 1]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State s = ls;
    s.kind = PK_NONE;
    s.nparts = 0;
    *a.sout = s;
  }
}

}  // namespace fm
