// IC(0) in natural order (Sec. III-B eq. (precon)) as a pipelined wavefront.
//
// The recurrences
//   forward   P_j = h_j - beta^2 sum_{k lower} 1/P_k,  x_j = (g_j + beta sum_{k lower} x_k) / P_j
//   backward  p_j = x_j + (beta / P_j) sum_{k upper} p_k
// (lower = -x, -y, -z neighbours in the mask, upper = +x, +y, +z) have a
// dependency chain of length nx+ny+nz-2.  The (x, y) plane is cut into 8x8
// column tiles, one wavefront each: lane (a, b) owns column (8ti+a, 8tj+b) and
// at step S handles z = S - a - b (backward: the mirror image), so its -x and
// -y inputs come from lanes t-8 and t-1 of the previous step (cross-lane
// moves) and its -z input from its own previous step.  Tiles exchange their
// boundary columns through the stored x, 1/P (forward) and p (backward)
// arrays, gated by per-tile progress counters (steps completed, published
// every kStepU steps after the stores have completed).
//
// Progress is deadlock-free: a wave takes a ticket from an atomic counter and
// processes the tile of that rank in anti-diagonal order, so it only waits on
// tiles held by waves that started earlier.  Every wait is bounded; on
// expiry the wave records FM_ERR_TIMEOUT and finishes its loop without
// further waiting.  The forward kernel clears the backward kernel's counters
// and the backward kernel the forward's (stream order separates them).
#pragma once

#include "fm_kernels.hpp"

namespace fm {

constexpr int kTile = 8;         // tile edge (8x8 columns = one wavefront)
constexpr int kStepU = 4;        // steps per unrolled group / prefetch distance (2, 3, 6, 8 and 16 measured slower)
constexpr int kSpinLimit = 1 << 16;  // polls per wait (each ~1 us): about 0.1 s

struct Wavefront {
  const int2 *order;     // [ntiles] tile (ti, tj) of each ticket, anti-diagonal order
  int32_t ntx, nty;      // tiles along x and y
  int32_t ntiles;
  uint32_t *ticket_fwd, *ticket_bwd;
  int32_t *prog_fwd, *prog_bwd;  // [ntiles] steps completed
  const int2 *blk[2];    // block red-black: the tiles of colour (ti + tj) mod 2 = 0 and 1
  int32_t nblk[2];
};

__device__ __forceinline__ int load_prog(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (lane 0 polls) until *p >= need; returns the value seen.  Bounded.
__device__ __forceinline__ int wait_prog(const int32_t *p, int need, int cached, int32_t *status, bool &timed_out) {
  if (cached >= need || timed_out) return cached;
  int v = cached;
  if ((threadIdx.x & 63) == 0) {
    int spins = 0;
    v = load_prog(p);
    while (v < need && spins < kSpinLimit) {
      __builtin_amdgcn_s_sleep(1);
      v = load_prog(p);
      ++spins;
    }
    if (v < need) set_status(status, 8);
  }
  v = __builtin_amdgcn_readfirstlane(v);
  if (v < need) timed_out = true;
  return v;
}

__device__ __forceinline__ void publish_prog(int32_t *p, int v) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int take_ticket(uint32_t *counter) {
  int t = 0;
  if ((threadIdx.x & 63) == 0) t = (int)atomicAdd(counter, 1u);
  return __builtin_amdgcn_readfirstlane(t);
}

template <typename T>
__device__ __forceinline__ T shfl_up_t(T v, int d) {
  return __shfl_up(v, (unsigned)d, 64);
}


// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_ic_fwd_wave(IterArgs<T> a, Wavefront w, const T *__restrict__ gsrc) {
  const Geo g = a.geo;
  const State st = take_state<64, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status);
  const int it = a.par;
  const T *__restrict__ gg = gsrc ? gsrc : a.G[it & 1];
  const int ticket = take_ticket(w.ticket_fwd);
  if (ticket >= w.ntiles) {  // counters not reset: refuse rather than index out of range
    set_status(a.status, 8);
    put_state(st, a.sout, PK_NONE, 0);
    return;
  }
  if (ticket == 0 && threadIdx.x == 0) *w.ticket_bwd = 0u;
  if (ticket == 0)
    for (int i = threadIdx.x; i < w.ntiles; i += 64) w.prog_bwd[i] = 0;
  const int2 tile = w.order[ticket];
  const int lane = threadIdx.x, la = lane >> 3, lb = lane & 7;
  const int x = tile.x * kTile + la, y = tile.y * kTile + lb;
  const bool col_ok = x < g.nx && y < g.ny;
  const int nz = g.nz;
  const int64_t jcol = col_ok ? ((int64_t)x * g.ny + y) * nz : 0;
  const int32_t *prog_x = tile.x > 0 ? w.prog_fwd + (tile.x - 1) * w.nty + tile.y : nullptr;
  const int32_t *prog_y = tile.y > 0 ? w.prog_fwd + tile.x * w.nty + (tile.y - 1) : nullptr;
  int32_t *my_prog = w.prog_fwd + tile.x * w.nty + tile.y;
  const double beta = a.beta, b2 = a.beta * a.beta;
  const int nsteps = nz + 2 * (kTile - 1);
  int px = prog_x ? 0 : 1 << 30, py = prog_y ? 0 : 1 << 30;
  bool timed_out = false;
  int bad = 0;
  // ring of prefetched inputs, slot = step % kStepU
  uint32_t rc[kStepU];
  double rbr[kStepU], rbyr[kStepU];
  T rd[kStepU];
  T rg[kStepU], rbx[kStepU], rbyx[kStepU];
  // Every lane issues the same loads at every step (addresses clamped into the
  // arrays, values masked afterwards), so the number of memory operations per
  // step is fixed and the compiler can wait for exactly the slot it consumes
  // instead of draining every outstanding load.  The ring holds the loaded
  // values only: anything computed from them at prefetch time would make the
  // wavefront wait for the load it has just issued.
  auto prefetch = [&](int S, int u) {
    const int z = S - la - lb;
    const int64_t j = jcol + (z < 0 ? 0 : (z >= nz ? nz - 1 : z));
    rc[u] = a.code[j];
    rd[u] = a.D[j];
    rg[u] = gg[j];
    const int64_t jx = (col_ok && la == 0 && x > 0) ? j - g.sx : j;  // tile boundary: the -x neighbour column
    const int64_t jy = (col_ok && lb == 0 && y > 0) ? j - g.sy : j;
    rbr[u] = ld_coh(a.ipiv + jx);
    rbx[u] = ld_coh(a.X + jx);
    rbyr[u] = ld_coh(a.ipiv + jy);
    rbyx[u] = ld_coh(a.X + jy);
  };
  // boundary data of steps [0, kStepU) must be stored by the neighbour tiles
  const int need0 = kStepU + kTile < nsteps ? kStepU + kTile : nsteps;
  if (prog_x) px = wait_prog(prog_x, need0, px, a.status, timed_out);
  if (prog_y) py = wait_prog(prog_y, need0, py, a.status, timed_out);
#pragma unroll
  for (int u = 0; u < kStepU; ++u) prefetch(u, u);
  double r_prev = 0.0, x_prev = 0.0;  // this lane's previous z (same column)
  double r_out = 0.0, x_out = 0.0;    // this lane's value of the previous step
  for (int S0 = 0; S0 < nsteps; S0 += kStepU) {
    const int need = S0 + 2 * kStepU + kTile;  // covers the prefetches of this group
    if (prog_x) px = wait_prog(prog_x, need < nsteps ? need : nsteps, px, a.status, timed_out);
    if (prog_y) py = wait_prog(prog_y, need < nsteps ? need : nsteps, py, a.status, timed_out);
#pragma unroll
    for (int u = 0; u < kStepU; ++u) {
      const int S = S0 + u;
      // values of lanes (a-1, b) and (a, b-1) from the previous step
      const double rx_l = shfl_up_t(r_out, kTile), xx_l = shfl_up_t(x_out, kTile);
      const double ry_l = shfl_up_t(r_out, 1), xy_l = shfl_up_t(x_out, 1);
      const int z = S - la - lb;
      const uint32_t c = rc[u];
      double r_new = 0.0, x_new = 0.0;
      if (col_ok && z >= 0 && z < nz) {
        if (c & NB_SELF) {
          double sr = 0.0, sx = 0.0;
          if (c & NB_XM) {
            sr += la ? rx_l : rbr[u];
            sx += la ? xx_l : (double)rbx[u];
          }
          if (c & NB_YM) {
            sr += lb ? ry_l : rbyr[u];
            sx += lb ? xy_l : (double)rbyx[u];
          }
          if (c & NB_ZM) {
            sr += r_prev;
            sx += x_prev;
          }
          const double piv = ((double)rd[u] + beta * nb_deg(c)) - b2 * sr;
          double ip = 1.0 / piv;
          if (!(piv > 0.0)) {
            bad = 1;
            ip = 0.0;
          }
          r_new = ip;
          x_new = (double)(T)(((double)rg[u] + beta * sx) * ip);
        }
        r_prev = r_new;
        x_prev = x_new;
      }
      {
        // out-of-range lanes store into the padding before voxel 0 (never read as data)
        const bool ok = col_ok && z >= 0 && z < nz;
        const int64_t j = ok ? jcol + z : -1;
        st_coh(a.ipiv + j, r_new);
        st_coh(a.X + j, (T)x_new);
      }
      r_out = r_new;
      x_out = x_new;
      // publish the group before its last prefetch, so the wait for the
      // stores does not also wait for a load issued just before it
      if (u == kStepU - 1) publish_prog(my_prog, S0 + kStepU < nsteps ? S0 + kStepU : nsteps);
      if (S + kStepU < nsteps) prefetch(S + kStepU, u);
    }
  }
  if (bad) set_status(a.status, 5);
  put_state(st, a.sout, PK_NONE, 0);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_ic_bwd_wave(IterArgs<T> a, Wavefront w, const T *__restrict__ gsrc) {
  const Geo g = a.geo;
  const State st = take_state<64, 1>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status);
  const int it = a.par;
  const T *__restrict__ gg = gsrc ? gsrc : a.G[it & 1];
  const T *__restrict__ gp = a.G[(it + 1) & 1];
  const int ticket = take_ticket(w.ticket_bwd);
  if (ticket >= w.ntiles) {
    set_status(a.status, 8);
    put_state(st, a.sout, PK_DOTS, 0);
    return;
  }
  if (ticket == 0 && threadIdx.x == 0) *w.ticket_fwd = 0u;
  if (ticket == 0)
    for (int i = threadIdx.x; i < w.ntiles; i += 64) w.prog_fwd[i] = 0;
  const int2 tile = w.order[w.ntiles - 1 - ticket];  // reverse anti-diagonal order
  const int lane = threadIdx.x, la = lane >> 3, lb = lane & 7;
  const int ra = kTile - 1 - la, rb = kTile - 1 - lb;  // skew of the mirrored sweep
  const int x = tile.x * kTile + la, y = tile.y * kTile + lb;
  const bool col_ok = x < g.nx && y < g.ny;
  const int nz = g.nz;
  const int64_t jcol = col_ok ? ((int64_t)x * g.ny + y) * nz : 0;
  const int32_t *prog_x = tile.x + 1 < w.ntx ? w.prog_bwd + (tile.x + 1) * w.nty + tile.y : nullptr;
  const int32_t *prog_y = tile.y + 1 < w.nty ? w.prog_bwd + tile.x * w.nty + (tile.y + 1) : nullptr;
  int32_t *my_prog = w.prog_bwd + tile.x * w.nty + tile.y;
  const double beta = a.beta;
  const int nsteps = nz + 2 * (kTile - 1);
  int px = prog_x ? 0 : 1 << 30, py = prog_y ? 0 : 1 << 30;
  bool timed_out = false;
  uint32_t rc[kStepU];
  double rip[kStepU];
  T rx[kStepU], rg[kStepU], rgp[kStepU], rbx[kStepU], rby[kStepU];
  // same fixed per-step load pattern as the forward sweep
  auto prefetch = [&](int S, int u) {
    const int z = nz - 1 - (S - ra - rb);
    const int64_t j = jcol + (z < 0 ? 0 : (z >= nz ? nz - 1 : z));
    rc[u] = a.code[j];
    rip[u] = ld_coh(a.ipiv + j);
    rx[u] = ld_coh(a.X + j);
    rg[u] = gg[j];
    rgp[u] = gp[j];
    rbx[u] = ld_coh(a.P + ((col_ok && la == kTile - 1 && x + 1 < g.nx) ? j + g.sx : j));
    rby[u] = ld_coh(a.P + ((col_ok && lb == kTile - 1 && y + 1 < g.ny) ? j + g.sy : j));
  };
  const int need0 = kStepU + kTile < nsteps ? kStepU + kTile : nsteps;
  if (prog_x) px = wait_prog(prog_x, need0, px, a.status, timed_out);
  if (prog_y) py = wait_prog(prog_y, need0, py, a.status, timed_out);
#pragma unroll
  for (int u = 0; u < kStepU; ++u) prefetch(u, u);
  double p_prev = 0.0, p_out = 0.0;
  double acc[2] = {0.0, 0.0};
  for (int S0 = 0; S0 < nsteps; S0 += kStepU) {
    const int need = S0 + 2 * kStepU + kTile;
    if (prog_x) px = wait_prog(prog_x, need < nsteps ? need : nsteps, px, a.status, timed_out);
    if (prog_y) py = wait_prog(prog_y, need < nsteps ? need : nsteps, py, a.status, timed_out);
#pragma unroll
    for (int u = 0; u < kStepU; ++u) {
      const int S = S0 + u;
      // lanes (a+1, b) and (a, b+1) are lanes t+8 and t+1
      const double px_l = __shfl_down(p_out, (unsigned)kTile, 64);
      const double py_l = __shfl_down(p_out, 1u, 64);
      const int z = nz - 1 - (S - ra - rb);
      const uint32_t c = rc[u];
      double p_new = 0.0;
      if (col_ok && z >= 0 && z < nz) {
        if (c & NB_SELF) {
          double s = 0.0;
          if (c & NB_XP) s += (la < kTile - 1) ? px_l : (double)rbx[u];
          if (c & NB_YP) s += (lb < kTile - 1) ? py_l : (double)rby[u];
          if (c & NB_ZP) s += p_prev;
          p_new = (double)(T)((double)rx[u] + beta * s * rip[u]);
          acc[0] += (double)rg[u] * p_new;
          acc[1] += (double)rgp[u] * p_new;
        }
        p_prev = p_new;
      }
      st_coh(a.P + (col_ok && z >= 0 && z < nz ? jcol + z : (int64_t)-1), (T)p_new);  // see the forward sweep
      p_out = p_new;
      if (u == kStepU - 1) publish_prog(my_prog, S0 + kStepU < nsteps ? S0 + kStepU : nsteps);  // as forward
      if (S + kStepU < nsteps) prefetch(S + kStepU, u);
    }
  }
  // per-tile partial sums, indexed by tile so the order is fixed
  store_partials_at<2, 64>(acc, tile.x * w.nty + tile.y, w.ntiles, a.pout);
  put_state(st, a.sout, PK_DOTS, w.ntiles);
}

// ---------------------------------------------------------------------------
// IC(0) in block red-black order: the tiles of one colour ((ti + tj) mod 2,
// colour 0 first) share no face, and inside a tile the order is natural, so
// one launch sweeps every tile of a colour at once, one wavefront per tile as
// above, with no waits between tiles.  A voxel's earlier neighbours are its
// in-tile -x, -y, -z neighbours and, in a colour-1 tile, every neighbour
// across a tile face (colour 0, factored by the previous launch); its later
// neighbours are the in-tile +x, +y, +z ones and, in a colour-0 tile, every
// neighbour across a face.  Forward: colour 0, then colour 1; backward:
// colour 1 (the first half of the dot products), then colour 0 (the rest).

// Per-tile views of the per-voxel arrays for the block sweeps: x-planes
// [q0, q1) of the volume (the tile's planes and one more on each side, all
// that a tile reads or writes) as a raw buffer with 32-bit byte offsets.  The
// hardware's range check reads 0 for an offset at or past the view's end and
// drops a store there; lanes without a voxel, face reads where there is no
// neighbour across the face, and stores of steps outside the column address
// the element one past the view (kPast below) and so need no masking.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_view(const void *base, uint32_t nbytes) {
  // descriptor word 3 of an untyped buffer on gfx9-family GPUs
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nbytes, 0x00020000);
}
__device__ __forceinline__ uint32_t view_u8(__amdgpu_buffer_rsrc_t r, uint32_t e) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, e, 0, 0);
}
__device__ __forceinline__ float view_ld(__amdgpu_buffer_rsrc_t r, uint32_t e, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4u, 0, 0));
}
__device__ __forceinline__ double view_ld(__amdgpu_buffer_rsrc_t r, uint32_t e, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8u, 0, 0));
}
__device__ __forceinline__ void view_st(__amdgpu_buffer_rsrc_t r, uint32_t e, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, e * 4u, 0, 0);
}
__device__ __forceinline__ void view_st(__amdgpu_buffer_rsrc_t r, uint32_t e, double v) {
  using B64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, v), r, e * 8u, 0, 0);
}

// The views and lane geometry of one tile (both sweeps).  Element indices are
// relative to plane q0; the host keeps ny * nz * 80 (10 planes of 8-byte
// elements) below 2^30, so no offset computed here wraps.
struct TileView {
  int la, lb;
  bool col_ok;
  uint32_t past;    // one past the view: reads 0, stores dropped
  uint32_t e0;      // this lane's column at z = 0 (past for a lane outside the volume)
  uint32_t dx, dy;  // offset to the neighbour across an x / y tile face, or one that lands past the view
  int64_t jq;       // voxel index of the view's first element
  uint32_t nq;      // elements in the view
};

__device__ __forceinline__ TileView tile_view(const Geo &g, int2 tile, bool faces) {
  TileView v;
  v.la = (int)threadIdx.x >> 3;
  v.lb = (int)threadIdx.x & 7;
  const int x = tile.x * kTile + v.la, y = tile.y * kTile + v.lb;
  v.col_ok = x < g.nx && y < g.ny;
  const int q0 = max(0, tile.x * kTile - 1), q1 = min(g.nx, tile.x * kTile + kTile + 1);
  v.jq = (int64_t)q0 * g.sx;
  v.nq = (uint32_t)((int64_t)(q1 - q0) * g.sx);
  v.past = v.nq;
  v.e0 = v.col_ok ? (uint32_t)((int64_t)(x - q0) * g.sx + (int64_t)y * g.sy) : v.past;
  // e0 + z + far >= past for every z >= 0: a face read with no neighbour reads 0
  const uint32_t far = v.nq;
  const bool fx = faces && v.col_ok && ((v.la == 0 && x > 0) || (v.la == kTile - 1 && x + 1 < g.nx));
  const bool fy = faces && v.col_ok && ((v.lb == 0 && y > 0) || (v.lb == kTile - 1 && y + 1 < g.ny));
  v.dx = fx ? (uint32_t)(v.la == 0 ? -g.sx : g.sx) : far;
  v.dy = fy ? (uint32_t)(v.lb == 0 ? -g.sy : g.sy) : far;
  return v;
}

// Prefetch distance of the block sweeps, in steps.  With one wavefront per CU
// there is no occupancy to lose: 16 measured faster than 8, 12 and 24.
constexpr int kStepB = 16;

template <typename T>
__global__ __launch_bounds__(64) void k_icb_fwd(IterArgs<T> a, Wavefront w, const T *__restrict__ gsrc, int colour) {
  const Geo g = a.geo;
  const State st = take_state<64, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status);
  const T *__restrict__ gg = gsrc ? gsrc : a.G[a.par & 1];
  // a colour-1 tile's neighbours across its faces come earlier (colour 0)
  const TileView v = tile_view(g, w.blk[colour][blockIdx.x], colour == 1);
  const int la = v.la, lb = v.lb, nz = g.nz;
  const auto vcode = plane_view(a.code + v.jq, v.nq), vd = plane_view(a.D + v.jq, v.nq * (uint32_t)sizeof(T));
  const auto vg = plane_view(gg + v.jq, v.nq * (uint32_t)sizeof(T));
  const auto vip = plane_view(a.ipiv + v.jq, v.nq * 8u), vx = plane_view(a.X + v.jq, v.nq * (uint32_t)sizeof(T));
  const double beta = a.beta, b2 = a.beta * a.beta;
  const int nsteps = nz + 2 * (kTile - 1);
  bool bad = false;
  uint32_t rc[kStepB];
  double rbr[kStepB], rbyr[kStepB];
  T rd[kStepB], rg[kStepB], rbx[kStepB], rbyx[kStepB];
  // raw loads only (z clamped into the column; the step masks what is outside it)
  auto prefetch = [&](int S, int u) {
    const uint32_t e = v.e0 + (uint32_t)min(max(S - la - lb, 0), nz - 1);
    rc[u] = view_u8(vcode, e);
    rd[u] = view_ld(vd, e, T());
    rg[u] = view_ld(vg, e, T());
    rbr[u] = view_ld(vip, e + v.dx, double());
    rbx[u] = view_ld(vx, e + v.dx, T());
    rbyr[u] = view_ld(vip, e + v.dy, double());
    rbyx[u] = view_ld(vx, e + v.dy, T());
  };
#pragma unroll
  for (int u = 0; u < kStepB; ++u) prefetch(u, u);
  double r_prev = 0.0, x_prev = 0.0, r_out = 0.0, x_out = 0.0;
  for (int S0 = 0; S0 < nsteps; S0 += kStepB) {
#pragma unroll
    for (int u = 0; u < kStepB; ++u) {
      const int S = S0 + u;
      const double rx_l = shfl_up_t(r_out, kTile), xx_l = shfl_up_t(x_out, kTile);
      // lane t-1 is in the same DPP row for every lane with lb > 0
      const double ry_l = dpp_d<0x111>(r_out), xy_l = dpp_d<0x111>(x_out);  // row_shr:1
      const int z = S - la - lb;
      const bool inr = v.col_ok && z >= 0 && z < nz;
      const uint32_t c = inr ? rc[u] : 0u;
      const bool self = (c & NB_SELF) != 0;
      // earlier neighbours in the order -x, +x, -y, +y, -z, each term 0 where
      // there is none: a voxel outside the mask holds 0 in 1/P and x (its lane
      // stores 0) and a face read with no neighbour reads 0.  A lane's one x
      // face is its -x neighbour (la = 0, in-tile term 0) or its +x one
      // (la = 7), so adding it after the in-tile term keeps that order; the
      // same for y.
      double sr = 0.0, sx = 0.0;
      sr += la ? rx_l : 0.0;
      sx += la ? xx_l : 0.0;
      sr += rbr[u];
      sx += (double)rbx[u];
      sr += lb ? ry_l : 0.0;
      sx += lb ? xy_l : 0.0;
      sr += rbyr[u];
      sx += (double)rbyx[u];
      sr += r_prev;
      sx += x_prev;
      const double piv = ((double)rd[u] + beta * nb_deg(c)) - b2 * sr;
      const bool pos = piv > 0.0;
      bad |= self && !pos;
      const double r_new = (self && pos) ? 1.0 / piv : 0.0;
      const double x_new = self ? (double)(T)(((double)rg[u] + beta * sx) * r_new) : 0.0;
      r_prev = r_new;
      x_prev = x_new;
      const uint32_t es = inr ? v.e0 + (uint32_t)z : v.past;
      view_st(vip, es, r_new);
      view_st(vx, es, (T)x_new);
      r_out = r_new;
      x_out = x_new;
      if (S + kStepB < nsteps) prefetch(S + kStepB, u);
    }
  }
  if (bad) set_status(a.status, 5);
  put_state(st, a.sout, PK_NONE, 0);
}

template <typename T>
__global__ __launch_bounds__(64) void k_icb_bwd(IterArgs<T> a, Wavefront w, const T *__restrict__ gsrc, int colour) {
  const Geo g = a.geo;
  const State st = take_state<64, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status);
  const T *__restrict__ gg = gsrc ? gsrc : a.G[a.par & 1];
  const T *__restrict__ gp = a.G[(a.par + 1) & 1];
  const bool first = colour == 0;  // its neighbours across the faces come later
  const TileView v = tile_view(g, w.blk[colour][blockIdx.x], first);
  const int la = v.la, lb = v.lb, nz = g.nz;
  const int ra = kTile - 1 - la, rb = kTile - 1 - lb;  // skew of the mirrored sweep
  const uint32_t nt = v.nq * (uint32_t)sizeof(T);
  const auto vcode = plane_view(a.code + v.jq, v.nq), vip = plane_view(a.ipiv + v.jq, v.nq * 8u);
  const auto vx = plane_view(a.X + v.jq, nt), vg = plane_view(gg + v.jq, nt), vgp = plane_view(gp + v.jq, nt);
  const auto vp = plane_view(a.P + v.jq, nt);
  const double beta = a.beta;
  const int nsteps = nz + 2 * (kTile - 1);
  uint32_t rc[kStepB];
  double rip[kStepB];
  T rx[kStepB], rg[kStepB], rgp[kStepB], rbx[kStepB], rby[kStepB];
  auto prefetch = [&](int S, int u) {
    const uint32_t e = v.e0 + (uint32_t)min(max(nz - 1 - (S - ra - rb), 0), nz - 1);
    rc[u] = view_u8(vcode, e);
    rip[u] = view_ld(vip, e, double());
    rx[u] = view_ld(vx, e, T());
    rg[u] = view_ld(vg, e, T());
    rgp[u] = view_ld(vgp, e, T());
    rbx[u] = view_ld(vp, e + v.dx, T());
    rby[u] = view_ld(vp, e + v.dy, T());
  };
#pragma unroll
  for (int u = 0; u < kStepB; ++u) prefetch(u, u);
  double p_prev = 0.0, p_out = 0.0;
  double acc[2] = {0.0, 0.0};
  for (int S0 = 0; S0 < nsteps; S0 += kStepB) {
#pragma unroll
    for (int u = 0; u < kStepB; ++u) {
      const int S = S0 + u;
      const double px_l = __shfl_down(p_out, (unsigned)kTile, 64);
      // lane t+1 is in the same DPP row for every lane with lb < 7
      const double py_l = dpp_d<0x101>(p_out);  // row_shl:1
      const int z = nz - 1 - (S - ra - rb);
      const bool inr = v.col_ok && z >= 0 && z < nz;
      const uint32_t c = inr ? rc[u] : 0u;
      const bool self = (c & NB_SELF) != 0;
      // later neighbours in the order -x, +x, -y, +y, +z (p is 0 outside the
      // mask, a face read with no neighbour reads 0)
      // (a lane's one x face, -x at la = 0 or +x at la = 7, added before the
      // in-tile +x term keeps that order; the same for y)
      double s = 0.0;
      s += (double)rbx[u];
      s += la < kTile - 1 ? px_l : 0.0;
      s += (double)rby[u];
      s += lb < kTile - 1 ? py_l : 0.0;
      s += p_prev;
      const double p_new = self ? (double)(T)((double)rx[u] + beta * s * rip[u]) : 0.0;
      acc[0] += (self ? (double)rg[u] : 0.0) * p_new;
      acc[1] += (self ? (double)rgp[u] : 0.0) * p_new;
      p_prev = p_new;
      view_st(vp, inr ? v.e0 + (uint32_t)z : v.past, (T)p_new);
      p_out = p_new;
      if (S + kStepB < nsteps) prefetch(S + kStepB, u);
    }
  }
  store_partials_at<2, 64>(acc, (int)blockIdx.x, (int)gridDim.x, a.pout);
  put_state(st, a.sout, first ? PK_DOTS : PK_DOTS_A, (int)gridDim.x);
}

}  // namespace fm
