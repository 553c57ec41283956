// Plane-marching tiles of the red-black passes (even column lengths).
//
// A workgroup owns a strip of ty whole columns (all of z) and walks a run of
// xc planes along x.  Per plane, thread slots hold voxel pairs (z even,
// z odd): one black and one red voxel, the black one first when x + y is odd.
// A voxel's six neighbours all have the other colour; they come from
//   -x, +x  the same slot one plane back / ahead, kept in registers as the
//           strip marches, so each plane is fetched once per strip;
//   -y, +y  an LDS copy of the plane's values of that colour, with one halo
//           column on each side of the strip, loaded by the first nz threads;
//   -z, +z  the pair's partner and the neighbouring pair's voxel (LDS).
// The arithmetic, the neighbour order and the outputs are those of
// k_rb_black_pair and k_rb_red_dir_pair; only the order in which voxels add
// to the partial sums differs.  Planes are fetched kTileDepth ahead into a
// ring of registers, so that loads are in flight across the barrier and the
// arithmetic of the planes before them; the LDS copy alternates between two
// buffers, so one barrier per plane suffices.  One pair slot per thread and
// two planes ahead keep the kernels at 4 waves per SIMD (about 120 VGPRs);
// two slots per thread or deeper rings cost occupancy and measured slower.
#pragma once

#include "fm_stream.hpp"

namespace fm {

#ifndef FM_TILE_PPT
#define FM_TILE_PPT 1
#endif
#ifndef FM_TILE_DEPTH
#define FM_TILE_DEPTH 2
#endif
constexpr int kTilePPT = FM_TILE_PPT;       // pair slots per thread
constexpr int kTileDepth = FM_TILE_DEPTH;   // planes fetched ahead of the current one (>= 1)
constexpr int kTileSlots = kTilePPT * kNT;  // pair slots of a workgroup per plane
constexpr int kTileMaxNz = kNT;             // the two halo columns hold nz pairs, one per thread
constexpr int kTileLds = kTileSlots + kTileMaxNz;  // LDS entries per buffer, halo included
static_assert(kTileDepth >= 1, "the +x neighbour plane must be in registers");

// Plane-march shape of a volume: columns per strip, planes per run, strips, grid.
struct TileShape {
  int ty, xc, nyt, grid;
};

// The shape a batched volume's descriptor holds.
__device__ __forceinline__ TileShape tile_of(const VolDesc &d) { return TileShape{d.tty, d.txc, d.tnyt, 0}; }

// A workgroup's strip and run, and this thread's slots in them.
struct TileSlots {
  int y0, x0, x1, nzp, ty;
  int cy[kTilePPT], zq[kTilePPT];  // column of the strip (LDS column cy + 1), pair
  bool ok[kTilePPT];
  int hy, hz, he;  // halo slot: column y0 - 1 (LDS column 0) or y0 + ty (LDS column ty + 1)
  bool hs, hok;    // this thread holds a halo slot; that column is in the volume
};

// Workgroups are dealt to the chip's XCDs in turn (workgroup i to XCD i mod
// kXcds), each with its own L2.  The tile index is remapped so that every XCD
// owns a contiguous range of strips and runs: the halo columns and planes a
// workgroup shares with its neighbours are then fetched into the same L2.
constexpr int kXcds = 8;

// Workgroup bl of the nb a volume has (a batched launch may give a volume more
// workgroups than its tiles: the surplus ones own no plane and only take part
// in the partial sums).  The XCD remap applies where the volume's workgroups
// start at a multiple of kXcds and come in multiples of it.
__device__ __forceinline__ TileSlots tile_slots(const Geo &g, const TileShape &ts, int bl, int nb, int b0) {
  TileSlots t;
  t.nzp = g.nz >> 1;
  t.ty = ts.ty;
  if (nb % kXcds == 0 && b0 % kXcds == 0) bl = (bl % kXcds) * (nb / kXcds) + bl / kXcds;
  t.y0 = (bl % ts.nyt) * ts.ty;
  t.x0 = (bl / ts.nyt) * ts.xc;
  const bool run = t.x0 < g.nx;
  t.x1 = !run ? t.x0 : (t.x0 + ts.xc < g.nx ? t.x0 + ts.xc : g.nx);
#pragma unroll
  for (int v = 0; v < kTilePPT; ++v) {
    const int s = (int)threadIdx.x + v * kNT;
    t.cy[v] = s / t.nzp;
    t.zq[v] = s - t.cy[v] * t.nzp;
    t.ok[v] = run && t.cy[v] < t.ty && t.y0 + t.cy[v] < g.ny;
  }
  const int side = (int)threadIdx.x / t.nzp;
  t.hz = (int)threadIdx.x - side * t.nzp;
  t.hs = side < 2;
  t.hy = side == 0 ? t.y0 - 1 : t.y0 + t.ty;
  t.hok = run && t.hs && t.hy >= 0 && t.hy < g.ny;
  t.he = (side == 0 ? 0 : t.ty + 1) * t.nzp + t.hz;
  return t;
}

// Plane p is fetched for a slot if it is in the volume and at most one past the run
// (the +x neighbour of the run's last plane); for a halo slot only inside the run.
__device__ __forceinline__ bool tile_need(const Geo &g, const TileSlots &t, int p) { return p < g.nx && p <= t.x1; }

// ---------------------------------------------------------------------------
// Black pass (Sec. III-B, the black half of the red-black IC(0) factor and its
// forward/backward solve): p_b for every black voxel from its six red
// neighbours' g, g_prev and 1/h, plus the partial sums of g^T p and
// g_prev^T p over all voxels.

template <typename T>
struct TileB {   // one slot's pair on one plane
  uint32_t c2;   // both codes (first voxel in the low byte)
  T gb, gpb, db; // g, g_prev, D of the black voxel
  T gr, gpr;     // g, g_prev of the red voxel
  double hr;     // 1/h of the red voxel
};

template <typename T>
struct TileBH {  // a halo pair's red voxel
  T gr, gpr;
  double hr;
};

template <typename T>
__device__ __forceinline__ TileB<T> tile_b_load(const VArgs<T> &a, const Geo &g, int x, int y, int zp, bool ok) {
  TileB<T> t{};
  if (!ok) return t;
  const int j0 = (x * g.ny + y) * g.nz + 2 * zp;
  const bool fb = ((x + y) & 1) != 0;
  t.c2 = *reinterpret_cast<const uint16_t *>(a.code + j0);
  const Duo<T> g2 = ld_duo(a.Gc, j0), gp2 = ld_duo(a.Gp, j0), d2 = ld_duo(a.D, j0);
  t.gb = fb ? g2.v0 : g2.v1;
  t.gr = fb ? g2.v1 : g2.v0;
  t.gpb = fb ? gp2.v0 : gp2.v1;
  t.gpr = fb ? gp2.v1 : gp2.v0;
  t.db = fb ? d2.v0 : d2.v1;
  t.hr = a.hinv[j0 >> 1];
  return t;
}

template <typename T>
__device__ __forceinline__ TileBH<T> tile_b_halo(const VArgs<T> &a, const Geo &g, int x, int y, int zp, bool ok) {
  TileBH<T> t{};
  if (!ok) return t;
  const int j0 = (x * g.ny + y) * g.nz + 2 * zp;
  const bool fb = ((x + y) & 1) != 0;
  const Duo<T> g2 = ld_duo(a.Gc, j0), gp2 = ld_duo(a.Gp, j0);
  t.gr = fb ? g2.v1 : g2.v0;
  t.gpr = fb ? gp2.v1 : gp2.v0;
  t.hr = a.hinv[j0 >> 1];
  return t;
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_rb_black_tile(IterArgs<T> a0, TileShape ts) {
  __shared__ double lh[2][kTileLds];
  __shared__ T lg[2][kTileLds], lgp[2][kTileLds];
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const TileSlots t = tile_slots(g, BATCH ? tile_of(a0.bt.vol[vw.vol]) : ts, vw.bl, vw.nb, BATCH ? vw.pfirst : 0);
  const int nzp = t.nzp;
  TileB<T> q[kTileDepth + 1][kTilePPT];  // planes x .. x + kTileDepth
  TileBH<T> hq[kTileDepth + 1];
  T prg[kTilePPT], prgp[kTilePPT];  // red g, g_prev one plane back
  double prh[kTilePPT];
#pragma unroll
  for (int v = 0; v < kTilePPT; ++v) {
    const TileB<T> pv = tile_b_load(a, g, t.x0 - 1, t.y0 + t.cy[v], t.zq[v], t.ok[v] && t.x0 > 0);
    prg[v] = pv.gr;
    prgp[v] = pv.gpr;
    prh[v] = pv.hr;
#pragma unroll
    for (int d = 0; d < kTileDepth; ++d)
      q[d][v] = tile_b_load(a, g, t.x0 + d, t.y0 + t.cy[v], t.zq[v], t.ok[v] && tile_need(g, t, t.x0 + d));
  }
#pragma unroll
  for (int d = 0; d < kTileDepth; ++d) hq[d] = tile_b_halo(a, g, t.x0 + d, t.hy, t.hz, t.hok && t.x0 + d < t.x1);
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow,
                                      vw.leader);
  const double beta = a.beta, b2 = a.beta * a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for (int x = t.x0; x < t.x1; ++x) {
    const int b = (x - t.x0) & 1;
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v)
      if (t.ok[v]) {
        const int e = (t.cy[v] + 1) * nzp + t.zq[v];
        lg[b][e] = q[0][v].gr;
        lgp[b][e] = q[0][v].gpr;
        lh[b][e] = q[0][v].hr;
      }
    if (t.hs) {
      lg[b][t.he] = hq[0].gr;
      lgp[b][t.he] = hq[0].gpr;
      lh[b][t.he] = hq[0].hr;
    }
    // plane x + kTileDepth is in flight during this plane's barrier and arithmetic
    const int xf = x + kTileDepth;
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v)
      q[kTileDepth][v] = tile_b_load(a, g, xf, t.y0 + t.cy[v], t.zq[v], t.ok[v] && tile_need(g, t, xf));
    hq[kTileDepth] = tile_b_halo(a, g, xf, t.hy, t.hz, t.hok && xf < t.x1);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v) {
      if (!t.ok[v]) continue;
      const TileB<T> &c = q[0][v];
      const TileB<T> &n = q[1][v];
      const int y = t.y0 + t.cy[v];
      const bool fb = ((x + y) & 1) != 0;
      const uint32_t cv = fb ? (c.c2 & 0xffu) : (c.c2 >> 8), cr = fb ? (c.c2 >> 8) : (c.c2 & 0xffu);
      if (cr & NB_SELF) {
        const double gh = (double)c.gr * c.hr;
        acc[0] += (double)c.gr * gh;
        acc[1] += (double)c.gpr * gh;
      }
      if (!(cv & NB_SELF)) continue;
      const int e = (t.cy[v] + 1) * nzp + t.zq[v];
      // -z / +z: the previous pair's red voxel and the partner (black first),
      // or the partner and the next pair's red voxel (red first)
      const int ez = fb ? (t.zq[v] > 0 ? e - 1 : e) : (t.zq[v] + 1 < nzp ? e + 1 : e);
      const double hn[6] = {prh[v], n.hr, lh[b][e - nzp], lh[b][e + nzp], fb ? lh[b][ez] : c.hr,
                            fb ? c.hr : lh[b][ez]};
      const T gn[6] = {prg[v], n.gr, lg[b][e - nzp], lg[b][e + nzp], fb ? lg[b][ez] : c.gr, fb ? c.gr : lg[b][ez]};
      const T gpn[6] = {prgp[v], n.gpr, lgp[b][e - nzp], lgp[b][e + nzp], fb ? lgp[b][ez] : c.gpr,
                        fb ? c.gpr : lgp[b][ez]};
      const double h = (double)c.db + beta * nb_deg(cv);
      double sp = 0.0, sxv = 0.0, syp = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (has_nb(cv, k)) {
          sp += hn[k];
          sxv += (double)gn[k] * hn[k];
          syp += (double)gpn[k] * hn[k];
        }
      const double piv = h - b2 * sp;
      double ip = 1.0 / piv;
      if (!(piv > 0.0)) {
        bad = 1;
        ip = 0.0;
      }
      const double yb = (double)c.gb + beta * sxv;
      const double xv = yb * ip;
      a.P[((x * g.ny + y) * g.nz >> 1) + t.zq[v]] = (T)xv;
      acc[0] += yb * xv;
      acc[1] += ((double)c.gpb + beta * syp) * xv;
    }
    // march one plane along the ring
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v) {
      prg[v] = q[0][v].gr;
      prgp[v] = q[0][v].gpr;
      prh[v] = q[0][v].hr;
#pragma unroll
      for (int d = 0; d < kTileDepth; ++d) q[d][v] = q[d + 1][v];
    }
#pragma unroll
    for (int d = 0; d < kTileDepth; ++d) hq[d] = hq[d + 1];
  }
  if (bad) set_status(a.status, 5);
  store_partials<2, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DOTS, vw.nb, vw.leader);
}

// ---------------------------------------------------------------------------
// Red pass fused with the direction (Sec. III-B, the red half of the backward
// solve; Sec. III eq. (ncg) for z; the line-search setup sums): p_r from the
// six black neighbours' p, then z = -p + mu z_prev for both voxels of the
// pair, and the partial sums of z^T C^T C f, ||C z||^2 and z^T D z.

template <typename T>
struct TileR {      // one slot's pair on one plane
  uint32_t c2;      // both codes (first voxel in the low byte)
  T pb, zb, fb, db; // p, z_prev, f, D of the black voxel
  T gr, zr, fr, dr; // g, z_prev, f, D of the red voxel
  double hr;        // 1/h of the red voxel
};

template <typename T>
struct TileRH {  // a halo pair's black voxel
  T pb, zb, fb;
};

template <typename T>
__device__ __forceinline__ TileR<T> tile_r_load(const VArgs<T> &a, const Geo &g, int x, int y, int zp, bool ok) {
  TileR<T> t{};
  if (!ok) return t;
  const int j0 = (x * g.ny + y) * g.nz + 2 * zp;
  const bool fb = ((x + y) & 1) != 0;
  t.c2 = *reinterpret_cast<const uint16_t *>(a.code + j0);
  const Duo<T> z2 = ld_duo(a.Zp, j0), f2 = ld_duo(a.Fc, j0), d2 = ld_duo(a.D, j0), g2 = ld_duo(a.Gc, j0);
  t.pb = a.P[j0 >> 1];
  t.zb = fb ? z2.v0 : z2.v1;
  t.zr = fb ? z2.v1 : z2.v0;
  t.fb = fb ? f2.v0 : f2.v1;
  t.fr = fb ? f2.v1 : f2.v0;
  t.db = fb ? d2.v0 : d2.v1;
  t.dr = fb ? d2.v1 : d2.v0;
  t.gr = fb ? g2.v1 : g2.v0;
  t.hr = a.hinv[j0 >> 1];
  return t;
}

template <typename T>
__device__ __forceinline__ TileRH<T> tile_r_halo(const VArgs<T> &a, const Geo &g, int x, int y, int zp, bool ok) {
  TileRH<T> t{};
  if (!ok) return t;
  const int j0 = (x * g.ny + y) * g.nz + 2 * zp;
  const bool fb = ((x + y) & 1) != 0;
  const Duo<T> z2 = ld_duo(a.Zp, j0), f2 = ld_duo(a.Fc, j0);
  t.pb = a.P[j0 >> 1];
  t.zb = fb ? z2.v0 : z2.v1;
  t.fb = fb ? f2.v0 : f2.v1;
  return t;
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_rb_red_dir_tile(IterArgs<T> a0, TileShape ts) {
  __shared__ T lp[2][kTileLds], lz[2][kTileLds], lf[2][kTileLds];
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const TileSlots t = tile_slots(g, BATCH ? tile_of(a0.bt.vol[vw.vol]) : ts, vw.bl, vw.nb, BATCH ? vw.pfirst : 0);
  const int nzp = t.nzp;
  TileR<T> q[kTileDepth + 1][kTilePPT];  // planes x .. x + kTileDepth
  TileRH<T> hq[kTileDepth + 1];
  T prp[kTilePPT], prz[kTilePPT], prf[kTilePPT];  // black p, z_prev, f one plane back
#pragma unroll
  for (int v = 0; v < kTilePPT; ++v) {
    const TileR<T> pv = tile_r_load(a, g, t.x0 - 1, t.y0 + t.cy[v], t.zq[v], t.ok[v] && t.x0 > 0);
    prp[v] = pv.pb;
    prz[v] = pv.zb;
    prf[v] = pv.fb;
#pragma unroll
    for (int d = 0; d < kTileDepth; ++d)
      q[d][v] = tile_r_load(a, g, t.x0 + d, t.y0 + t.cy[v], t.zq[v], t.ok[v] && tile_need(g, t, t.x0 + d));
  }
#pragma unroll
  for (int d = 0; d < kTileDepth; ++d) hq[d] = tile_r_halo(a, g, t.x0 + d, t.hy, t.hz, t.hok && t.x0 + d < t.x1);
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow,
                                      vw.leader);
  const double beta = a.beta;
  const T mu = (T)st.mu;
  double acc[3] = {0.0, 0.0, 0.0};
  int bad = 0;
  for (int x = t.x0; x < t.x1; ++x) {
    const int b = (x - t.x0) & 1;
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v)
      if (t.ok[v]) {
        const int e = (t.cy[v] + 1) * nzp + t.zq[v];
        lp[b][e] = q[0][v].pb;
        lz[b][e] = q[0][v].zb;
        lf[b][e] = q[0][v].fb;
      }
    if (t.hs) {
      lp[b][t.he] = hq[0].pb;
      lz[b][t.he] = hq[0].zb;
      lf[b][t.he] = hq[0].fb;
    }
    const int xf = x + kTileDepth;
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v)
      q[kTileDepth][v] = tile_r_load(a, g, xf, t.y0 + t.cy[v], t.zq[v], t.ok[v] && tile_need(g, t, xf));
    hq[kTileDepth] = tile_r_halo(a, g, xf, t.hy, t.hz, t.hok && xf < t.x1);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v) {
      if (!t.ok[v]) continue;
      const TileR<T> &c = q[0][v];
      const TileR<T> &n = q[1][v];
      const int y = t.y0 + t.cy[v];
      const bool fb = ((x + y) & 1) != 0;
      const uint32_t cb = fb ? (c.c2 & 0xffu) : (c.c2 >> 8), cv = fb ? (c.c2 >> 8) : (c.c2 & 0xffu);
      T zrv = T(0), zbv = T(0);
      if (cv & NB_SELF) {
        const int e = (t.cy[v] + 1) * nzp + t.zq[v];
        // -z / +z: the partner and the next pair's black voxel (black first),
        // or the previous pair's black voxel and the partner (red first)
        const int ez = fb ? (t.zq[v] + 1 < nzp ? e + 1 : e) : (t.zq[v] > 0 ? e - 1 : e);
        const T pn[6] = {prp[v], n.pb, lp[b][e - nzp], lp[b][e + nzp], fb ? c.pb : lp[b][ez], fb ? lp[b][ez] : c.pb};
        const T zn[6] = {prz[v], n.zb, lz[b][e - nzp], lz[b][e + nzp], fb ? c.zb : lz[b][ez], fb ? lz[b][ez] : c.zb};
        const T fn[6] = {prf[v], n.fb, lf[b][e - nzp], lf[b][e + nzp], fb ? c.fb : lf[b][ez], fb ? lf[b][ez] : c.fb};
        double sp = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(cv, k)) sp += (double)pn[k];
        const double ip = c.hr;
        if (!(ip > 0.0)) bad = 1;
        const T pj = (T)((double)c.gr * ip + beta * sp * ip);
        zrv = -pj + mu * c.zr;
        acc[2] += (double)zrv * (double)zrv * (double)c.dr;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (has_nb(cv, k)) {
            const double dz = (double)(zrv - (-pn[k] + mu * zn[k]));
            acc[0] += dz * (double)(c.fr - fn[k]);
            acc[1] += dz * dz;
          }
      }
      if (cb & NB_SELF) {
        zbv = -c.pb + mu * c.zb;
        acc[2] += (double)zbv * (double)zbv * (double)c.db;
      }
      Duo<T> out;
      out.v0 = fb ? zbv : zrv;
      out.v1 = fb ? zrv : zbv;
      *reinterpret_cast<Duo<T> *>(a.Zc + (x * g.ny + y) * g.nz + 2 * t.zq[v]) = out;
    }
#pragma unroll
    for (int v = 0; v < kTilePPT; ++v) {
      prp[v] = q[0][v].pb;
      prz[v] = q[0][v].zb;
      prf[v] = q[0][v].fb;
#pragma unroll
      for (int d = 0; d < kTileDepth; ++d) q[d][v] = q[d + 1][v];
    }
#pragma unroll
    for (int d = 0; d < kTileDepth; ++d) hq[d] = hq[d + 1];
  }
  if (bad) set_status(a.status, 5);
  store_partials<3, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_DIR, vw.nb, vw.leader);
}

}  // namespace fm
