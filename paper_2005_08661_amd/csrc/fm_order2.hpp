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
// with r the row indicators.  Passes for single volumes with the diagonal,
// identity or IC(0) (three-colour order) preconditioner; voxel-order arrays
// are padded by two x-planes so that the +-2 neighbour addresses stay in
// bounds, and the arrays of three-colour IC(0) are colour-major (below).
#pragma once

#include "fm_stream.hpp"

namespace fm {

// Voxels per thread of the gradient and direction passes (FP32 working type).
// One voxel per thread in the gradient pass (its 26 neighbour values and the
// echoes of a second voxel cost occupancy): 24.2 -> 19.5 us at 128x128x64.
#ifndef FM_V_GRAD2
#define FM_V_GRAD2 1
#endif
#ifndef FM_V_DIR2
#define FM_V_DIR2 FM_VPT32
#endif

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

// Quotient and remainder of 0 <= j < 2^31 by d > 0 through a float64
// reciprocal: the rounded product is within 2^-21 of j / d, so its truncation
// is off by at most one, which one correction step on the remainder removes.
struct Div {
  int d;
  double inv;
  __device__ __forceinline__ explicit Div(int d_) : d(d_), inv(1.0 / (double)d_) {}
  __device__ __forceinline__ int operator()(int j, int &r) const {
    int q = (int)((double)j * inv);
    r = j - q * d;
    if (r < 0) {
      --q;
      r += d;
    }
    if (r >= d) {
      ++q;
      r -= d;
    }
    return q;
  }
};

// Colour-major layout of the arrays the three-colour passes share (g, g_prev,
// D, p, the inverted pivots, y, y', the neighbour codes and diag(C^T C)):
// block c holds the voxels of colour c, voxel (x, y, z) at slot
// (x + 2) plane + y m + z / 3 of it, with m = ceil(nz / 3) slots per z-column,
// plane = ny m, and two padding planes on either side of x.  Along x and y the
// +-1 and +-2 neighbours of a colour-c voxel sit at the same within-column slot
// of a neighbouring column in block c +- 1 (the +1 and -2 neighbours in block
// c + 1, the -1 and +2 ones in block c - 1); along z the slot moves by at most
// one, by an amount fixed by z mod 3.  A pass over one colour therefore reads
// and writes that colour's block contiguously and the two others at a few
// constant strides, and touches no cache line of the other colours' values.
struct Cm {
  int m, plane, S;  // slots per column, slots per x-plane, elements per colour block
  Div dz, dy;       // division by nz and ny
  __device__ __forceinline__ explicit Cm(const Geo &g)
      : m((g.nz + 2) / 3), plane(g.ny * ((g.nz + 2) / 3)), S((g.nx + 4) * g.ny * ((g.nz + 2) / 3)), dz(g.nz),
        dy(g.ny) {}
  // element of slot t (0 <= t < nx plane) of colour c
  __device__ __forceinline__ int at(int c, int t) const { return c * S + 2 * plane + t; }
  // coordinates of voxel j
  __device__ __forceinline__ void xyz(int j, int &x, int &y, int &z) const {
    const int yx = dz(j, z);
    x = dy(yx, y);
  }
  // element of voxel j
  __device__ __forceinline__ int of(int j) const {
    int x, y, z;
    xyz(j, x, y, z);
    return ((x + y + z) % 3) * S + (x + 2) * plane + y * m + z / 3;
  }
};

// Gradient pass with the second-order regulariser (as k_grad): also loads the
// +-2 neighbours of f and z and the neighbour codes; g and D go to their
// colour-major elements in three-colour IC(0) plans (and D to its voxel-order
// copy, which the direction pass reads).
template <typename T, int LMAX, bool BATCH = false>
__global__ __launch_bounds__(kNT) void k_grad2(IterArgs<T> a0) {
  constexpr int V = Vk<T, FM_V_GRAD2>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
  const Geo g = a.geo;
  const T *__restrict__ fin = a.Fp;
  const T *__restrict__ zp = a.Zp;
  T *__restrict__ fo = a.Fc;
  T *__restrict__ gg = a.Gc;
  const Offs of(g);
  const Cm q(g);
  const bool cm = a0.cm != 0;
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
      // g and D of three-colour IC(0) plans in the colour-major layout
      const int jw = cm ? q.of(j) : j;
      if (!(cv & NB_SELF)) {
        fo[j] = T(0);
        if (a.fout) a.fout[j] = 0.0;
        if (!a.final_pass) {
          gg[jw] = T(0);
          a.D[jw] = T(0);
          if (cm) a0.Dv[j] = T(0);
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
        gg[jw] = gj;
        a.D[jw] = curv;
        if (cm) a0.Dv[j] = curv;
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

// The iteration's gradient pass of k_grad2 with four consecutive voxels of a
// column per thread (FP32, NE echoes fixed at compile time, nz a multiple of
// 4, single volumes): codes in 4-byte loads; f, z, the echo data and the
// +-1, +-2 neighbours along x and y in 16-byte loads; the z neighbours inside
// the four from registers and the two below and above in 8-byte loads.  Every
// value is formed with the expressions k_grad2 uses, so f, g and D are the
// same bits; only the order of the partial sums differs.
template <int NE>
__global__ __launch_bounds__(kNT) void k_grad2_q(IterArgs<float> a0) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<float> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const int nq = (int)(g.n >> 2), stride = vw.nb * kNT, sx = (int)g.sx, sy = (int)g.sy;
  const int64_t es = vw.es;
  const float *__restrict__ fin = a.Fp;
  const float *__restrict__ zin = a.Zp;
  const Cm cmv(g);
  const bool cm = a0.cm != 0;
  // neighbour slots in the order -x, +x, -y, +y (d = 1 and d = 2 apart)
  const int off[4] = {-sx, sx, -sy, sy};
  uint32_t c4, cx[4];
  float4 f4, z4, f1[4], z1[4], f2[4], z2[4], d4[NE][2];
  float2 fzm, zzm, fzp, zzp;  // f, z of the two voxels below (j-2, j-1) and above (j+4, j+5)
  uint32_t czm, czp;          // codes of voxels j-1 and j+4
  auto load = [&](int q) {
    const int j = 4 * q;
    c4 = *reinterpret_cast<const uint32_t *>(a.code + j);
    f4 = *reinterpret_cast<const float4 *>(fin + j);
    z4 = *reinterpret_cast<const float4 *>(zin + j);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cx[k] = *reinterpret_cast<const uint32_t *>(a.code + j + off[k]);
      f1[k] = *reinterpret_cast<const float4 *>(fin + j + off[k]);
      z1[k] = *reinterpret_cast<const float4 *>(zin + j + off[k]);
      f2[k] = *reinterpret_cast<const float4 *>(fin + j + 2 * off[k]);
      z2[k] = *reinterpret_cast<const float4 *>(zin + j + 2 * off[k]);
    }
    fzm = *reinterpret_cast<const float2 *>(fin + j - 2);
    zzm = *reinterpret_cast<const float2 *>(zin + j - 2);
    fzp = *reinterpret_cast<const float2 *>(fin + j + 4);
    zzp = *reinterpret_cast<const float2 *>(zin + j + 4);
    czm = a.code[j - 1];
    czp = a.code[j + 4];
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
  PairC<float> pc[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pc[k] = uniform_pair(a.pairs[k]);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (; q < nq; q += stride) {
    load(q);
    keep(c4);
    keep(f4);
    keep(z4);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      keep(cx[k]);
      keep(f1[k]);
      keep(z1[k]);
      keep(f2[k]);
      keep(z2[k]);
    }
    const int j = 4 * q;
    const float fv[4] = {f4.x, f4.y, f4.z, f4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
    // f and z of column voxels j-2 .. j+5
    const float fc[8] = {fzm.x, fzm.y, f4.x, f4.y, f4.z, f4.w, fzp.x, fzp.y};
    const float zc[8] = {zzm.x, zzm.y, z4.x, z4.y, z4.z, z4.w, zzp.x, zzp.y};
    float fo[4], go[4], dout[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t cv = (c4 >> (8 * i)) & 0xffu;
      const bool in = cv & NB_SELF;
      const float fj = fv[i] + alpha * zv[i];
      float v1[6], v2[6];
      uint32_t cn[6];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float a1[4] = {f1[k].x, f1[k].y, f1[k].z, f1[k].w}, b1[4] = {z1[k].x, z1[k].y, z1[k].z, z1[k].w};
        const float a2[4] = {f2[k].x, f2[k].y, f2[k].z, f2[k].w}, b2[4] = {z2[k].x, z2[k].y, z2[k].z, z2[k].w};
        v1[k] = a1[i] + alpha * b1[i];
        v2[k] = a2[i] + alpha * b2[i];
        cn[k] = (cx[k] >> (8 * i)) & 0xffu;
      }
      v1[4] = fc[i + 1] + alpha * zc[i + 1];  // z - 1
      v1[5] = fc[i + 3] + alpha * zc[i + 3];  // z + 1
      v2[4] = fc[i] + alpha * zc[i];          // z - 2
      v2[5] = fc[i + 4] + alpha * zc[i + 4];  // z + 2
      cn[4] = i > 0 ? (c4 >> (8 * (i - 1))) & 0xffu : czm;
      cn[5] = i < 3 ? (c4 >> (8 * (i + 1))) & 0xffu : czp;
      const Rows2 R(cv, cn);
      const float lap = ctc2(R, fj, v1, v2);
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
      acc[0] += in ? (double)phi : 0.0;
      acc[1] += in ? (double)fj * (double)lap : 0.0;
      acc[2] += in ? (double)gj * (double)gj : 0.0;
      acc[3] += in ? (double)zv[i] * (double)gj : 0.0;
    }
    *reinterpret_cast<float4 *>(a.Fc + j) = make_float4(fo[0], fo[1], fo[2], fo[3]);
    if (cm) {
      // g and D of three-colour IC(0) plans in the colour-major layout, D also in voxel order
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int jw = cmv.of(j + i);
        a.Gc[jw] = go[i];
        a.D[jw] = dout[i];
      }
      *reinterpret_cast<float4 *>(a0.Dv + j) = make_float4(dout[0], dout[1], dout[2], dout[3]);
    } else {
      *reinterpret_cast<float4 *>(a.Gc + j) = make_float4(go[0], go[1], go[2], go[3]);
      *reinterpret_cast<float4 *>(a.D + j) = make_float4(dout[0], dout[1], dout[2], dout[3]);
    }
  }
  store_partials<4, kNT>(acc, a.pout);
  put_state(st, a.sout, PK_GRAD, vw.nb, vw.leader);
}

// Diagonal (P = diag H with diag(C^T C) of the second-order operator) or
// identity preconditioner (as k_diag).
template <typename T, bool BATCH = false>
__global__ __launch_bounds__(kNT) void k_diag2(IterArgs<T> a0, const T *__restrict__ gsrc, int identity) {
  constexpr int V = Vpt<T>::v;
  const VolView vw = vol_view<BATCH>(a0);
  const VArgs<T> a = at_volume<BATCH>(a0, vw);
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
// In three-colour IC(0) plans p and D are the voxel-order copies that the
// preconditioner and gradient passes write beside the colour-major arrays.
template <typename T, bool BATCH = false>
__global__ __launch_bounds__(kNT) void k_dir2(IterArgs<T> a0) {
  constexpr int V = Vk<T, FM_V_DIR2>::v;
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

// Elements of the +-1, +-2 axis neighbours of the colour-c voxel at slot t
// (z mod 3 = z0): m1 = j - e, p1 = j + e, m2 = j - 2e, p2 = j + 2e per axis.
struct Nb2 {
  int m1[3], p1[3], m2[3], p2[3];
  __device__ __forceinline__ Nb2(const Cm &q, int c, int t, int z0) {
    const int up = q.at(c == 2 ? 0 : c + 1, t), dn = q.at(c == 0 ? 2 : c - 1, t);
    const int s[2] = {q.plane, q.m};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      m1[a] = dn - s[a];
      p1[a] = up + s[a];
      m2[a] = up - 2 * s[a];
      p2[a] = dn + 2 * s[a];
    }
    m1[2] = dn - (z0 == 0 ? 1 : 0);
    p1[2] = up + (z0 == 2 ? 1 : 0);
    m2[2] = up - (z0 <= 1 ? 1 : 0);
    p2[2] = dn + (z0 >= 1 ? 1 : 0);
  }
};

// In-mask flags and row indicators on the axis line through voxel j (in the
// mask, code c), from the codes at j-+e (cm1, cp1) and j-+2e (cm2, cp2), all
// loaded unconditionally (the blocks carry two padding planes and the codes of
// padding and unused slots are 0; a code read past the volume's edge is never
// trusted: j-2e counts only through an in-mask j-e, whose own code then says
// whether j-2e is in the mask, and a +-2 neighbour behind a hole couples to j
// through nothing), and the entries of H among them.
struct Line2 {
  bool m1, p1, m2, p2;   // j-e, j+e, j-2e, j+2e in the mask
  double hm1, hp1;       // H(j,j-e), H(j,j+e)
  double hm2, hp2;       // H(j,j-2e), H(j,j+2e)
  double hm1m2, hp1p2;   // H(j-e,j-2e), H(j+e,j+2e)
  double hm1p1;          // H(j-e,j+e)
  __device__ __forceinline__ Line2(uint32_t c, uint32_t cm1, uint32_t cp1, uint32_t cm2, uint32_t cp2, int a,
                                   double beta) {
    m1 = has_nb(c, 2 * a);
    p1 = has_nb(c, 2 * a + 1);
    m2 = m1 && has_nb(cm1, 2 * a);
    p2 = p1 && has_nb(cp1, 2 * a + 1);
    const double r0 = row2(c, a) ? 1.0 : 0.0;
    const double rm1 = (m1 && row2(cm1, a)) ? 1.0 : 0.0, rp1 = (p1 && row2(cp1, a)) ? 1.0 : 0.0;
    const double rm2 = (m2 && row2(cm2, a)) ? 1.0 : 0.0, rp2 = (p2 && row2(cp2, a)) ? 1.0 : 0.0;
    hm1 = beta * (-2.0 * r0 - 2.0 * rm1);
    hp1 = beta * (-2.0 * r0 - 2.0 * rp1);
    hm2 = beta * rm1;
    hp2 = beta * rp1;
    hm1m2 = beta * (-2.0 * rm1 - 2.0 * rm2);
    hp1p2 = beta * (-2.0 * rp1 - 2.0 * rp2);
    hm1p1 = beta * r0;
  }
};

// The codes at j-+e and j-+2e of the three axes, issued together.
struct Codes2 {
  uint32_t m1[3], p1[3], m2[3], p2[3];
  __device__ __forceinline__ Codes2(const uint8_t *__restrict__ code, const Nb2 &nb) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      m1[a] = code[nb.m1[a]];
      p1[a] = code[nb.p1[a]];
      m2[a] = code[nb.m2[a]];
      p2[a] = code[nb.p2[a]];
    }
  }
};

// Visit the slots of colour c that hold a voxel (every slot of the block's
// interior but the last of a column whose colour-c voxels number m - 1),
// workgroup-strided: f(t, z mod 3, voxel index).
template <typename F>
__device__ __forceinline__ void for_colour(const Geo &g, const Cm &q, int c, int first, int step, F &&f) {
  const int total = g.nx * q.plane;
  const Div dm(q.m);
  for (int t = first; t < total; t += step) {
    int k, y;
    const int col = dm(t, k);
    const int x = q.dy(col, y);
    const int z0 = (c + 3 - (x + y) % 3) % 3;
    const int z = z0 + 3 * k;
    if (z < g.nz) f(t, z0, col * g.nz + z);
  }
}

// Colour-major codes and diag(C^T C) (0 outside the mask, in the padding planes
// and in unused slots), once per setup; every element of both arrays is written.
__global__ __launch_bounds__(kBlock) void k_colour_major2(Geo g, const uint8_t *__restrict__ code, uint8_t *ccode,
                                                          uint8_t *rdiag) {
  const Cm q(g);
  const Offs of(g);
  const int total = 3 * q.S;
  for (int e = (int)blockIdx.x * kBlock + (int)threadIdx.x; e < total; e += (int)gridDim.x * kBlock) {
    const int c = e / q.S, r = e - c * q.S;
    const int xp = r / q.plane, w = r - xp * q.plane;
    const int x = xp - 2, y = w / q.m, k = w - y * q.m;
    uint32_t cv = 0u;
    int j = 0;
    if (x >= 0 && x < g.nx) {
      const int z = (c + 3 - (x + y) % 3) % 3 + 3 * k;
      if (z < g.nz) {
        j = x * (int)g.sx + y * g.nz + z;
        cv = code[j];
      }
    }
    uint8_t d = 0;
    if (cv & NB_SELF) {
      uint32_t cn[6];
#pragma unroll
      for (int s = 0; s < 6; ++s) cn[s] = has_nb(cv, s) ? code[j + of.o[s]] : 0u;
      d = (uint8_t)Rows2(cv, cn).diag();
    }
    ccode[e] = (uint8_t)cv;
    rdiag[e] = d;
  }
}

// Conversions between voxel order (user float64 arrays) and the colour-major
// working arrays.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_cm(Geo g, const double *__restrict__ src, T *dst) {
  const Cm q(g);
  for (int j = (int)blockIdx.x * kBlock + (int)threadIdx.x; j < (int)g.n; j += (int)gridDim.x * kBlock)
    dst[q.of(j)] = (T)src[j];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_cm(Geo g, const T *__restrict__ src, double *dst) {
  const Cm q(g);
  for (int j = (int)blockIdx.x * kBlock + (int)threadIdx.x; j < (int)g.n; j += (int)gridDim.x * kBlock)
    dst[j] = (double)src[q.of(j)];
}

__global__ __launch_bounds__(kBlock) void k_pivots_cm(Geo g, const double *__restrict__ ipiv, double *piv) {
  const Cm q(g);
  for (int j = (int)blockIdx.x * kBlock + (int)threadIdx.x; j < (int)g.n; j += (int)gridDim.x * kBlock) {
    const double ip = ipiv[q.of(j)];
    piv[j] = ip > 0.0 ? 1.0 / ip : 0.0;
  }
}

// Forward pass over colours 0 and 1: pivots (stored inverted), y and y' of
// colour 1, and their terms of the two dot products.  gsrc: standalone call.
template <typename T>
__global__ __launch_bounds__(kNT) void k_ic3_fwd1(IterArgs<T> a0, const T *__restrict__ gsrc) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const Cm q(g);
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const uint8_t *__restrict__ cc = a0.ccode;
  const uint8_t *__restrict__ rd = a0.rdiag;
  const State st = take_state<kNT, 4>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  const int first = vw.bl * kNT + (int)threadIdx.x, step = vw.nb * kNT;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for_colour(g, q, 0, first, step, [&](int t, int, int) {
    const int j = q.at(0, t);
    const uint32_t c = cc[j];
    const double d = (double)a.D[j] + beta * (double)rd[j], y = (double)gg[j], y2 = (double)gp[j];
    double ip = 1.0 / d;
    if (!(c & NB_SELF)) {
      ip = 0.0;
    } else if (!(d > 0.0)) {
      bad = 1;
      ip = 0.0;
    }
    a.ipiv[j] = ip;
    acc[0] += y * y * ip;
    acc[1] += y2 * y * ip;
  });
  // colour 1: earlier neighbours j-e and j+2e (colour 0, pivots D + beta diag(C^T C))
  for_colour(g, q, 1, first, step, [&](int t, int z0, int) {
    const int j = q.at(1, t);
    const uint32_t c = cc[j];
    const Nb2 nb(q, 1, t, z0);
    const Codes2 cs(cc, nb);
    double dk[6], hk[6], gk[6], gpk[6];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = u ? nb.p2[ax] : nb.m1[ax];
        dk[2 * ax + u] = (double)a.D[k] + beta * (double)rd[k];
        gk[2 * ax + u] = (double)gg[k];
        gpk[2 * ax + u] = (double)gp[k];
      }
      const Line2 l(c, cs.m1[ax], cs.p1[ax], cs.m2[ax], cs.p2[ax], ax, beta);
      hk[2 * ax] = l.m1 ? l.hm1 : 0.0;
      hk[2 * ax + 1] = l.p2 ? l.hp2 : 0.0;
    }
    double d = (double)a.D[j] + beta * (double)rd[j];
    double y = (double)gg[j], y2 = (double)gp[j];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double lk = hk[k] != 0.0 ? hk[k] / dk[k] : 0.0;
      d -= hk[k] * lk;
      y -= hk[k] != 0.0 ? lk * gk[k] : 0.0;
      y2 -= hk[k] != 0.0 ? lk * gpk[k] : 0.0;
    }
    double ip = 1.0 / d;
    if (!(c & NB_SELF)) {
      ip = 0.0;
      y = 0.0;
      y2 = 0.0;
    } else if (!(d > 0.0)) {
      bad = 1;
      ip = 0.0;
    }
    a.ipiv[j] = ip;
    a0.X[j] = (T)y;
    a0.X2[j] = (T)y2;
    acc[0] += y * y * ip;
    acc[1] += y2 * y * ip;
  });
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
  const Cm q(g);
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const T *__restrict__ gp = a.Gp;
  const uint8_t *__restrict__ cc = a0.ccode;
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  double acc[2] = {0.0, 0.0};
  int bad = 0;
  for_colour(g, q, 2, vw.bl * kNT + (int)threadIdx.x, vw.nb * kNT, [&](int t, int z0, int jv) {
    const int j = q.at(2, t);
    const uint32_t c = cc[j];
    const Nb2 nb(q, 2, t, z0);
    const Codes2 cs(cc, nb);
    // per axis: 1/D at j-e, j+e, j-2e, j+2e; g, g_prev at j+e, j-2e (colour 0); y, y' at j-e, j+2e (colour 1)
    double ip4[3][4], g2[3][2], gp2[3][2], x2[3][2], xp2[3][2];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      ip4[ax][0] = a.ipiv[nb.m1[ax]];
      ip4[ax][1] = a.ipiv[nb.p1[ax]];
      ip4[ax][2] = a.ipiv[nb.m2[ax]];
      ip4[ax][3] = a.ipiv[nb.p2[ax]];
      g2[ax][0] = (double)gg[nb.p1[ax]];
      g2[ax][1] = (double)gg[nb.m2[ax]];
      gp2[ax][0] = (double)gp[nb.p1[ax]];
      gp2[ax][1] = (double)gp[nb.m2[ax]];
      x2[ax][0] = (double)a0.X[nb.m1[ax]];
      x2[ax][1] = (double)a0.X[nb.p2[ax]];
      xp2[ax][0] = (double)a0.X2[nb.m1[ax]];
      xp2[ax][1] = (double)a0.X2[nb.p2[ax]];
    }
    double d = (double)a.D[j] + beta * (double)a0.rdiag[j];
    double y = (double)gg[j], y2 = (double)gp[j];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const Line2 l(c, cs.m1[ax], cs.p1[ax], cs.m2[ax], cs.p2[ax], ax, beta);
      const double ipm1 = l.m1 ? ip4[ax][0] : 0.0, ipp1 = l.p1 ? ip4[ax][1] : 0.0;
      const double ipm2 = l.m2 ? ip4[ax][2] : 0.0, ipp2 = l.p2 ? ip4[ax][3] : 0.0;
      // colour 0: j+e and j-2e; colour 1: j-e and j+2e (entries times the pivot of the neighbour)
      const double np1 = l.hp1, nm2 = l.hm2;
      const double nm1 = l.hm1 - l.hm2 * l.hm1m2 * ipm2 - l.hp1 * l.hm1p1 * ipp1;
      const double np2 = l.hp2 - l.hp1 * l.hp1p2 * ipp1;
      const double lp1 = np1 * ipp1, lm2 = nm2 * ipm2, lm1 = nm1 * ipm1, lp2 = np2 * ipp2;
      d -= np1 * lp1 + nm2 * lm2 + nm1 * lm1 + np2 * lp2;
      y -= (l.p1 ? lp1 * g2[ax][0] : 0.0) + (l.m2 ? lm2 * g2[ax][1] : 0.0) + (l.m1 ? lm1 * x2[ax][0] : 0.0) +
           (l.p2 ? lp2 * x2[ax][1] : 0.0);
      y2 -= (l.p1 ? lp1 * gp2[ax][0] : 0.0) + (l.m2 ? lm2 * gp2[ax][1] : 0.0) + (l.m1 ? lm1 * xp2[ax][0] : 0.0) +
            (l.p2 ? lp2 * xp2[ax][1] : 0.0);
    }
    double ip = 1.0 / d;
    if (!(c & NB_SELF)) {
      ip = 0.0;
      y = 0.0;
      y2 = 0.0;
    } else if (!(d > 0.0)) {
      bad = 1;
      ip = 0.0;
    }
    a.ipiv[j] = ip;
    const T pj = (T)(y * ip);
    a.P[j] = pj;
    a0.Pv[jv] = pj;
    acc[0] += y * y * ip;
    acc[1] += y2 * y * ip;
  });
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
  const Cm q(g);
  const uint8_t *__restrict__ cc = a0.ccode;
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  for_colour(g, q, 1, vw.bl * kNT + (int)threadIdx.x, vw.nb * kNT, [&](int t, int z0, int jv) {
    const int j = q.at(1, t);
    const uint32_t c = cc[j];
    const Nb2 nb(q, 1, t, z0);
    const Codes2 cs(cc, nb);
    double ipm1[3], ipp2[3], pp1[3], pm2[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      ipm1[ax] = a.ipiv[nb.m1[ax]];
      ipp2[ax] = a.ipiv[nb.p2[ax]];
      pp1[ax] = (double)a.P[nb.p1[ax]];
      pm2[ax] = (double)a.P[nb.m2[ax]];
    }
    const double ip = a.ipiv[j], yj = (double)a0.X[j];
    double s = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const Line2 l(c, cs.m1[ax], cs.p1[ax], cs.m2[ax], cs.p2[ax], ax, beta);
      const double im1 = l.m1 ? ipm1[ax] : 0.0, ip2 = l.p2 ? ipp2[ax] : 0.0;
      // i = j+e: L(i,j) D_j = H(i,j) - H(i,j-e) H(j,j-e)/D(j-e) - H(i,j+2e) H(j,j+2e)/D(j+2e)
      const double n1 = l.hp1 - l.hm1p1 * l.hm1 * im1 - l.hp1p2 * l.hp2 * ip2;
      // i = j-2e: L(i,j) D_j = H(i,j) - H(i,j-e) H(j-e,j)/D(j-e)
      const double n2 = l.hm2 - l.hm1m2 * l.hm1 * im1;
      s += (l.p1 ? n1 * pp1[ax] : 0.0) + (l.m2 ? n2 * pm2[ax] : 0.0);
    }
    const T pj = (c & NB_SELF) ? (T)((yj - s) * ip) : T(0);
    a.P[j] = pj;
    a0.Pv[jv] = pj;
  });
  put_state(st, a.sout, PK_NONE, 0, vw.leader);
}

// Backward pass over colour 0: p_j = (g_j - sum_i H(j,i) p_i) / D_j over the
// stencil neighbours (colours 1 and 2).
template <typename T>
__global__ __launch_bounds__(kNT) void k_ic3_bwd0(IterArgs<T> a0, const T *__restrict__ gsrc) {
  const VolView vw = vol_view<false>(a0);
  const VArgs<T> a = at_volume<false>(a0, vw);
  const Geo g = a.geo;
  const Cm q(g);
  const T *__restrict__ gg = gsrc ? gsrc : a.Gc;
  const uint8_t *__restrict__ cc = a0.ccode;
  const State st = take_state<kNT, 2>(a.sin, a.pin, a.nparts_in, a.nvals_in, a.beta, a.trace, a.status, vw.prow, vw.leader);
  const double beta = a.beta;
  for_colour(g, q, 0, vw.bl * kNT + (int)threadIdx.x, vw.nb * kNT, [&](int t, int z0, int jv) {
    const int j = q.at(0, t);
    const uint32_t c = cc[j];
    const Nb2 nb(q, 0, t, z0);
    const Codes2 cs(cc, nb);
    double pn[3][4];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      pn[ax][0] = (double)a.P[nb.m1[ax]];
      pn[ax][1] = (double)a.P[nb.p1[ax]];
      pn[ax][2] = (double)a.P[nb.m2[ax]];
      pn[ax][3] = (double)a.P[nb.p2[ax]];
    }
    double s = (double)gg[j];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const Line2 l(c, cs.m1[ax], cs.p1[ax], cs.m2[ax], cs.p2[ax], ax, beta);
      s -= (l.m1 ? l.hm1 * pn[ax][0] : 0.0) + (l.p1 ? l.hp1 * pn[ax][1] : 0.0) + (l.m2 ? l.hm2 * pn[ax][2] : 0.0) +
           (l.p2 ? l.hp2 * pn[ax][3] : 0.0);
    }
    const T pj = (c & NB_SELF) ? (T)(s * a.ipiv[j]) : T(0);
    a.P[j] = pj;
    a0.Pv[jv] = pj;
  });
  put_state(st, a.sout, PK_NONE, 0, vw.leader);
}

}  // namespace fm
