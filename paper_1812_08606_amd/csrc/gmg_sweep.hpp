// gmg_sweep.hpp -- one symmetric red-black Gauss-Seidel sweep on the finest
// level (cell coefficient a, face = arithmetic mean; eq. e18) in a single
// pass over HBM.
//
// A sweep updates every cell of the first colour c1 from the old iterate,
// then every cell of the other colour from the new first-colour values
// (pre-smoothing: red then black; post-smoothing: black then red).  It reads
// x_old, a and b once and writes x_new once (ping-pong buffers, so no block
// sees another block's partial update).
//
// Blocking: a block owns a 64 x TY tile of (x, y) cells and marches a chunk
// of z-planes.  Per plane it keeps in LDS the tile plus a ring of 2 cells
// (positions (r, q), r in [0, TY+4), q in [0, 68); global x = 64 bx - 2 + q,
// y = TY by - 2 + r), in ring buffers over planes:
//   xo: x_old on planes t-1, t, t+1     a: coefficient on planes t-2 .. t+1
//   b : right side on planes t-1, t     rn: new first-colour values on t-2 .. t
// A row of LDS holds its even columns first, then its odd columns, so that
// the cells of one colour, and each of their x-neighbours, are contiguous.
// Step t stores plane t+1 (x_old, a) and plane t (b) into LDS (fetched into
// registers during step t-1), computes the new first-colour values of plane
// t on the tile and a 1-cell ring (the ring values are recomputed by every
// block that needs them), then the new second-colour values of plane t-1 on
// the tile, and stores plane t-1.
//
// The phase functions below are device functions called by the kernel in
// gmg_kernels.hpp between block barriers.
#pragma once

#include <stddef.h>

#include "gmg_common.hpp"

namespace gmg {

enum SweepX { SWEEP_X_ZERO = 0, SWEEP_X_LOAD = 1 };

template <int TY_>
struct SweepTile {
  static constexpr int TX = 64;
  static constexpr int TY = TY_;
  static constexpr int W = TX + 4;  // positions per row (2-cell ring)
  static constexpr int HW = W / 2;  // positions per row and column parity
  static constexpr int H = TY + 4;  // rows
  static constexpr int P = W * H;   // positions per plane
};

template <typename T, int TY>
struct SweepSmem {
  static constexpr int P = SweepTile<TY>::P;
  T xo[3][P];
  T a[4][P];
  T b[2][P];
  T rn[3][P];
};

template <typename T, typename TB>
struct SweepArgs {
  const T* x_in;         // old iterate (SWEEP_X_LOAD)
  const TB* b;           // right side, read as b * (*bscale)
  const double* bscale;  // null = 1
  T* b_out;              // when given, b (in T) is stored for the tile's cells
  const T* a;            // cell coefficient
  T* x_out;              // new iterate
  Geom g;
  int c1;  // colour updated first: 0 red (pre-smoothing), 1 black (post)
  int kc;  // planes per block
};

// Ring-buffer slots of plane p (p >= -8).
__device__ __forceinline__ int slot3(int p) { return (p + 9) % 3; }
__device__ __forceinline__ int slot4(int p) { return (p + 8) % 4; }
__device__ __forceinline__ int slot2(int p) { return (p + 8) % 2; }

// LDS index of position (r, q): even columns of a row, then odd columns.
template <int TY>
__device__ __forceinline__ int sweep_lidx(int r, int q) {
  return r * SweepTile<TY>::W + (q & 1) * SweepTile<TY>::HW + (q >> 1);
}

// 1 / d: the hardware reciprocal (1 ulp) in the float32 preconditioner, an
// exact division in float64.
__device__ __forceinline__ float sweep_recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double sweep_recip(double d) { return 1.0 / d; }

// Geometry of this thread's fetch positions (pos = tid + e * nthreads),
// computed once per block.
template <int NPT, int XM>
struct SweepPlan {
  int off[NPT];   // in-plane offset y * nx + x, -1 outside the grid or the region
  int lds[NPT];   // LDS index
  unsigned tile;  // bit e: a tile cell (its b is stored to b_out)
};

template <int TY, int NPT, int XM>
__device__ __forceinline__ void sweep_plan(SweepPlan<NPT, XM>& P, const Geom& g, int bx, int by, int tid,
                                           int nthreads) {
  typedef SweepTile<TY> Tl;
  const int X0 = bx * Tl::TX - 2, Y0 = by * TY - 2;
  P.tile = 0u;
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    const int pos = tid + e * nthreads;
    const int r = pos / Tl::W, q = pos - r * Tl::W;
    const int x = X0 + q, y = Y0 + r;
    const bool in = pos < Tl::P && x >= 0 && x < g.nx && y >= 0 && y < g.ny;
    P.off[e] = in ? y * g.nx + x : -1;
    P.lds[e] = pos < Tl::P ? sweep_lidx<TY>(r, q) : 0;
    if (in && r >= 2 && r < TY + 2 && q >= 2 && q < Tl::TX + 2) P.tile |= 1u << e;
  }
}

// Values one thread fetches from HBM for one plane (software pipelining:
// fetched one step ahead into registers, stored into LDS at the next step).
template <typename T, int XM, int NPT>
struct SweepFetch {
  T xv[XM == SWEEP_X_LOAD ? NPT : 1];  // x_old
  T av[NPT];                           // coefficient
  T bv[NPT];                           // right side
};

// Fetch phase: x_old and a of plane pxa (if load_xa) and b of plane pb (if
// load_b) for this thread's positions; positions outside the grid get 0
// (their faces have weight 0).  The tile's b is stored to b_out when store_b.
template <typename T, typename TB, int XM, int NPT, bool SCALED>
__device__ __forceinline__ void sweep_fetch(SweepFetch<T, XM, NPT>& R, const SweepPlan<NPT, XM>& P,
                                            const SweepArgs<T, TB>& A, int pxa, bool load_xa, int pb, bool load_b,
                                            bool store_b, double bsc) {
  const Geom& g = A.g;
  const size_t nxy = (size_t)g.nx * g.ny;
  const T* ap = A.a + (size_t)(load_xa ? pxa : 0) * nxy;
  const T* xp = XM != SWEEP_X_ZERO ? A.x_in + (size_t)(load_xa ? pxa : 0) * nxy : nullptr;
  const TB* bp = A.b + (size_t)(load_b ? pb : 0) * nxy;
  T* bo = store_b ? A.b_out + (size_t)pb * nxy : nullptr;
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    const int o = P.off[e];
    const bool in = o >= 0;
    if (load_xa) {
      R.av[e] = in ? ap[o] : T(0);
      if (XM == SWEEP_X_LOAD) R.xv[XM == SWEEP_X_LOAD ? e : 0] = in ? xp[o] : T(0);
    }
    if (load_b) {
      T bv = T(0);
      if (in) bv = SCALED ? (T)((double)bp[o] * bsc) : (T)bp[o];
      R.bv[e] = bv;
      if (store_b && ((P.tile >> e) & 1u)) bo[o] = bv;
    }
  }
}

// Stash phase: the fetched values into the LDS ring slots of their planes.
template <typename T, int XM, int TY, int NPT>
__device__ __forceinline__ void sweep_stash(SweepSmem<T, TY>& s, const SweepFetch<T, XM, NPT>& R,
                                            const SweepPlan<NPT, XM>& P, int tid, int nthreads, int pxa,
                                            bool load_xa, int pb, bool load_b) {
  typedef SweepTile<TY> Tl;
  T* xo = s.xo[slot3(pxa)];
  T* av = s.a[slot4(pxa)];
  T* bv = s.b[slot2(pb)];
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    if (tid + e * nthreads >= Tl::P) continue;
    const int l = P.lds[e];
    if (load_xa) {
      if (XM == SWEEP_X_LOAD) xo[l] = R.xv[XM == SWEEP_X_LOAD ? e : 0];
      av[l] = R.av[e];
    }
    if (load_b) bv[l] = R.bv[e];
  }
}

// Gauss-Seidel value of the cell at LDS index l of plane t from the x-values
// xc (same plane), xb, xt (planes below and above) and the coefficients of
// the three planes; the flags say which faces exist.  Values beyond a
// missing face (outside the grid, never computed) are discarded by selects.
template <typename T, bool ZERO>
__device__ __forceinline__ T gs_value(int l, int W, const T* __restrict__ xc, const T* __restrict__ xb,
                                      const T* __restrict__ xt, const T* __restrict__ ac_, const T* __restrict__ ab_,
                                      const T* __restrict__ at_, T bval, bool hw, bool he, bool hs, bool hn, bool hb,
                                      bool ht, int lw, int le, T hx, T hy, T hz, T pz) {
  const T ac = ac_[l];
  const T ww = hw ? (ac + ac_[lw]) * hx : T(0);
  const T we = he ? (ac + ac_[le]) * hx : T(0);
  const T ws = hs ? (ac + ac_[l - W]) * hy : T(0);
  const T wn = hn ? (ac + ac_[l + W]) * hy : T(0);
  const T wb = hb ? (ac + ab_[l]) * hz : T(0);
  const T wt = ht ? (ac + at_[l]) * hz : T(0);
  const T D = ww + we + ws + wn + wb + wt + (hb ? T(0) : pz * ac) + (ht ? T(0) : pz * ac);
  T off = T(0);
  if (!ZERO) {
    off = (hw ? ww * xc[lw] : T(0)) + (he ? we * xc[le] : T(0));
    off += (hs ? ws * xc[l - W] : T(0)) + (hn ? wn * xc[l + W] : T(0));
    off += hb ? wb * xb[l] : T(0);
    off += ht ? wt * xt[l] : T(0);
  }
  return (bval + off) * sweep_recip(D);
}

// Per-thread geometry of the two update phases, for both parities of the
// plane index (the colour pattern of a plane alternates with its parity),
// computed once per block.  Each entry packs the LDS index of the cell (bits
// 0-15) and flags: bit 16 valid, 17 west face, 18 east face, 19 south face,
// 20 north face.
template <int TY>
struct SweepPhasePlan {
  static constexpr int NF = ((SweepTile<TY>::TX + 2) / 2 * (TY + 2) + NTHREADS - 1) / NTHREADS;
  static constexpr int NS = (SweepTile<TY>::TX / 2 * TY + NTHREADS - 1) / NTHREADS;
  int first[2][NF];
  int second[2][NS];   // second-colour cell of the pair
  int second1[2][NS];  // LDS index of the first-colour cell of the pair; bit 16: it is element 1
  int out[NS];         // in-plane offset of the pair's first cell (x0), -1 if not stored; bit 30: x0+1 stored
};

__device__ __forceinline__ int sweep_pack(int l, bool valid, bool w, bool e, bool s, bool n) {
  return l | (valid ? 1 << 16 : 0) | (w ? 1 << 17 : 0) | (e ? 1 << 18 : 0) | (s ? 1 << 19 : 0) | (n ? 1 << 20 : 0);
}

template <int TY>
__device__ __forceinline__ void sweep_phase_plan(SweepPhasePlan<TY>& Q, const Geom& g, int c1, int bx, int by,
                                                 int tid) {
  typedef SweepTile<TY> Tl;
  typedef SweepPhasePlan<TY> Pl;
  const int X0 = bx * Tl::TX - 2, Y0 = by * TY - 2;
  constexpr int per_row = (Tl::TX + 2) / 2;
  constexpr int nf = per_row * (TY + 2);
  constexpr int pairs = Tl::TX / 2;
  constexpr int ns = pairs * TY;
#pragma unroll
  for (int par = 0; par < 2; ++par) {
#pragma unroll
    for (int k = 0; k < Pl::NF; ++k) {
      const int f = tid + k * NTHREADS;
      const int rr = f / per_row, m = f - rr * per_row;
      const int r = 1 + rr;
      const int sft = (c1 + X0 + 1 + Y0 + r + par) & 1;
      const int q = 1 + sft + 2 * m;
      const int x = X0 + q, y = Y0 + r;
      const bool valid = f < nf && x >= 0 && x < g.nx && y >= 0 && y < g.ny;
      Q.first[par][k] = sweep_pack(valid ? sweep_lidx<TY>(r, q) : 0, valid, x > 0, x < g.nx - 1, y > 0,
                                   y < g.ny - 1);
    }
#pragma unroll
    for (int k = 0; k < Pl::NS; ++k) {
      const int f = tid + k * NTHREADS;
      const int rr = f / pairs, pp = f - rr * pairs;
      const int r = 2 + rr, q0 = 2 + 2 * pp;
      const int y = Y0 + r, x0 = X0 + q0;
      const bool stored = f < ns && y < g.ny && x0 < g.nx;
      const int e1 = (c1 + x0 + y + par) & 1;
      const int q2 = q0 + (1 - e1), x2 = x0 + (1 - e1);
      const bool valid = stored && x2 < g.nx;
      Q.second[par][k] = sweep_pack(valid ? sweep_lidx<TY>(r, q2) : 0, valid, x2 > 0, x2 < g.nx - 1, y > 0,
                                    y < g.ny - 1);
      Q.second1[par][k] = (stored ? sweep_lidx<TY>(r, q0 + e1) : 0) | (e1 ? 1 << 16 : 0);
      if (par == 0) Q.out[k] = stored ? ((y * g.nx + x0) | (x0 + 1 < g.nx ? 1 << 30 : 0)) : -1;
    }
  }
}

// First-colour update of plane t on the tile and its 1-cell ring.
template <typename T, int XM, int TY>
__device__ __forceinline__ void sweep_first(SweepSmem<T, TY>& s, const SweepPhasePlan<TY>& Q, const Geom& g, int t) {
  typedef SweepTile<TY> Tl;
  const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2), pz = (T)(2.0 * g.ihz2);
  const T* xo_c = s.xo[slot3(t)];
  const T* xo_b = s.xo[slot3(t - 1)];
  const T* xo_t = s.xo[slot3(t + 1)];
  const T* a_c = s.a[slot4(t)];
  const T* a_b = s.a[slot4(t - 1)];
  const T* a_t = s.a[slot4(t + 1)];
  const T* b_c = s.b[slot2(t)];
  T* rn = s.rn[slot3(t)];
  const bool hb = t > 0, ht = t < g.nz - 1;
  const int par = t & 1;
#pragma unroll
  for (int k = 0; k < SweepPhasePlan<TY>::NF; ++k) {
    const int e = Q.first[par][k];
    if (!(e & (1 << 16))) continue;
    const int l = e & 0xffff;
    // the x-neighbours of an even column sit in the odd half of the row
    // (same or previous slot), those of an odd column in the even half
    const int lw = (l % Tl::W) >= Tl::HW ? l - Tl::HW : l + Tl::HW - 1;
    const int le = (l % Tl::W) >= Tl::HW ? l - Tl::HW + 1 : l + Tl::HW;
    rn[l] = gs_value<T, XM == SWEEP_X_ZERO>(l, Tl::W, xo_c, xo_b, xo_t, a_c, a_b, a_t, b_c[l], (e >> 17) & 1,
                                            (e >> 18) & 1, (e >> 19) & 1, (e >> 20) & 1, hb, ht, lw, le, hx, hy, hz,
                                            pz);
  }
}

// Second-colour update of plane tb on the tile, and the store of plane tb
// (both colours) into x_out.  Each work item is a pair of x-adjacent cells
// (one of each colour).
template <typename T, int TY>
__device__ __forceinline__ void sweep_second(SweepSmem<T, TY>& s, const SweepPhasePlan<TY>& Q, const Geom& g,
                                             T* __restrict__ x_out, int tb) {
  typedef SweepTile<TY> Tl;
  const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2), pz = (T)(2.0 * g.ihz2);
  const T* rn_c = s.rn[slot3(tb)];
  const T* rn_b = s.rn[slot3(tb - 1)];
  const T* rn_t = s.rn[slot3(tb + 1)];
  const T* a_c = s.a[slot4(tb)];
  const T* a_b = s.a[slot4(tb - 1)];
  const T* a_t = s.a[slot4(tb + 1)];
  const T* b_c = s.b[slot2(tb)];
  const bool hb = tb > 0, ht = tb < g.nz - 1;
  T* plane = x_out + (size_t)tb * g.nx * g.ny;
  const int par = tb & 1;
#pragma unroll
  for (int k = 0; k < SweepPhasePlan<TY>::NS; ++k) {
    const int o = Q.out[k];
    if (o < 0) continue;
    const int e = Q.second[par][k];
    const int e1 = Q.second1[par][k];
    const T v1 = rn_c[e1 & 0xffff];
    T v2 = T(0);
    if (e & (1 << 16)) {
      const int l = e & 0xffff;
      const int lw = (l % Tl::W) >= Tl::HW ? l - Tl::HW : l + Tl::HW - 1;
      const int le = (l % Tl::W) >= Tl::HW ? l - Tl::HW + 1 : l + Tl::HW;
      v2 = gs_value<T, false>(l, Tl::W, rn_c, rn_b, rn_t, a_c, a_b, a_t, b_c[l], (e >> 17) & 1, (e >> 18) & 1,
                              (e >> 19) & 1, (e >> 20) & 1, hb, ht, lw, le, hx, hy, hz, pz);
    }
    const bool first_is_1 = (e1 >> 16) & 1;
    T* out = plane + (o & ((1 << 30) - 1));
    out[0] = first_is_1 ? v2 : v1;
    if (o & (1 << 30)) out[1] = first_is_1 ? v1 : v2;
  }
}

// Plane schedule of one block (z-chunk [k0, k1)): step t runs from k0-3 to
// k1; it stashes plane t+1 (x_old, a) and plane t (b), computes the first
// colour of plane t and the second colour of plane t-1.
struct SweepStep {
  int pxa;
  bool load_xa;
  int pb;
  bool load_b, store_b;
  bool do_first;
  bool do_second;
};

__device__ __forceinline__ SweepStep sweep_step(const Geom& g, int k0, int k1, int t) {
  SweepStep st;
  const int lo = k0 - 1 > 0 ? k0 - 1 : 0;       // first plane whose first-colour values are needed
  const int hi = k1 < g.nz - 1 ? k1 : g.nz - 1;  // last such plane
  st.pxa = t + 1;
  st.load_xa = st.pxa >= (k0 - 2 > 0 ? k0 - 2 : 0) && st.pxa <= (k1 + 1 < g.nz - 1 ? k1 + 1 : g.nz - 1);
  st.pb = t;
  st.load_b = t >= lo && t <= hi;
  st.store_b = t >= k0 && t < k1;
  st.do_first = t >= lo && t <= hi;
  st.do_second = t - 1 >= k0 && t - 1 < k1;
  return st;
}

}  // namespace gmg
