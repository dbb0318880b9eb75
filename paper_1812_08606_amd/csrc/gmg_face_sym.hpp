// gmg_face_sym.hpp -- fused symmetric red-black sweep on a coarse level
// (natural layout, stored face coefficients): both half-sweeps of one
// symmetric Gauss-Seidel sweep in one pass, with the values of two
// k_gs_pair_face launches to the bit.
#pragma once

#include "gmg_kernels.hpp"
#include "gmg_sym.hpp"

namespace gmg {

// One plane of one lane's pair (cells 2m, 2m + 1 of row j), reduced to what
// the two colour updates read: the pair's colour-c1 cell is e1 = (c1 + j +
// p) % 2, its colour-c2 cell the other one.  The face below a cell on plane
// p + 1 is the face above the cell of the same column on plane p, whose
// colour is the other one: the top face of the c1 cell on plane p is wb2 of
// plane p + 1 (and the top plate's tp1 on the last plane).
template <typename T>
struct FaceCol {
  T b1, b2;        // right sides of the c1 and the c2 cell
  T wy0, wy1;      // south faces of cells 2m and 2m + 1 (also staged: row j - 1's north faces)
  T hwy0, hwy1;    // the same of row j + 1 (row R - 1 stages it for itself)
  T wb1, wb2;      // their bottom faces
  T tp1, tp2;      // their top-plate faces (last plane only)
  T wx0, wx1, wxe; // x-faces: west of cell 2m, between the cells, east of 2m + 1 (the last lane
                   // of a wave loads wxe; the others take the next lane's wx0)
  T xo;            // old value of the c2 cell
  T hxo;           // old c2 value of the same column in the row beyond the block (rows 0 and R - 1)
};

// Block: 64 WX lanes per row (the whole row: no x-halo) times R = 16 / WX
// rows (float32; 8 / WX in float64, whose registers would not fit 1024
// threads), of which rows 0 and R - 1 are a halo (their c1 values feed rows 1
// and R - 2 and are not stored).  Lane m owns pair m of row j = (R - 2) by
// + r - 1 and marches a z-chunk: on iteration k it updates colour c1 on
// plane k from the old iterate Xin (the other colour's old values of rows
// j - 1 and j + 1 and of pairs m - 1 and m + 1 from an LDS stage of two
// planes), writes the new value into an LDS ring of three planes, waits at
// a barrier, and updates colour c2 on plane k - 1 from the ring.  Planes
// k0 - 1 and k1 get c1 only (for the c2 updates of the chunk's end planes).
// FIRST: the first sweep from x = 0 (c1 = b / D; Xin not read).  Xout must
// not be Xin unless FIRST: other blocks still read the old values.
template <typename T, int WX>
struct FaceSymShape {
  static constexpr int W = 64 * WX;
  static constexpr int R = (sizeof(T) == 4 ? 16 : 8) / WX;
  static constexpr int IY = R - 2;
  static_assert(IY >= 1, "a block needs a row that owns cells");
};

template <typename T, bool FIRST, int WX>
__global__ __launch_bounds__((FaceSymShape<T, WX>::W * FaceSymShape<T, WX>::R)) void k_sym_face(const T* __restrict__ Xin, T* __restrict__ Xout,
                                                   const T* __restrict__ b, FaceCoef<T> co, Geom g, int kc,
                                                   int c1) {
  using T2 = typename Pair2<T>::type;
  constexpr int W = FaceSymShape<T, WX>::W, R = FaceSymShape<T, WX>::R, IY = FaceSymShape<T, WX>::IY;
  constexpr int NS = 2;  // planes of staged old values (c2 updates read only the ring)
  __shared__ T sx[NS][R + 2][W];  // old c2 values of block rows -1 .. R (array rows 0 .. R+1)
  // south-face pairs of block rows 0 .. R (array rows 1 .. R+1): the north
  // faces of rows -1 .. R-1; four planes, since the c2 update reads plane
  // k-1's after the barrier while plane k+1's is staged
  __shared__ T2 swy[4][R + 2][W];
  __shared__ T ring[3][R][W];     // new c1 values of planes k-1, k, k+1 (mod 3)
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = threadIdx.x, r = threadIdx.y;
  const int j = tl.y * IY + r - 1;
  const bool owner = m < H && j >= 0 && j < g.ny && r >= 1 && r <= IY;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const T ix = (T)g.ihx2, iy = (T)g.ihy2, iz = (T)g.ihz2;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  const bool hwo = m > 0, heo = m < H - 1, hs = j > 0, hn = j < g.ny - 1;
  // clamped (always valid) column of this lane and of the row beyond the
  // block that rows 0 and R-1 stage; neighbour lanes for the LDS reads
  const int mm = min(m, H - 1), jj = min(max(j, 0), g.ny - 1);
  const size_t ccol = (size_t)jj * g.nx + 2 * mm;
  const bool hrow = r == 0 || r == R - 1;
  const int jh = min(max(r == 0 ? j - 1 : j + 1, 0), g.ny - 1);
  const size_t chcol = (size_t)jh * g.nx + 2 * mm;
  const int arow = r == 0 ? 0 : R + 1;
  const int mw = m > 0 ? m - 1 : 0, me = m < W - 1 ? m + 1 : W - 1;
  const size_t dn = hn ? sy : 0, de = heo ? 2 : 0;
  auto pl = [&](int k) { return min(max(k, 0), g.nz - 1); };

  auto load = [&](int p, FaceCol<T>& L) {
    const int kq = pl(p);
    const int e1 = (c1 + j + p) & 1;
    const size_t c = (size_t)kq * sz + ccol;
    const T2 bv = load_pair(b, c), ws = load_pair(co.wy, c);
    const T2 wb = load_pair(co.wz, c), wx = load_pair(co.wx, c);
    L.b1 = e1 ? bv.y : bv.x;
    L.b2 = e1 ? bv.x : bv.y;
    L.wy0 = ws.x;
    L.wy1 = ws.y;
    if (r == R - 1) {
      const T2 hn2 = load_pair(co.wy, c + dn);
      L.hwy0 = hn2.x;
      L.hwy1 = hn2.y;
    }
    L.wb1 = e1 ? wb.y : wb.x;
    L.wb2 = e1 ? wb.x : wb.y;
    L.wx0 = wx.x;
    L.wx1 = wx.y;
    if ((m & 63) == 63) L.wxe = co.wx[c + de];
    if (kq == g.nz - 1) {
      const T2 tp = load_pair(co.tp, ccol);
      L.tp1 = e1 ? tp.y : tp.x;
      L.tp2 = e1 ? tp.x : tp.y;
    } else {
      L.tp1 = L.tp2 = T(0);
    }
    if (!FIRST) {
      L.xo = Xin[c + (e1 ^ 1)];
      if (hrow) L.hxo = Xin[(size_t)kq * sz + chcol + ((c1 + jh + p) & 1 ^ 1)];
    } else {
      L.xo = L.hxo = T(0);
    }
  };
  auto stage = [&](int p, const FaceCol<T>& L) {
    swy[p & 3][r + 1][m] = T2{L.wy0, L.wy1};
    if (r == R - 1) swy[p & 3][R + 1][m] = T2{L.hwy0, L.hwy1};
    if (!FIRST) {
      const int sl = p & (NS - 1);
      sx[sl][r + 1][m] = L.xo;
      if (hrow) sx[sl][arow][m] = L.hxo;
    }
  };
  // one colour update of the cell at position e of the pair (e = 0: cell
  // 2m), in the arithmetic order of k_gs_pair_face
  auto update = [&](int k, int e, T bv, T ws, T wn, T wb, T wt, T wx0, T wx1, T wxe, T xw, T xe, T xs, T xn,
                    T xb, T xt, bool first) {
    const bool top = k >= g.nz - 1;
    const T ww = e ? wx1 : (hwo ? wx0 : T(0)), we = e ? (heo ? wxe : T(0)) : wx1;
    const T wsv = hs ? ws : T(0), wnv = hn ? wn : T(0);
    const T D = (ww + we) * ix + (wsv + wnv) * iy + (k > 0 ? wb : T(2) * wb) * iz + (top ? T(2) * wt : wt) * iz;
    if (first) return bv * recip(D);
    T off = (ww * xw + we * xe) * ix + (wsv * xs + wnv * xn) * iy;
    off += k > 0 ? wb * iz * xb : T(0);
    off += !top ? wt * iz * xt : T(0);
    return (bv + off) * recip(D);
  };

  // history: index 0 = plane k-1, 1 = plane k, 2 = plane k+1 (after the
  // rotation at the top of iteration k)
  FaceCol<T> P0, P1, P2;
  T c1n[3] = {T(0), T(0), T(0)};  // new c1 of the column on planes k-2 .. k
  load(k0 - 2, P1);
  load(k0 - 1, P2);
  stage(k0 - 1, P2);
  lds_barrier();

  auto iterate = [&](int k, const FaceCol<T>& L) {
    P0 = P1;
    P1 = P2;
    P2 = L;
    stage(k + 1, L);
    // --- colour c1 on plane k ---
    const int e1 = (c1 + j + k) & 1;
    const int sl = k & (NS - 1);
    const bool top = k >= g.nz - 1;
    T xw = P1.xo, xe = P1.xo;  // the pair's other cell
    if (!FIRST) {
      if (e1) xe = sx[sl][r + 1][me];  // cell 2m + 2 (pair m + 1)
      else xw = sx[sl][r + 1][mw];     // cell 2m - 1 (pair m - 1)
    }
    const T xs = FIRST ? T(0) : sx[sl][r][m], xn = FIRST ? T(0) : sx[sl][r + 2][m];
    const bool wave_end = (m & 63) == 63;
    const T wxe1 = __shfl_down(P1.wx0, 1, 64), wxe2 = __shfl_down(P0.wx0, 1, 64);
    const T2 pn1 = swy[k & 3][r + 2][m];
    const T v1 = update(k, e1, P1.b1, e1 ? P1.wy1 : P1.wy0, e1 ? pn1.y : pn1.x, P1.wb1, top ? P1.tp1 : P2.wb2, P1.wx0, P1.wx1,
                        wave_end ? P1.wxe : wxe1, xw, xe, xs, xn, P0.xo, P2.xo, FIRST);
    if (owner && k >= k0 && k < k1) Xout[(size_t)k * sz + ccol + e1] = v1;
    c1n[0] = c1n[1];
    c1n[1] = c1n[2];
    c1n[2] = v1;
    ring[(k + 3) % 3][r][m] = v1;
    lds_barrier();
    // --- colour c2 on plane kk = k-1 ---
    const int kk = k - 1;
    if (owner && kk >= k0 && kk < k1) {
      const int e2 = ((c1 + j + kk) & 1) ^ 1;
      const int rl = (kk + 3) % 3;
      const T yw = e2 ? c1n[1] : ring[rl][r][mw];
      const T ye = e2 ? ring[rl][r][me] : c1n[1];
      const bool ktop = kk >= g.nz - 1;
      const T2 pn2 = swy[kk & 3][r + 2][m];
      const T v2 = update(kk, e2, P0.b2, e2 ? P0.wy1 : P0.wy0, e2 ? pn2.y : pn2.x, P0.wb2, ktop ? P0.tp2 : P1.wb1, P0.wx0, P0.wx1,
                          wave_end ? P0.wxe : wxe2, yw, ye, ring[rl][r - 1][m], ring[rl][r + 1][m], c1n[0], c1n[2],
                          false);
      Xout[(size_t)kk * sz + ccol + e2] = v2;
    }
  };

  // two load buffers: iteration k consumes plane k+1, loaded one iteration
  // earlier; loads past the grid read a clamped valid plane
  FaceCol<T> L[2];
  load(k0, L[0]);
  for (int k = k0 - 1; k <= k1; k += 4) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      load(k + t + 2, L[(t + 1) & 1]);
      if (k + t > k1) return;  // (an exit, not a break: no second path into the loop's back edge)
      iterate(k + t, L[t & 1]);
    }
  }
}

}  // namespace gmg
