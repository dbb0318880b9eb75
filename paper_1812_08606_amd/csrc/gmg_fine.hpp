// gmg_fine.hpp -- finest-level kernels on colour-split storage.
//
// On the finest level (at least two levels, so nx, ny, nz are even) the
// V-cycle iterate x (which becomes z = M v) and its right side b are stored
// by colour: X_c = X + c * hn holds, for every x-pair (2m, 2m+1) of row j on
// plane k, the one cell of the pair whose colour (i + j + k) % 2 is c, at
// index idx = (k * ny + j) * H + m, H = nx / 2.  In X_c at (m, j, k) sits the
// cell i = 2m + e, e = (c + j + k) % 2.
//
// A red-black half-sweep of colour c then reads only X_{1-c} (every
// neighbour of a colour-c cell has the other colour) and writes only X_c, in
// whole cache lines: the neighbours of the colour-c cell of pair m sit in
// X_{1-c} at m (the pair's other cell, and the cells above, below, north and
// south), and at m - 1 or m + 1 (the x-neighbour outside the pair).  The
// coefficient a stays in the natural (k, j, i) layout.
#pragma once

#include "gmg_kernels.hpp"

namespace gmg {

// Index of pair m of row j on plane k in a colour array.
__device__ __forceinline__ size_t sidx(const Geom& g, int m, int j, int k) {
  return ((size_t)k * g.ny + j) * (size_t)(g.nx >> 1) + m;
}

// Red-black half-sweep of colour `colour` (cell coefficient a, face = mean of
// the two cells).  Lane tx owns pair m = 64 bx + tx of row j = 4 by + ty and
// marches its z-chunk, keeping a of the pair and X_{1-c} at m on the planes
// k-1, k, k+1 in registers.  Every load of a plane is issued in one group
// with clamped (always valid) addresses and no branches -- the values behind
// a missing face are multiplied by zero weights -- and the group of plane k+1
// is issued before plane k is computed.  FIRST: the first pre-smoothing
// half-sweep from x = 0: b is read from the natural-layout u (times *bscale
// when SCALED), stored by colour into B for both cells, and X_c = b / D;
// X_{1-c} is left as it is (the next half-sweep overwrites it without
// reading it).
constexpr int SPLIT_BATCH = 2;  // planes whose loads are issued together
constexpr int GS_ROWS = 4;      // rows per block of the finest-level half-sweep

template <typename T>
struct SplitSide {
  T at0, at1;    // a of the pair on plane k+1
  T xot;         // X_{1-c} at m on plane k+1
  T as, an;      // a of the updated cell's south / north neighbours
  T xs, xn;      // X_{1-c} at m on rows j-1 / j+1
  T aout, xout;  // a and X_{1-c} of the x-neighbour outside the pair
  T b0, b1;      // right side (FIRST: of both cells of the pair; else b0 = B_c)
};

template <typename T, bool FIRST, bool SCALED>
__device__ __forceinline__ void split_side_load(SplitSide<T>& S, const T* __restrict__ Xo, const T* __restrict__ Bc,
                                                const double* __restrict__ u, double s, const T* __restrict__ a,
                                                const Geom& g, int H, int m, int j, int k, int colour, bool act) {
  const size_t ty = (size_t)H, tz = (size_t)H * g.ny;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const int e = (colour + j + k) & 1;
  const int kk = act ? k : 0, jj = act ? j : 0, mm = act ? m : 0;
  const size_t q = sidx(g, mm, jj, kk), cn = 2 * q, ce = cn + e;
  const bool up = act && kk + 1 < g.nz;
  const size_t qt = up ? q + tz : q, ct = up ? cn + sz : cn;
  const size_t dys = (act && jj > 0) ? ty : 0, dyn = (act && jj < g.ny - 1) ? ty : 0;
  const size_t das = (act && jj > 0) ? sy : 0, dan = (act && jj < g.ny - 1) ? sy : 0;
  // outside the pair: cell 2m-1 (e = 0) or 2m+2 (e = 1), clamped to the pair
  const bool hout = act && (e ? mm < H - 1 : mm > 0);
  const size_t qo = hout ? (e ? q + 1 : q - 1) : q;
  const size_t co = hout ? (e ? cn + 2 : cn - 1) : ce;
  S.at0 = a[ct];
  S.at1 = a[ct + 1];
  S.as = a[ce - das];
  S.an = a[ce + dan];
  S.aout = a[co];
  if (!FIRST) {
    S.xot = Xo[qt];
    S.xs = Xo[q - dys];
    S.xn = Xo[q + dyn];
    S.xout = Xo[qo];
    S.b0 = Bc[q];
    S.b1 = T(0);
  } else {
    S.xot = S.xs = S.xn = S.xout = T(0);
    S.b0 = (T)(SCALED ? u[cn] * s : u[cn]);
    S.b1 = (T)(SCALED ? u[cn + 1] * s : u[cn + 1]);
  }
}

template <typename T, bool FIRST, bool SCALED>
__global__ __launch_bounds__(BX* GS_ROWS) void k_gs_split(T* __restrict__ X, T* __restrict__ B,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ bscale, const T* __restrict__ a,
                                                       Geom g, size_t hn, int kc, int colour) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * GS_ROWS + threadIdx.y;
  const bool act = m < H && j < g.ny;
  const size_t sz = (size_t)g.nx * g.ny, tz = (size_t)H * g.ny;
  const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2), pz = (T)(2.0 * g.ihz2);
  const double s = SCALED ? *bscale : 1.0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  const bool hs = j > 0, hn_ = j < g.ny - 1;
  T* __restrict__ Xc = X + (size_t)colour * hn;
  const T* __restrict__ Xo = X + (size_t)(1 - colour) * hn;
  T* __restrict__ Bc = B + (size_t)colour * hn;
  T* __restrict__ Bo = B + (size_t)(1 - colour) * hn;
  // planes k and k-1 (clamped loads; plane k0-1 is used only when k0 > 0)
  T ac0, ac1, ab0, ab1, xo = T(0), xob = T(0);
  {
    const size_t q = act ? sidx(g, m, j, k0) : 0, cn = 2 * q;
    const size_t qb = (act && k0 > 0) ? q - tz : q, cb = (act && k0 > 0) ? cn - sz : cn;
    ac0 = a[cn];
    ac1 = a[cn + 1];
    ab0 = a[cb];
    ab1 = a[cb + 1];
    if (!FIRST) {
      xo = Xo[q];
      xob = Xo[qb];
    }
  }
  // update of plane k from its loaded values Sc
  auto plane = [&](int k, const SplitSide<T>& Sc) {
    const bool top = k == g.nz - 1;
    const int e = (colour + j + k) & 1;  // element of the pair being updated
    const bool hout = e ? m < H - 1 : m > 0;
    const T acv = e ? ac1 : ac0, ain = e ? ac0 : ac1;
    const T abv = e ? ab1 : ab0, atv = e ? Sc.at1 : Sc.at0;
    const T wi = (acv + ain) * hx;
    const T wo = hout ? (acv + Sc.aout) * hx : T(0);
    const T ws = hs ? (acv + Sc.as) * hy : T(0);
    const T wn = hn_ ? (acv + Sc.an) * hy : T(0);
    const T wb = k > 0 ? (acv + abv) * hz : T(0);
    const T wt = !top ? (acv + atv) * hz : T(0);
    const T D = wi + wo + ws + wn + (k > 0 ? wb : pz * acv) + (!top ? wt : pz * acv);
    if (act) {
      const size_t q = sidx(g, m, j, k);
      if (FIRST) {
        const T bc = e ? Sc.b1 : Sc.b0;
        Bc[q] = bc;
        Bo[q] = e ? Sc.b0 : Sc.b1;
        Xc[q] = bc * recip(D);
      } else {
        const T off = wi * xo + wo * Sc.xout + ws * Sc.xs + wn * Sc.xn + wb * xob + wt * Sc.xot;
        Xc[q] = (Sc.b0 + off) * recip(D);
      }
    }
    ab0 = ac0;
    ab1 = ac1;
    ac0 = Sc.at0;
    ac1 = Sc.at1;
    xob = xo;
    xo = Sc.xot;
  };
  // planes in batches of SPLIT_BATCH: the loads of a whole batch are issued
  // before its first plane is updated (planes past the chunk load a valid
  // clamped plane and are not updated)
  for (int k = k0; k < k1; k += SPLIT_BATCH) {
    SplitSide<T> S[SPLIT_BATCH];
#pragma unroll
    for (int t = 0; t < SPLIT_BATCH; ++t)
      split_side_load<T, FIRST, SCALED>(S[t], Xo, Bc, u, s, a, g, H, m, j, min(k + t, k1 - 1), colour, act);
#pragma unroll
    for (int t = 0; t < SPLIT_BATCH; ++t)
      if (k + t < k1) plane(k + t, S[t]);
  }
}

// Values of the pair (left = cell 2m, right = cell 2m+1) at colour-array
// index q on a row/plane whose cell 2m has colour p.
template <typename TO, typename T>
__device__ __forceinline__ void split_pair(const T* __restrict__ X, size_t hn, size_t q, int p, TO& l, TO& r) {
  const TO v0 = (TO)X[q], v1 = (TO)X[q + hn];
  l = p ? v1 : v0;
  r = p ? v0 : v1;
}

// Barrier for data exchanged through LDS only: waits for this wave's LDS
// operations, not for its global loads in flight (a __syncthreads would also
// wait for those).  The signal fences keep the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt not waited for
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One symmetric red-black sweep in one pass: colour c1 everywhere from the
// old iterate Xin, then colour c2 from the new c1 values (pre-smoothing c1 =
// red, post-smoothing c1 = black), written to Xout (colour-split, both
// colours).  It equals two half-sweeps: the c1 update reads only old c2
// values, the c2 update only new c1 values.
//
// Block: 64 lanes x R rows (R = 16 in float32, 8 in float64); lane tx owns
// pair m = 62 bx + tx - 1 of row j = (R-2) by + ty - 1, marching a z-chunk.
// Lanes 0 and 63 and rows 0 and R-1 are a halo: they compute the c1 values
// their neighbours need (the same arithmetic as the block that owns those
// cells) but store nothing.  On iteration k the block updates c1 on plane k,
// puts the new values into an LDS ring, waits at a barrier, and updates c2
// on plane k-1 from the new c1 values of planes k-2, k-1, k: its own column
// from registers, rows j-1 and j+1 from LDS, the x-neighbour outside the
// pair from the adjacent lane.  Planes k0-1 and k1 of the chunk are computed
// (c1 only) for the same reason and not stored.  FIRST: the first sweep
// from x = 0 (c1 = b / D; b from the natural-layout u times *bscale when
// SCALED, stored by colour into B).
//
// Each thread loads only its own column of every plane -- the coefficient
// pair, the old colour-c2 value and the two right sides -- and stages the
// coefficient pair and the old c2 value in LDS, where rows j-1 and j+1 read
// them (rows 0 and R-1 of the block also load and stage the row beyond the
// block): 4 loads per thread and plane, each cache line requested once per
// block.  (Loading the side rows from global memory as well, 14 loads per
// thread and plane with every line requested by three rows, took 0.66-0.70
// ms per sweep at 512^3 against 0.50 ms.)  LDS holds NS = 4 planes of side
// values: plane k+1 is staged at iteration k, read at iterations k+1 and
// k+2, and its slot is rewritten four iterations later, after two barriers.
//
// Block shape: SX = 64 lanes per row (one row per wave; 32-lane rows were
// measured slower) times R rows; the block owns (SX - 2) x (R - 2) pairs.
// Float64 takes 12 rows: 1024 threads would leave too few registers per
// thread (measured at 512^3: 1.16, 1.03 and 1.12 ms per sweep with 8, 12
// and 16 rows, the last spilling).
template <typename T>
struct SymShape {
  static constexpr int SX = 64;
  static constexpr int R = sizeof(T) == 4 ? 16 : 12;
  static constexpr int IX = SX - 2;  // pairs per block row that the block owns
  static constexpr int IY = R - 2;   // rows the block owns
};
// Planes whose loads are in flight (the loads of iteration k+1 are issued
// before iteration k runs; a third buffer was slower), and iterations per
// loop trip: a multiple of SYM_DEPTH, so the load buffers rotate whole
// periods per trip and no value still in flight is copied at the back edge
// (copying one makes the compiler wait for every load).
constexpr int SYM_DEPTH = 2;
constexpr int SYM_UNROLL = 4;
static_assert(SYM_UNROLL % SYM_DEPTH == 0, "the load buffers must rotate whole periods per trip");

template <typename T>
struct SymCol {
  T a0, a1;         // a of the pair (cells 2m, 2m+1)
  T xo;             // old value of colour c2 at the pair
  T b1, b2;         // right side of the pair's c1 and c2 cells
  T ha0, ha1, hxo;  // rows 0 and R-1: a pair and old c2 of the row beyond the block
};

template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
  using type = float2;
};
template <>
struct Pair2<double> {
  using type = double2;
};

// The coefficient pair (cells 2m, 2m+1) at natural index cn (even): one
// 8-byte load in float32 (the workspace copy is 256-byte aligned); two loads
// in float64, where a is the caller's array, only 8-byte aligned.
template <typename T>
__device__ __forceinline__ typename Pair2<T>::type load_pair(const T* __restrict__ a, size_t cn) {
  if constexpr (sizeof(T) == 4) {
    return *reinterpret_cast<const float2*>(a + cn);
  } else {
    return typename Pair2<T>::type{a[cn], a[cn + 1]};
  }
}

template <typename T, bool FIRST, bool SCALED>
__global__ __launch_bounds__(SymShape<T>::SX* SymShape<T>::R) void k_sym_split(const T* __restrict__ Xin,
                                                                             T* __restrict__ Xout,
                                                                             T* __restrict__ B,
                                                                             const double* __restrict__ u,
                                                                             const double* __restrict__ bscale,
                                                                             const T* __restrict__ a, Geom g,
                                                                             size_t hn, int kc, int c1) {
  using T2 = typename Pair2<T>::type;
  constexpr int SX = SymShape<T>::SX, IX = SymShape<T>::IX, R = SymShape<T>::R, IY = SymShape<T>::IY;
  constexpr int NS = 4;              // planes of side values held in LDS
  __shared__ T2 sa[NS][R + 2][SX];  // a pairs of block rows -1 .. R (array rows 0 .. R+1)
  __shared__ T so[NS][R + 2][SX];   // old values of colour c2, same rows
  __shared__ T ring[3][R][SX];      // new c1 values of planes k-1, k, k+1 (mod 3)
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int lane = threadIdx.x, r = threadIdx.y;
  const int m = tl.x * IX + lane - 1;
  const int j = tl.y * IY + r - 1;
  const bool ing = m >= 0 && m < H && j >= 0 && j < g.ny;
  const bool owner = ing && lane >= 1 && lane <= IX && r >= 1 && r <= IY;
  const int c2 = 1 - c1;
  const size_t tz = (size_t)H * g.ny;
  const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2), pz = (T)(2.0 * g.ihz2);
  const double s = SCALED ? *bscale : 1.0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  // faces outside the pair (false for threads outside the grid, whose
  // addresses are clamped to it)
  const bool hw = m > 0 && m < H, he = m >= 0 && m < H - 1, hs = j > 0, hn_ = j < g.ny - 1;
  // clamped (always valid) column of this thread, and of the row beyond the
  // block that rows 0 and R-1 stage (array row 0 or R+1)
  const int mm = min(max(m, 0), H - 1), jj = min(max(j, 0), g.ny - 1);
  const size_t qcol = (size_t)jj * H + mm;
  const bool hrow = r == 0 || r == R - 1;
  const int jh = min(max(r == 0 ? j - 1 : j + 1, 0), g.ny - 1);
  const size_t qhcol = (size_t)jh * H + mm;
  const int arow = r == 0 ? 0 : R + 1;
  const T* __restrict__ Xo = Xin + (size_t)c2 * hn;  // old values of colour c2
  T* __restrict__ Y1 = Xout + (size_t)c1 * hn;
  T* __restrict__ Y2 = Xout + (size_t)c2 * hn;
  T* __restrict__ B1 = B + (size_t)c1 * hn;
  T* __restrict__ B2 = B + (size_t)c2 * hn;
  auto pl = [&](int k) { return min(max(k, 0), g.nz - 1); };

  auto load = [&](int p, SymCol<T>& L) {
    const int kq = pl(p);
    const size_t q = (size_t)kq * tz + qcol, cn = 2 * q;
    const T2 av = load_pair(a, cn);
    L.a0 = av.x;
    L.a1 = av.y;
    if (!FIRST) {
      L.xo = Xo[q];
      L.b1 = B1[q];
      L.b2 = B2[q];
    } else {
      const double2 uv = *reinterpret_cast<const double2*>(u + cn);
      const T u0 = (T)(SCALED ? uv.x * s : uv.x), u1 = (T)(SCALED ? uv.y * s : uv.y);
      const int e1 = (c1 + j + p) & 1;
      L.b1 = e1 ? u1 : u0;
      L.b2 = e1 ? u0 : u1;
      L.xo = T(0);
    }
    if (hrow) {
      const size_t qh = (size_t)kq * tz + qhcol;
      const T2 hv = load_pair(a, 2 * qh);
      L.ha0 = hv.x;
      L.ha1 = hv.y;
      L.hxo = FIRST ? T(0) : Xo[qh];
    }
  };
  auto stage = [&](int p, const SymCol<T>& L) {
    const int sl = p & (NS - 1);
    sa[sl][r + 1][lane] = T2{L.a0, L.a1};
    so[sl][r + 1][lane] = L.xo;
    if (hrow) {
      sa[sl][arow][lane] = T2{L.ha0, L.ha1};
      so[sl][arow][lane] = L.hxo;
    }
  };

  // registers: a of the pair on planes k-2 .. k+1, old c2 of the column on
  // k-1 .. k+1, new c1 of the column on k-2 .. k; right sides: c1 and c2 of
  // plane k (cb1, cb2), c2 of plane k-1 (pb2)
  T a0[4], a1[4], xo[3], c1n[3], cb1, cb2, pb2 = T(0);
#pragma unroll
  for (int t = 0; t < 3; ++t) c1n[t] = T(0);
  a0[0] = a1[0] = a0[1] = a1[1] = T(0);
  xo[0] = T(0);
  {
    // plane k0-2 (own column only) and plane k0-1 (staged), rotated into
    // place at the top of the first iteration
    SymCol<T> Lb, Lc;
    load(k0 - 2, Lb);
    load(k0 - 1, Lc);
    a0[2] = Lb.a0;
    a1[2] = Lb.a1;
    xo[1] = Lb.xo;
    a0[3] = Lc.a0;
    a1[3] = Lc.a1;
    xo[2] = Lc.xo;
    cb1 = Lc.b1;
    cb2 = Lc.b2;
    stage(k0 - 1, Lc);
  }
  lds_barrier();

  // iteration k: stage plane k+1, colour c1 on plane k, colour c2 on plane k-1
  auto iterate = [&](int k, const SymCol<T>& L) {
    a0[0] = a0[1];
    a1[0] = a1[1];
    a0[1] = a0[2];
    a1[1] = a1[2];
    a0[2] = a0[3];
    a1[2] = a1[3];
    a0[3] = L.a0;
    a1[3] = L.a1;
    xo[0] = xo[1];
    xo[1] = xo[2];
    xo[2] = L.xo;
    stage(k + 1, L);
    // (a0[3] is plane k+1, a0[2] plane k, a0[1] plane k-1, a0[0] plane k-2;
    // xo[2] plane k+1, xo[1] plane k, xo[0] plane k-1)
    const int e1 = (c1 + j + k) & 1;
    const bool hout = e1 ? he : hw;
    // a and old c2 of the cell outside the pair: element 0 of pair m+1
    // (e1 = 1) or element 1 of pair m-1 (e1 = 0), from the adjacent lane
    const int src = lane + (e1 ? 1 : -1);
    const T aout = __shfl(e1 ? a0[2] : a1[2], src, SX);
    const T xout = __shfl(xo[1], src, SX);
    T v1;
    {
      const int sl = k & (NS - 1);
      const T2 ps = sa[sl][r][lane], pn = sa[sl][r + 2][lane];
      const bool top = k >= g.nz - 1, bot = k <= 0;
      const T acv = e1 ? a1[2] : a0[2], ain = e1 ? a0[2] : a1[2];
      const T abv = e1 ? a1[1] : a0[1], atv = e1 ? a1[3] : a0[3];
      const T wi = (acv + ain) * hx;
      const T wo = hout ? (acv + aout) * hx : T(0);
      const T ws = hs ? (acv + (e1 ? ps.y : ps.x)) * hy : T(0);
      const T wn = hn_ ? (acv + (e1 ? pn.y : pn.x)) * hy : T(0);
      const T wb = !bot ? (acv + abv) * hz : T(0);
      const T wt = !top ? (acv + atv) * hz : T(0);
      const T D = wi + wo + ws + wn + (!bot ? wb : pz * acv) + (!top ? wt : pz * acv);
      if (FIRST) {
        v1 = cb1 * recip(D);
      } else {
        const T xs = so[sl][r][lane], xn = so[sl][r + 2][lane];
        const T off = wi * xo[1] + (hout ? wo * xout : T(0)) + (hs ? ws * xs : T(0)) + (hn_ ? wn * xn : T(0)) +
                      (!bot ? wb * xo[0] : T(0)) + (!top ? wt * xo[2] : T(0));
        v1 = (cb1 + off) * recip(D);
      }
      if (owner && k >= k0 && k < k1) {
        const size_t q = (size_t)k * tz + qcol;
        Y1[q] = v1;
        if (FIRST) {
          B1[q] = cb1;
          B2[q] = cb2;
        }
      }
    }
    c1n[0] = c1n[1];
    c1n[1] = c1n[2];
    c1n[2] = v1;
    ring[(k + 3) % 3][r][lane] = v1;
    lds_barrier();
    // --- colour c2 on plane kk = k-1 ---
    const int kk = k - 1;
    const int e2 = (c2 + j + kk) & 1;
    // x-neighbour outside the pair (the adjacent lane's values on plane kk)
    const int src2 = lane + (e2 ? 1 : -1);
    const T cov = __shfl(c1n[1], src2, SX);
    const T aov = __shfl(e2 ? a0[1] : a1[1], src2, SX);
    if (owner && kk >= k0 && kk < k1) {
      const int sl = kk & (NS - 1);
      const T2 ps = sa[sl][r][lane], pn = sa[sl][r + 2][lane];
      const bool top = kk == g.nz - 1, bot = kk == 0;
      const bool ho = e2 ? he : hw;
      const T acv = e2 ? a1[1] : a0[1], ain = e2 ? a0[1] : a1[1];
      const T abv = e2 ? a1[0] : a0[0], atv = e2 ? a1[2] : a0[2];
      const T wi = (acv + ain) * hx;
      const T wo = ho ? (acv + aov) * hx : T(0);
      const T ws = hs ? (acv + (e2 ? ps.y : ps.x)) * hy : T(0);
      const T wn = hn_ ? (acv + (e2 ? pn.y : pn.x)) * hy : T(0);
      const T wb = !bot ? (acv + abv) * hz : T(0);
      const T wt = !top ? (acv + atv) * hz : T(0);
      const T D = wi + wo + ws + wn + (!bot ? wb : pz * acv) + (!top ? wt : pz * acv);
      const int rl = (kk + 3) % 3;
      const T ys = ring[rl][r - 1][lane], yn = ring[rl][r + 1][lane];
      const T off = wi * c1n[1] + (ho ? wo * cov : T(0)) + (hs ? ws * ys : T(0)) + (hn_ ? wn * yn : T(0)) +
                    (!bot ? wb * c1n[0] : T(0)) + (!top ? wt * c1n[2] : T(0));
      Y2[(size_t)kk * tz + qcol] = (pb2 + off) * recip(D);
    }
    pb2 = cb2;
    cb1 = L.b1;
    cb2 = L.b2;
  };

  // SYM_DEPTH load buffers: iteration k consumes plane k+1, whose loads were
  // issued SYM_DEPTH - 1 iterations earlier into the buffer the iteration
  // before them released; loads past the grid read a clamped valid plane
  SymCol<T> L[SYM_DEPTH];
#pragma unroll
  for (int t = 0; t < SYM_DEPTH - 1; ++t) load(k0 + t, L[t]);
  for (int k = k0 - 1; k <= k1; k += SYM_UNROLL) {
#pragma unroll
    for (int t = 0; t < SYM_UNROLL; ++t) {
      load(k + t + SYM_DEPTH, L[(t + SYM_DEPTH - 1) % SYM_DEPTH]);
      if (k + t > k1) return;  // (an exit, not a break: no second path into the loop's back edge)
      iterate(k + t, L[t % SYM_DEPTH]);
    }
  }
}

// Residual and restriction from the colour-split iterate and right side:
// b_coarse = mean over the 8 children of (b - A x).  Lane tx owns pair m
// (= the coarse x-index) of fine row j and marches the fine planes of its
// z-chunk, 2 per coarse plane, keeping x and a of the pair on planes k-1, k
// in registers; the loads of both fine planes of a coarse plane are issued in
// one branch-free group with clamped addresses.  The two fine rows of a
// coarse row are summed through LDS.  kc counts coarse planes.
template <typename T>
struct ResidSide {
  T xt0, xt1, at0, at1;  // pair on plane k+1
  T xs0, xs1, as0, as1;  // pair on row j-1
  T xn0, xn1, an0, an1;  // pair on row j+1
  T xw, aw, xe, ae;      // cells 2m-1 and 2m+2
  T b0, b1;              // right side of the pair
};

template <typename T>
__device__ __forceinline__ void resid_side_load(ResidSide<T>& S, const T* __restrict__ X, const T* __restrict__ B,
                                                const T* __restrict__ a, const Geom& g, size_t hn, int H, int m,
                                                int j, int k, bool act) {
  const size_t ty = (size_t)H, tz = (size_t)H * g.ny;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const int kk = act ? k : 0, jj = act ? j : 0, mm = act ? m : 0;
  const int p = (jj + kk) & 1;  // colour of cell 2m on row j, plane k
  const size_t q = sidx(g, mm, jj, kk), cn = 2 * q;
  const bool up = kk + 1 < g.nz;
  const size_t qt = up ? q + tz : q, ct = up ? cn + sz : cn;
  const size_t qs = jj > 0 ? q - ty : q, cs = jj > 0 ? cn - sy : cn;
  const size_t qn = jj < g.ny - 1 ? q + ty : q, cnn = jj < g.ny - 1 ? cn + sy : cn;
  split_pair(X, hn, qt, p ^ 1, S.xt0, S.xt1);
  S.at0 = a[ct];
  S.at1 = a[ct + 1];
  split_pair(X, hn, qs, p ^ 1, S.xs0, S.xs1);
  S.as0 = a[cs];
  S.as1 = a[cs + 1];
  split_pair(X, hn, qn, p ^ 1, S.xn0, S.xn1);
  S.an0 = a[cnn];
  S.an1 = a[cnn + 1];
  // cell 2m-1 has colour p^1, cell 2m+2 colour p (clamped to the pair)
  S.xw = X[(mm > 0 ? q - 1 : q) + (size_t)(p ^ 1) * hn];
  S.aw = a[mm > 0 ? cn - 1 : cn];
  S.xe = X[(mm < H - 1 ? q + 1 : q) + (size_t)p * hn];
  S.ae = a[mm < H - 1 ? cn + 2 : cn];
  split_pair(B, hn, q, p, S.b0, S.b1);
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_resid_restrict_split(const T* __restrict__ X, const T* __restrict__ B,
                                                                   const T* __restrict__ a, Geom g, size_t hn,
                                                                   T* __restrict__ bc, int kc) {
  __shared__ T part[BY][BX];
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1, NY = g.ny >> 1, NZ = g.nz >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  const bool act = m < H && j < g.ny;
  const size_t tz = (size_t)H * g.ny, sz = (size_t)g.nx * g.ny;
  const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2), pz = (T)(2.0 * g.ihz2);
  const int K0 = tl.z * kc, K1 = min(NZ, K0 + kc);
  const bool hw = m > 0, he = m < H - 1, hs = j > 0, hn_ = j < g.ny - 1;
  // pair registers: [0] cell 2m, [1] cell 2m+1, planes k-1 and k
  T xb[2], xc[2], ab[2], ac[2];
  {
    const int k0 = 2 * K0;
    const size_t q = act ? sidx(g, m, j, k0) : 0, cn = 2 * q;
    const int p = act ? (j + k0) & 1 : 0;
    const bool dn = act && k0 > 0;
    split_pair(X, hn, q, p, xc[0], xc[1]);
    split_pair(X, hn, dn ? q - tz : q, p ^ 1, xb[0], xb[1]);
    ac[0] = a[cn];
    ac[1] = a[cn + 1];
    ab[0] = a[dn ? cn - sz : cn];
    ab[1] = a[dn ? cn - sz + 1 : cn + 1];
  }
  auto plane = [&](int k, const ResidSide<T>& S) -> T {
    const bool top = k == g.nz - 1;
    const T xt[2] = {S.xt0, S.xt1}, at[2] = {S.at0, S.at1};
    const T xs[2] = {S.xs0, S.xs1}, as_[2] = {S.as0, S.as1};
    const T xn[2] = {S.xn0, S.xn1}, an[2] = {S.an0, S.an1};
    const T bv[2] = {S.b0, S.b1};
    T rsum = T(0);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const T acv = ac[e], xcv = xc[e];
      const T xo = e == 0 ? S.xw : S.xe, ao = e == 0 ? S.aw : S.ae;
      const bool ho = e == 0 ? hw : he;
      T Ax = (acv + ac[1 - e]) * hx * (xcv - xc[1 - e]);
      Ax += ho ? (acv + ao) * hx * (xcv - xo) : T(0);
      Ax += hs ? (acv + as_[e]) * hy * (xcv - xs[e]) : T(0);
      Ax += hn_ ? (acv + an[e]) * hy * (xcv - xn[e]) : T(0);
      Ax += k > 0 ? (acv + ab[e]) * hz * (xcv - xb[e]) : pz * acv * xcv;
      Ax += !top ? (acv + at[e]) * hz * (xcv - xt[e]) : pz * acv * xcv;
      rsum += bv[e] - Ax;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      xb[e] = xc[e];
      xc[e] = xt[e];
      ab[e] = ac[e];
      ac[e] = at[e];
    }
    return rsum;
  };
  for (int K = K0; K < K1; ++K) {
    ResidSide<T> S0, S1;
    resid_side_load(S0, X, B, a, g, hn, H, m, j, 2 * K, act);
    resid_side_load(S1, X, B, a, g, hn, H, m, j, 2 * K + 1, act);
    T acc = plane(2 * K, S0);
    acc += plane(2 * K + 1, S1);
    // both fine planes of coarse plane K done: add the row pair
    part[threadIdx.y][threadIdx.x] = acc;
    __syncthreads();
    if (!(threadIdx.y & 1) && act) {
      const T tot = acc + part[threadIdx.y + 1][threadIdx.x];
      bc[((size_t)K * NY + (j >> 1)) * H + m] = tot * T(0.125);
    }
    __syncthreads();
  }
}

// x_fine += P x_coarse, cell-centred trilinear (per dimension 3/4 of the
// parent and 1/4 of the nearer coarse neighbour; outside the grid the
// neighbour is the parent (x, y: Neumann) or minus the parent (z: plates)).
// Lane tx owns pair m of fine row j -- m is also the parent's coarse x-index
// -- and marches the coarse planes of its z-chunk (kc of them), keeping the
// row- and x-interpolated coarse values of planes K-1, K, K+1 in registers;
// coarse plane K feeds fine planes 2K (with K-1) and 2K+1 (with K+1).  The
// two cells of a pair differ only in their x-neighbour (m-1 for cell 2m, m+1
// for cell 2m+1).  SPLIT: the fine x is colour-split and only the colours
// in the bit mask cmask (1 red, 2 black) are written; otherwise the fine x
// is natural (every cell).
// SET: x = P xc (the interpolated initial guess of a full multigrid cycle)
// instead of x += P xc.
template <typename T, bool SPLIT, bool SET = false>
__global__ __launch_bounds__(NTHREADS) void k_prolong_pair(T* __restrict__ x, const T* __restrict__ xc, Geom g,
                                                           size_t hn, int cmask, int kc) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (m >= H || j >= g.ny) return;
  const int NX = H, NY = g.ny >> 1, NZ = g.nz >> 1;
  const T q3 = T(0.75), q1 = T(0.25);
  const int J = j >> 1;
  int J2 = J + ((j & 1) ? 1 : -1);
  if (J2 < 0 || J2 >= NY) J2 = J;
  const int Il = m > 0 ? m - 1 : m, Ir = m < NX - 1 ? m + 1 : m;
  const size_t rJ = (size_t)J * NX, rJ2 = (size_t)J2 * NX, sZ = (size_t)NY * NX;
  auto interp = [&](int K, T& left, T& right) {
    const T* p = xc + (size_t)K * sZ;
    const T c0 = p[rJ + m], cl = p[rJ + Il], cr = p[rJ + Ir];
    const T d0 = p[rJ2 + m], dl = p[rJ2 + Il], dr = p[rJ2 + Ir];
    left = q3 * (q3 * c0 + q1 * cl) + q1 * (q3 * d0 + q1 * dl);
    right = q3 * (q3 * c0 + q1 * cr) + q1 * (q3 * d0 + q1 * dr);
  };
  const int K0 = tl.z * kc, K1 = min(NZ, K0 + kc);
  T lb, rb, lc, rc, lt, rt;  // coarse planes K-1, K, K+1 (left / right variant)
  interp(K0, lc, rc);
  if (K0 > 0) {
    interp(K0 - 1, lb, rb);
  } else {
    lb = -lc;
    rb = -rc;
  }
  for (int K = K0; K < K1; ++K) {
    if (K + 1 < NZ) {
      interp(K + 1, lt, rt);
    } else {
      lt = -lc;
      rt = -rc;
    }
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      const int k = 2 * K + sub;
      const T vl = q3 * lc + q1 * (sub ? lt : lb);  // cell 2m
      const T vr = q3 * rc + q1 * (sub ? rt : rb);  // cell 2m+1
      if (SPLIT) {
        for (int c = 0; c < 2; ++c) {
          if (!((cmask >> c) & 1)) continue;
          const int e = (c + j + k) & 1;
          T& dst = x[(size_t)c * hn + sidx(g, m, j, k)];
          dst = SET ? (e ? vr : vl) : dst + (e ? vr : vl);
        }
      } else {
        const size_t cn = ((size_t)k * g.ny + j) * g.nx + 2 * m;
        x[cn] = SET ? vl : x[cn] + vl;
        x[cn + 1] = SET ? vr : x[cn + 1] + vr;
      }
    }
    lb = lc;
    rb = rc;
    lc = lt;
    rc = rt;
  }
}

// Right sides of a full multigrid cycle on the finest level: B = s u stored
// by colour (s = *bscale, or 1 when bscale is null; rounded to T) and the
// next level's right side bc = mean over the 8 children of the rounded
// values.  One thread per coarse cell, reading its children as x-pairs.
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_restrict_split_rhs(const double* __restrict__ u,
                                                                 const double* __restrict__ bscale,
                                                                 T* __restrict__ B, T* __restrict__ bc, Geom g,
                                                                 size_t hn) {
  const int H = g.nx >> 1, NY = g.ny >> 1;
  const int I = blockIdx.x * BX + threadIdx.x;
  const int J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= H || J >= NY) return;
  const double s = bscale ? *bscale : 1.0;
  T sum = T(0);
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
      const int j = 2 * J + dj, k = 2 * K + dk;
      const size_t cn = ((size_t)k * g.ny + j) * g.nx + 2 * I;
      const double2 v = *reinterpret_cast<const double2*>(u + cn);
      const T v0 = (T)(v.x * s), v1 = (T)(v.y * s);
      const size_t q = sidx(g, I, j, k);
      const int e = (j + k) & 1;  // colour of cell 2I
      B[(size_t)e * hn + q] = v0;
      B[(size_t)(1 - e) * hn + q] = v1;
      sum += v0 + v1;
    }
  bc[((size_t)K * NY + J) * H + I] = sum * T(0.125);
}

// bc = mean over the 8 children of b (natural layout, every dimension even).
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_restrict_mean(const T* __restrict__ b, T* __restrict__ bc, Geom g) {
  const int NX = g.nx >> 1, NY = g.ny >> 1;
  const int I = blockIdx.x * BX + threadIdx.x;
  const int J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= NX || J >= NY) return;
  T sum = T(0);
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj) {
      const size_t cn = ((size_t)(2 * K + dk) * g.ny + 2 * J + dj) * g.nx + 2 * I;
      sum += b[cn] + b[cn + 1];
    }
  bc[((size_t)K * NY + J) * NX + I] = sum * T(0.125);
}

// Weights of the 1-D transpose of the cell-centred linear interpolation for
// coarse index I of n: fine cells 2I-1 .. 2I+2 weigh 1/4, 3/4, 3/4, 1/4; a
// fine cell outside the grid gets weight 0 (its address is clamped) and the
// ghost it stands for folds onto the end cell with sign sg (+1 mirror, -1
// negated mirror).
__device__ __forceinline__ void fw_weights(int I, int n, double sg, int idx[4], double w[4]) {
  const int nf = 2 * n;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int f = 2 * I - 1 + t;
    idx[t] = min(max(f, 0), nf - 1);
    w[t] = (t == 0 || t == 3) ? 0.25 : 0.75;
  }
  if (I == 0) {
    w[0] = 0.0;
    w[1] += 0.25 * sg;
  }
  if (I == n - 1) {
    w[3] = 0.0;
    w[2] += 0.25 * sg;
  }
}

// bc = P^T r / 8: the transpose of the trilinear prolongation (negated
// mirror through the plates, mirror on the sides) applied to the fine
// residual r (natural layout, fine geometry g, every dimension even),
// i.e. full weighting over the 4 x 4 x 4 fine cells around each coarse cell.
// One thread per coarse cell; sums in float64.
template <typename TI, typename TO>
__global__ __launch_bounds__(NTHREADS) void k_restrict_fw(const TI* __restrict__ r, TO* __restrict__ bc, Geom g) {
  const int NX = g.nx >> 1, NY = g.ny >> 1, NZ = g.nz >> 1;
  const int I = blockIdx.x * BX + threadIdx.x;
  const int J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= NX || J >= NY) return;
  int ix[4], iy[4], iz[4];
  double wx[4], wy[4], wz[4];
  fw_weights(I, NX, 1.0, ix, wx);
  fw_weights(J, NY, 1.0, iy, wy);
  fw_weights(K, NZ, -1.0, iz, wz);
  double sum = 0.0;
#pragma unroll
  for (int tk = 0; tk < 4; ++tk) {
    double sy = 0.0;
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      const size_t row = ((size_t)iz[tk] * g.ny + iy[tj]) * g.nx;
      double sx = 0.0;
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) sx += wx[ti] * (double)r[row + ix[ti]];
      sy += wy[tj] * sx;
    }
    sum += wz[tk] * sy;
  }
  bc[((size_t)K * NY + J) * NX + I] = (TO)(0.125 * sum);
}

// w = A z (z colour-split, promoted to float64) and the dots (w, u_v),
// v < NV.  Lane tx owns pair m of row j (rows strided by the grid's y extent)
// and marches its z-chunk keeping z and a of the pair on planes k-1, k, k+1
// in registers; the x-neighbours outside the pair come from the adjacent
// lanes.
template <typename TZ, int NV>
__global__ __launch_bounds__(NTHREADS) void k_op_multidot_split(const TZ* __restrict__ Z, size_t hn,
                                                                const double* __restrict__ a, Geom g,
                                                                double* __restrict__ w, const double* __restrict__ U,
                                                                size_t stride, double* __restrict__ partials, int kc) {
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const bool act = m < H;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const size_t ty = (size_t)H, tz = (size_t)H * g.ny;
  const double hx = 0.5 * g.ihx2, hy = 0.5 * g.ihy2, hz = 0.5 * g.ihz2, pz = 2.0 * g.ihz2;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  const bool hw = m > 0, he = m < H - 1;
  const int lane = threadIdx.x;
  for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
    const bool hs = j > 0, hn_ = j < g.ny - 1;
    size_t cn = act ? 2 * sidx(g, m, j, k0) : 0;
    size_t q = act ? sidx(g, m, j, k0) : 0;
    double zb[2] = {0.0, 0.0}, zc[2] = {0.0, 0.0}, ab[2] = {0.0, 0.0}, ac[2] = {0.0, 0.0};
    if (act) {
      split_pair(Z, hn, q, (j + k0) & 1, zc[0], zc[1]);
      ac[0] = a[cn];
      ac[1] = a[cn + 1];
      if (k0 > 0) {
        split_pair(Z, hn, q - tz, (j + k0 - 1) & 1, zb[0], zb[1]);
        ab[0] = a[cn - sz];
        ab[1] = a[cn - sz + 1];
      }
    }
    for (int k = k0; k < k1; ++k) {
      const bool top = k == g.nz - 1;
      const int p = (j + k) & 1;
      double zt[2] = {0.0, 0.0}, at[2] = {0.0, 0.0};
      if (act && !top) {
        split_pair(Z, hn, q + tz, p ^ 1, zt[0], zt[1]);
        at[0] = a[cn + sz];
        at[1] = a[cn + sz + 1];
      }
      double zw = __shfl_up(zc[1], 1, 64), aw = __shfl_up(ac[1], 1, 64);
      double ze = __shfl_down(zc[0], 1, 64), ae = __shfl_down(ac[0], 1, 64);
      if (act && lane == 0 && hw) {
        zw = (double)Z[q - 1 + (size_t)(p ^ 1) * hn];
        aw = a[cn - 1];
      }
      if (act && lane == BX - 1 && he) {
        ze = (double)Z[q + 1 + (size_t)p * hn];
        ae = a[cn + 2];
      }
      if (act) {
        double zs[2] = {0.0, 0.0}, as_[2] = {0.0, 0.0}, zn[2] = {0.0, 0.0}, an[2] = {0.0, 0.0};
        if (hs) {
          split_pair(Z, hn, q - ty, p ^ 1, zs[0], zs[1]);
          as_[0] = a[cn - sy];
          as_[1] = a[cn - sy + 1];
        }
        if (hn_) {
          split_pair(Z, hn, q + ty, p ^ 1, zn[0], zn[1]);
          an[0] = a[cn + sy];
          an[1] = a[cn + sy + 1];
        }
        double wv[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const double acv = ac[e], zcv = zc[e];
          const double zo = e == 0 ? zw : ze, ao = e == 0 ? aw : ae;
          const bool ho = e == 0 ? hw : he;
          double s = (acv + ac[1 - e]) * hx * (zcv - zc[1 - e]);
          s += ho ? (acv + ao) * hx * (zcv - zo) : 0.0;
          s += hs ? (acv + as_[e]) * hy * (zcv - zs[e]) : 0.0;
          s += hn_ ? (acv + an[e]) * hy * (zcv - zn[e]) : 0.0;
          s += k > 0 ? (acv + ab[e]) * hz * (zcv - zb[e]) : pz * acv * zcv;
          s += !top ? (acv + at[e]) * hz * (zcv - zt[e]) : pz * acv * zcv;
          wv[e] = s;
        }
        w[cn] = wv[0];
        w[cn + 1] = wv[1];
#pragma unroll
        for (int v = 0; v < NV; ++v)
          acc[v] += wv[0] * U[(size_t)v * stride + cn] + wv[1] * U[(size_t)v * stride + cn + 1];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          zb[e] = zc[e];
          zc[e] = zt[e];
          ab[e] = ac[e];
          ac[e] = at[e];
        }
        cn += sz;
        q += tz;
      }
    }
  }
  block_store_partials<NV>(acc, NV, partials, gridDim.x * gridDim.y * gridDim.z);
}

// phi += sum_v y_v z_v with z_v colour-split (z promoted to float64).
template <typename TZ, int NV>
__global__ __launch_bounds__(NTHREADS) void k_update_split(double* __restrict__ phi, const TZ* __restrict__ Z,
                                                           size_t hn, size_t stride, Coeffs16 y, Geom g, int kc) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (m >= H || j >= g.ny) return;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int k = k0; k < k1; ++k) {
    const size_t q = sidx(g, m, j, k), cn = 2 * q;
    const int p = (j + k) & 1;
    double l = phi[cn], r = phi[cn + 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double zl, zr;
      split_pair(Z + (size_t)v * stride, hn, q, p, zl, zr);
      l += y.v[v] * zl;
      r += y.v[v] * zr;
    }
    phi[cn] = l;
    phi[cn + 1] = r;
  }
}

}  // namespace gmg
