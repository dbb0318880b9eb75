// gmg_sym.hpp -- the fused symmetric red-black sweep of the finest level
// (colour-split storage, cell coefficient): both half-sweeps of one
// symmetric Gauss-Seidel sweep in one pass over memory.
#pragma once

#include <type_traits>

#include "gmg_common.hpp"

namespace gmg {

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
// Block: 64 lanes x R rows (R = 16 in float32, 12 in float64); lane tx owns
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

// The parity of a plane in k_sym_split: computed where it is needed
// (RuntimeParity), or a compile-time constant.
struct RuntimeParity {};
__device__ __forceinline__ int parity_of(RuntimeParity, int v) { return v; }
template <int E>
__device__ __forceinline__ int parity_of(std::integral_constant<int, E>, int) {
  return E;
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
  // one row per wave: in float64 the row (and every parity below) is made
  // wave-uniform for the compiler
  const int lane = threadIdx.x;
  const int r = sizeof(T) == 8 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.y) : (int)threadIdx.y;
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

  // e1c: RuntimeParity or the compile-time value of (c1 + j + p) % 2
  auto load = [&](int p, SymCol<T>& L, auto e1c) {
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
      const int e1 = parity_of(e1c, (c1 + j + p) & 1);
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
    load(k0 - 2, Lb, RuntimeParity{});
    load(k0 - 1, Lc, RuntimeParity{});
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
  auto iterate = [&](int k, const SymCol<T>& L, auto e1c) {
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
    const int e1 = parity_of(e1c, (c1 + j + k) & 1);
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
    const int e2 = parity_of(e1c, (c2 + j + kk) & 1);  // = e1
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
  if constexpr (sizeof(T) == 8) {
    // the colour-c1 cell of plane k0 - 1 + 2 n + t sits at e1 = E0 ^ (t % 2)
    // with E0 uniform over the wave: the loop is instantiated for both E0 so
    // that every parity select is resolved at compile time (float64: 1.02 ->
    // 0.97 ms per sweep at 512^3; float32, whose arithmetic is cheaper, was
    // not faster so)
    static_assert(SYM_UNROLL % 2 == 0 && SYM_DEPTH == 2, "parity pattern of the unrolled loop");
    auto run = [&](auto E0c) {
      using P0 = std::integral_constant<int, decltype(E0c)::value>;
      using P1 = std::integral_constant<int, decltype(E0c)::value ^ 1>;
      load(k0, L[0], P1{});
      for (int k = k0 - 1; k <= k1; k += SYM_UNROLL) {
#pragma unroll
        for (int t = 0; t < SYM_UNROLL; t += 2) {
          // planes k + t + 2 and k + t + 3 have the parities of k and k + 1
          load(k + t + 2, L[1], P0{});
          if (k + t > k1) return;  // (an exit, not a break: no second path into the loop's back edge)
          iterate(k + t, L[0], P0{});
          load(k + t + 3, L[0], P1{});
          if (k + t + 1 > k1) return;
          iterate(k + t + 1, L[1], P1{});
        }
      }
    };
    if ((c1 + j + k0 - 1) & 1)
      run(std::integral_constant<int, 1>{});
    else
      run(std::integral_constant<int, 0>{});
  } else {
#pragma unroll
    for (int t = 0; t < SYM_DEPTH - 1; ++t) load(k0 + t, L[t], RuntimeParity{});
    for (int k = k0 - 1; k <= k1; k += SYM_UNROLL) {
#pragma unroll
      for (int t = 0; t < SYM_UNROLL; ++t) {
        load(k + t + SYM_DEPTH, L[(t + SYM_DEPTH - 1) % SYM_DEPTH], RuntimeParity{});
        if (k + t > k1) return;  // (an exit, not a break: no second path into the loop's back edge)
        iterate(k + t, L[t % SYM_DEPTH], RuntimeParity{});
      }
    }
  }
}

}  // namespace gmg
