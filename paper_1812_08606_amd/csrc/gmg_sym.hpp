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
// pair from the adjacent lane.  Each face joins one cell of either colour, so
// the c2 update computes no face weight: it takes the six weights its c1
// neighbours computed (kept in registers, passed through LDS with the c1
// values, or from the adjacent lane).  Planes k0-1 and k1 of the chunk are
// computed (c1 only) for the same reason and not stored.  FIRST: the first
// sweep from x = 0 (c1 = b / D; b from the natural-layout u times *bscale
// when SCALED, stored by colour into B).
//
// Each thread loads only its own column of every plane -- the coefficient
// pair, the old colour-c2 value and the two right sides -- and stages the
// coefficient pair and the old c2 value in LDS, where rows j-1 and j+1 read
// them (rows 0 and R-1 of the block also load and stage the row beyond the
// block): 4 loads per thread and plane, each cache line requested once per
// block.  (Loading the side rows from global memory as well, 14 loads per
// thread and plane with every line requested by three rows, took 0.66-0.70
// ms per sweep at 512^3 against 0.50 ms.)  LDS holds NS = 2 planes of side
// values: plane k+1 is staged at iteration k (after every wave has passed
// the barrier that ends iteration k-1's c1 update, the slot's last reader)
// and read at iteration k+1.
//
// RESID: the block also forms the residual b - A x of the result and its
// mean over each 2 x 2 x 2 cell group, the right side bc of level 1 (the
// values of k_resid_restrict_split to rounding, formed as it forms them:
// b minus the face fluxes w (x - x_nb) in the same order).  Iteration k
// takes plane k-2, whose values are final once c2 of plane k-1 is: the c2
// cell's residual is formed in its update (its equation was just solved
// with the final c1 neighbours: rounding only); the c1 cell's from the
// weights and right side its update used two planes earlier and the new c2
// values around it (own column from registers, rows j-1, j+1 from an LDS
// ring, the outer x-neighbour from the adjacent lane).  Pairs of planes
// add in registers, pairs of rows (waves r, r+1) through LDS.  A residual
// needs the final values one cell beyond it, so the block updates c1 and c2
// one lane, row and plane further and owns (SX - 4) x (R - 4) pairs.
//
// Block shape: SX = 64 lanes per row (one row per wave; 32-lane rows were
// measured slower) times R rows; the block owns (SX - 2) x (R - 2) pairs.
// Float64 takes 12 rows: 1024 threads would leave too few registers per
// thread (measured at 512^3: 1.16, 1.03 and 1.12 ms per sweep with 8, 12
// and 16 rows, the last spilling).  The residual variant runs in float32
// (126 registers at 1024 threads).
//
// DEPTH: planes whose loads are in flight (the loads of iteration k+1 are
// issued before iteration k runs); UNROLL: iterations per loop trip, a
// multiple of DEPTH, so the load buffers rotate whole periods per trip and
// no value still in flight is copied at the back edge (copying one makes the
// compiler wait for every load).
template <typename T, bool RESID = false>
struct SymShape {
  static constexpr int SX = 64;
  static constexpr int R = sizeof(T) == 4 ? 16 : 12;
  static constexpr int HALO = RESID ? 2 : 1;  // lanes and rows on each side the block does not own
  static constexpr int IX = SX - 2 * HALO;    // pairs per block row that the block owns
  static constexpr int IY = R - 2 * HALO;     // rows the block owns
  static constexpr int DEPTH = 2;
  static constexpr int UNROLL = 4;
  static_assert(UNROLL % DEPTH == 0, "the load buffers must rotate whole periods per trip");
  static_assert(IY % 2 == 0, "a block owns whole coarse rows");
};

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

// Raw buffer resource over `bytes` bytes from p (no stride, no swizzle).
// Loads and stores through it add a per-lane byte offset and a wave-uniform
// byte offset held in a scalar register, so a block marching the planes
// computes each plane's offset once in scalar arithmetic rather than a
// 64-bit address per lane and array.  Both offsets are 32-bit: the launch
// keeps a block's planes within 2^31 bytes of its base.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, size_t bytes) {
  const uint32_t n = bytes < 0xFFFFFFFFull ? (uint32_t)bytes : 0xFFFFFFFFu;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, (int)voff, (int)soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), rs,
                                          (int)voff, (int)soff, 0);
}
// The coefficient pair at byte offset voff + soff: one 8-byte load in float32;
// two loads in float64 (the caller's array is only 8-byte aligned).
template <typename T>
__device__ __forceinline__ typename Pair2<T>::type buf_load_pair(__amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                                                 uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
  } else {
    return double2{buf_load<double>(rs, voff, soff), buf_load<double>(rs, voff + 8, soff)};
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

template <typename T, bool FIRST, bool SCALED, bool RESID>
__global__ __launch_bounds__((SymShape<T, RESID>::SX * SymShape<T, RESID>::R)) void k_sym_split(
    const T* __restrict__ Xin, T* __restrict__ Xout, T* __restrict__ B, const double* __restrict__ u,
    const double* __restrict__ bscale, const T* __restrict__ a, Geom g, size_t hn, int kc, int c1,
    T* __restrict__ bc) {
  static_assert(!(FIRST && RESID), "the residual is fused into a sweep from a guess only");
  using T2 = typename Pair2<T>::type;
  using S = SymShape<T, RESID>;
  constexpr int SX = S::SX, IX = S::IX, R = S::R, IY = S::IY, HALO = S::HALO;
  constexpr int NS = 2;              // planes of side values held in LDS
  __shared__ T2 sa[NS][R + 2][SX];  // a pairs of block rows -1 .. R (array rows 0 .. R+1)
  __shared__ T so[NS][R + 2][SX];   // old values of colour c2, same rows
  __shared__ T ring[4][R][SX];      // new c1 values of planes k-3 .. k (mod 4)
  __shared__ T2 ringw[4][R][SX];    // their south and north face weights, same planes
  // RESID: new c2 values of planes k-2, k-1 (mod 2) and the odd rows' halves
  // of the restricted residual
  __shared__ T ring2[RESID ? 2 : 1][RESID ? R : 1][SX];
  __shared__ T part[RESID ? R : 1][SX];
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  // one row per wave: in float64 the row (and every parity below) is made
  // wave-uniform for the compiler
  const int lane = threadIdx.x;
  const int r = sizeof(T) == 8 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.y) : (int)threadIdx.y;
  const int m = tl.x * IX + lane - HALO;
  const int j = tl.y * IY + r - HALO;
  const bool ing = m >= 0 && m < H && j >= 0 && j < g.ny;
  const bool owner = ing && lane >= HALO && lane < SX - HALO && r >= HALO && r < R - HALO;
  // colour c2 is updated one lane and row inside the block's edge (where all
  // its c1 neighbours are), on the chunk's planes and, for the residual, on
  // the planes next to it
  const bool calc2 = ing && lane >= 1 && lane <= SX - 2 && r >= 1 && r <= R - 2;
  const int c2 = 1 - c1;
  const size_t tz = (size_t)H * g.ny;
  const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2), pz = (T)(2.0 * g.ihz2);
  const double s = SCALED ? *bscale : 1.0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  const int c2lo = RESID ? max(k0 - 1, 0) : k0, c2hi = RESID ? min(k1 + 1, g.nz) : k1;
  // iterations kstart .. kend update c1 on plane k, c2 on plane k-1 and (RESID)
  // take the residual of plane k-2
  const int kstart = k0 - HALO, kend = k1 + HALO - 1;
  // faces outside the pair: present when both cells lie in the grid (for
  // threads outside it, whose addresses are clamped to it, every such face
  // weight is zero)
  const bool hw = m > 0 && m < H, he = m >= 0 && m < H - 1, hs = j > 0 && j < g.ny, hn_ = j >= 0 && j < g.ny - 1;
  // clamped (always valid) column of this thread, and of the row beyond the
  // block that rows 0 and R-1 stage (array row 0 or R+1)
  const int mm = min(max(m, 0), H - 1), jj = min(max(j, 0), g.ny - 1);
  const size_t qcol = (size_t)jj * H + mm;
  const bool hrow = r == 0 || r == R - 1;
  const int jh = min(max(r == 0 ? j - 1 : j + 1, 0), g.ny - 1);
  const size_t qhcol = (size_t)jh * H + mm;
  const int arow = r == 0 ? 0 : R + 1;
  auto pl = [&](int k) { return min(max(k, 0), g.nz - 1); };
  // every array is addressed from plane kb, the lowest the block reads, with
  // per-lane byte offsets of the column (colour arrays: ST per pair; a and the
  // natural-layout u: two cells per pair) and a scalar offset per plane
  const int kb = pl(kstart - 1);
  const size_t pb = (size_t)kb * tz;  // first pair of plane kb
  constexpr uint32_t ST = sizeof(T);
  const size_t cbytes = (hn - pb) * ST, nbytes = 2 * (hn - pb) * ST;
  // (Xin is not read by the first sweep, u only by it)
  const auto rXo = buf_rsrc(FIRST ? nullptr : Xin + (size_t)c2 * hn + pb, FIRST ? 0 : cbytes);  // old colour c2
  const auto rY1 = buf_rsrc(Xout + (size_t)c1 * hn + pb, cbytes);
  const auto rY2 = buf_rsrc(Xout + (size_t)c2 * hn + pb, cbytes);
  const auto rB1 = buf_rsrc(B + (size_t)c1 * hn + pb, cbytes);
  const auto rB2 = buf_rsrc(B + (size_t)c2 * hn + pb, cbytes);
  const auto rA = buf_rsrc(a + 2 * pb, nbytes);
  const auto rU = buf_rsrc(FIRST ? u + 2 * pb : nullptr, FIRST ? 2 * (hn - pb) * sizeof(double) : 0);
  const uint32_t vq = (uint32_t)qcol * ST, vqh = (uint32_t)qhcol * ST;
  const uint32_t ptb = (uint32_t)tz * ST;  // bytes per plane of a colour array
  auto soff = [&](int k) { return (uint32_t)(k - kb) * ptb; };

  // e1c: RuntimeParity or the compile-time value of (c1 + j + p) % 2
  auto load = [&](int p, SymCol<T>& L, auto e1c) {
    const uint32_t so1 = soff(pl(p));
    const T2 av = buf_load_pair<T>(rA, 2 * vq, 2 * so1);
    L.a0 = av.x;
    L.a1 = av.y;
    if (!FIRST) {
      L.xo = buf_load<T>(rXo, vq, so1);
      L.b1 = buf_load<T>(rB1, vq, so1);
      L.b2 = buf_load<T>(rB2, vq, so1);
    } else {
      constexpr uint32_t W = sizeof(double) / ST;  // u bytes per colour-array byte, per cell pair
      const double u0d = buf_load<double>(rU, 2 * W * vq, 2 * W * so1);
      const double u1d = buf_load<double>(rU, 2 * W * vq + 8, 2 * W * so1);
      const T u0 = (T)(SCALED ? u0d * s : u0d), u1 = (T)(SCALED ? u1d * s : u1d);
      const int e1 = parity_of(e1c, (c1 + j + p) & 1);
      L.b1 = e1 ? u1 : u0;
      L.b2 = e1 ? u0 : u1;
      L.xo = T(0);
    }
    if (hrow) {
      const T2 hv = buf_load_pair<T>(rA, 2 * vqh, 2 * so1);
      L.ha0 = hv.x;
      L.ha1 = hv.y;
      L.hxo = FIRST ? T(0) : buf_load<T>(rXo, vqh, so1);
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

  // registers: a of the pair on planes k-1 .. k+1, old c2 of the column on
  // k-1 .. k+1, new c1 of the column on k-3 .. k; right sides: c1 and c2 of
  // plane k (cb1, cb2), c2 of plane k-1 (pb2); face weights of the column's
  // c1 cell: inner and outer x-faces on plane k-1 (wip, wop), top faces on
  // planes k-1 and k-2 (wtp, wtpp).  RESID: new c2 of the column on k-3 ..
  // k-1 (c2h), and of the c1 cell on planes k-2 .. k its right side, plate
  // coefficient (2 a / hz^2) and inner, outer x-, bottom and top face weights
  // (index 0: plane k-2)
  T a0[3], a1[3], xo[3], c1n[4], cb1, cb2, pb2 = T(0);
  T wip = T(0), wop = T(0), wtp = T(0), wtpp = T(0);
  T c2h[3], hb1[3], hdz[3], hwi[3], hwo[3], hwb[3], hwt[3];
  T r2p = T(0), accz = T(0);  // RESID: residual of the c2 cell on plane k-2; coarse-plane sum
#pragma unroll
  for (int t = 0; t < 3; ++t) c2h[t] = hb1[t] = hdz[t] = hwi[t] = hwo[t] = hwb[t] = hwt[t] = T(0);
#pragma unroll
  for (int t = 0; t < 4; ++t) c1n[t] = T(0);
  a0[0] = a1[0] = T(0);
  xo[0] = T(0);
  {
    // plane kstart-1 (own column only) and plane kstart (staged), rotated
    // into place at the top of the first iteration
    SymCol<T> Lb, Lc;
    load(kstart - 1, Lb, RuntimeParity{});
    load(kstart, Lc, RuntimeParity{});
    a0[1] = Lb.a0;
    a1[1] = Lb.a1;
    xo[1] = Lb.xo;
    a0[2] = Lc.a0;
    a1[2] = Lc.a1;
    xo[2] = Lc.xo;
    cb1 = Lc.b1;
    cb2 = Lc.b2;
    stage(kstart, Lc);
  }
  lds_barrier();

  // iteration k: stage plane k+1, colour c1 on plane k, colour c2 on plane k-1.
  // Every face joins a c1 and a c2 cell, so the c2 update takes all six face
  // weights from the c1 updates: inner and outer x-faces from its pair's and
  // the adjacent lane's c1 cell on plane k-1, the y-faces from rows j-1 and
  // j+1 on plane k-1 (LDS), the z-faces from the column's c1 cells on planes
  // k-2 and k.
  auto iterate = [&](int k, const SymCol<T>& L, auto e1c) {
    a0[0] = a0[1];
    a1[0] = a1[1];
    a0[1] = a0[2];
    a1[1] = a1[2];
    a0[2] = L.a0;
    a1[2] = L.a1;
    xo[0] = xo[1];
    xo[1] = xo[2];
    xo[2] = L.xo;
    stage(k + 1, L);
    // (a0[2] is plane k+1, a0[1] plane k, a0[0] plane k-1; xo[2] plane k+1,
    // xo[1] plane k, xo[0] plane k-1)
    const int e1 = parity_of(e1c, (c1 + j + k) & 1);
    const bool hout = e1 ? he : hw;
    // a and old c2 of the cell outside the pair: element 0 of pair m+1
    // (e1 = 1) or element 1 of pair m-1 (e1 = 0), from the adjacent lane
    const int src = lane + (e1 ? 1 : -1);
    const T aout = __shfl(e1 ? a0[1] : a1[1], src, SX);
    const T xout = __shfl(xo[1], src, SX);
    T v1, wi, wo, wb, wt, D1, dz1;
    {
      const int sl = k & (NS - 1);
      const T2 ps = sa[sl][r][lane], pn = sa[sl][r + 2][lane];
      const bool top = k >= g.nz - 1, bot = k <= 0;
      const T acv = e1 ? a1[1] : a0[1], ain = e1 ? a0[1] : a1[1];
      const T abv = e1 ? a1[0] : a0[0], atv = e1 ? a1[2] : a0[2];
      wi = (acv + ain) * hx;
      wo = hout ? (acv + aout) * hx : T(0);
      const T ws = hs ? (acv + (e1 ? ps.y : ps.x)) * hy : T(0);
      const T wn = hn_ ? (acv + (e1 ? pn.y : pn.x)) * hy : T(0);
      wb = (acv + abv) * hz;
      wt = (acv + atv) * hz;
      dz1 = pz * acv;
      D1 = wi + wo + ws + wn + (!bot ? wb : dz1) + (!top ? wt : dz1);
      if (FIRST) {
        v1 = cb1 * recip(D1);
      } else {
        // (absent faces have zero weight and finite neighbour values)
        const T xs = so[sl][r][lane], xn = so[sl][r + 2][lane];
        const T off = wi * xo[1] + wo * xout + ws * xs + wn * xn + (!bot ? wb * xo[0] : T(0)) +
                      (!top ? wt * xo[2] : T(0));
        v1 = (cb1 + off) * recip(D1);
      }
      if (owner && k >= k0 && k < k1) {
        const uint32_t so1 = soff(k);
        buf_store<T>(v1, rY1, vq, so1);
        if (FIRST) {
          buf_store<T>(cb1, rB1, vq, so1);
          buf_store<T>(cb2, rB2, vq, so1);
        }
      }
      ringw[k & 3][r][lane] = T2{ws, wn};
    }
    c1n[0] = c1n[1];
    c1n[1] = c1n[2];
    c1n[2] = c1n[3];
    c1n[3] = v1;
    ring[k & 3][r][lane] = v1;
    lds_barrier();
    // --- colour c2 on plane kk = k-1 (element e1 of the pair) ---
    const int kk = k - 1;
    // the adjacent lane's new c1 value and outer x-face on plane kk
    const int src2 = lane + (e1 ? 1 : -1);
    const T cov = __shfl(c1n[2], src2, SX);
    const T wov = __shfl(wop, src2, SX);
    T v2 = T(0), r2 = T(0);
    if (calc2 && kk >= c2lo && kk < c2hi) {
      const bool top = kk == g.nz - 1, bot = kk == 0;
      const int rl = kk & 3;
      const T ys = ring[rl][r - 1][lane], yn = ring[rl][r + 1][lane];
      const T wsv = ringw[rl][r - 1][lane].y, wnv = ringw[rl][r + 1][lane].x;
      const T acv = e1 ? a1[0] : a0[0];
      const T D = wip + wov + wsv + wnv + (!bot ? wtpp : pz * acv) + (!top ? wb : pz * acv);
      const T off = wip * c1n[2] + wov * cov + wsv * ys + wnv * yn + (!bot ? wtpp * c1n[1] : T(0)) +
                    (!top ? wb * c1n[3] : T(0));
      v2 = (pb2 + off) * recip(D);
      if (owner && kk >= k0 && kk < k1) buf_store<T>(v2, rY2, vq, soff(kk));
      if (RESID) {
        // its residual b - A x, the fluxes summed face by face as
        // k_resid_restrict_split does (the update solved this equation with
        // these neighbours: only rounding is left)
        T Ax = wip * (v2 - c1n[2]);
        Ax += wov * (v2 - cov);
        Ax += wsv * (v2 - ys);
        Ax += wnv * (v2 - yn);
        Ax += !bot ? wtpp * (v2 - c1n[1]) : pz * acv * v2;
        Ax += !top ? wb * (v2 - c1n[3]) : pz * acv * v2;
        r2 = pb2 - Ax;
      }
    }
    if constexpr (RESID) {
      c2h[0] = c2h[1];
      c2h[1] = c2h[2];
      c2h[2] = v2;
      ring2[kk & 1][r][lane] = v2;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        hb1[t] = hb1[t + 1];
        hdz[t] = hdz[t + 1];
        hwi[t] = hwi[t + 1];
        hwo[t] = hwo[t + 1];
        hwb[t] = hwb[t + 1];
        hwt[t] = hwt[t + 1];
      }
      hb1[2] = cb1;
      hdz[2] = dz1;
      hwi[2] = wi;
      hwo[2] = wo;
      hwb[2] = wb;
      hwt[2] = wt;
      // --- residual of plane p = k-2, where every value is final: the c1
      // cell from its kept weights and the new c2 values around it (the own
      // pair and planes p-1, p+1 from registers, the outer x-neighbour from
      // the adjacent lane, rows j-1 and j+1 from LDS, written before this
      // iteration's barrier); summed over the pair and the plane pair of a
      // coarse cell, then over the row pair through LDS ---
      const int p = k - 2;
      const int srcr = lane + (e1 ? 1 : -1);  // the c1 cell of plane p is element e1 of the pair, as on plane k
      const T x2out = __shfl(c2h[1], srcr, SX);
      if (p >= k0 && p < k1) {
        T rsum = T(0);
        if (owner) {
          const bool top = p == g.nz - 1, bot = p == 0;
          const int rl = p & 1;
          const T ys = ring2[rl][r - 1][lane], yn = ring2[rl][r + 1][lane];
          const T2 wsn = ringw[p & 3][r][lane];
          const T x1 = c1n[1];
          T Ax = hwi[0] * (x1 - c2h[1]);
          Ax += hwo[0] * (x1 - x2out);
          Ax += wsn.x * (x1 - ys);
          Ax += wsn.y * (x1 - yn);
          Ax += !bot ? hwb[0] * (x1 - c2h[0]) : hdz[0] * x1;
          Ax += !top ? hwt[0] * (x1 - c2h[2]) : hdz[0] * x1;
          rsum = (hb1[0] - Ax) + r2p;
        }
        if (!(p & 1)) {
          accz = rsum;
        } else {
          accz += rsum;
          if (r & 1) part[r][lane] = accz;
          lds_barrier();
          if (owner && !(r & 1)) {
            const int NY = g.ny >> 1;
            bc[((size_t)(p >> 1) * NY + (j >> 1)) * H + m] = (accz + part[r + 1][lane]) * T(0.125);
          }
        }
      }
      r2p = r2;
    }
    wtpp = wtp;
    wtp = wt;
    wip = wi;
    wop = wo;
    pb2 = cb2;
    cb1 = L.b1;
    cb2 = L.b2;
  };

  // DEPTH load buffers: iteration k consumes plane k+1, whose loads were
  // issued DEPTH - 1 iterations earlier into the buffer the iteration before
  // them released; loads past the grid read a clamped valid plane
  constexpr int DEPTH = S::DEPTH, UNROLL = S::UNROLL;
  SymCol<T> L[DEPTH];
  if constexpr (sizeof(T) == 8) {
    // the colour-c1 cell of plane kstart + 2 n + t sits at e1 = E0 ^ (t % 2)
    // with E0 uniform over the wave: the loop is instantiated for both E0 so
    // that every parity select is resolved at compile time (float64: 1.02 ->
    // 0.97 ms per sweep at 512^3; float32, whose arithmetic is cheaper, was
    // not faster so)
    static_assert(UNROLL % 2 == 0 && DEPTH == 2, "parity pattern of the unrolled loop");
    auto run = [&](auto E0c) {
      using P0 = std::integral_constant<int, decltype(E0c)::value>;
      using P1 = std::integral_constant<int, decltype(E0c)::value ^ 1>;
      load(kstart + 1, L[0], P1{});
      for (int k = kstart; k <= kend; k += UNROLL) {
#pragma unroll
        for (int t = 0; t < UNROLL; t += 2) {
          // planes k + t + 2 and k + t + 3 have the parities of k and k + 1
          load(k + t + 2, L[1], P0{});
          if (k + t > kend) return;  // (an exit, not a break: no second path into the loop's back edge)
          iterate(k + t, L[0], P0{});
          load(k + t + 3, L[0], P1{});
          if (k + t + 1 > kend) return;
          iterate(k + t + 1, L[1], P1{});
        }
      }
    };
    if ((c1 + j + kstart) & 1)
      run(std::integral_constant<int, 1>{});
    else
      run(std::integral_constant<int, 0>{});
  } else {
#pragma unroll
    for (int t = 0; t < DEPTH - 1; ++t) load(kstart + 1 + t, L[t], RuntimeParity{});
    for (int k = kstart; k <= kend; k += UNROLL) {
#pragma unroll
      for (int t = 0; t < UNROLL; ++t) {
        load(k + t + DEPTH, L[(t + DEPTH - 1) % DEPTH], RuntimeParity{});
        if (k + t > kend) return;  // (an exit, not a break: no second path into the loop's back edge)
        iterate(k + t, L[t % DEPTH], RuntimeParity{});
      }
    }
  }
}

}  // namespace gmg
