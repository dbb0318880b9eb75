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
#include "gmg_sym.hpp"

namespace gmg {

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
// instead of x += P xc.  xin (natural layout only; null otherwise): x = xin
// + P xc, xin another buffer.
template <typename T, bool SPLIT, bool SET = false>
__global__ __launch_bounds__(NTHREADS) void k_prolong_pair(T* __restrict__ x, const T* __restrict__ xc, Geom g,
                                                           size_t hn, int cmask, int kc,
                                                           const T* __restrict__ xin) {
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
        if (SET) {
          x[cn] = vl;
          x[cn + 1] = vr;
        } else if (xin) {
          x[cn] = xin[cn] + vl;
          x[cn + 1] = xin[cn + 1] + vr;
        } else {
          x[cn] = x[cn] + vl;
          x[cn + 1] = x[cn + 1] + vr;
        }
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
        // w and the basis vectors stream through once (non-temporal), so
        // that L2 keeps the z and a rows that the adjacent rows' blocks re-read
        __builtin_nontemporal_store(wv[0], &w[cn]);
        __builtin_nontemporal_store(wv[1], &w[cn + 1]);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          acc[v] += wv[0] * __builtin_nontemporal_load(&U[(size_t)v * stride + cn]) +
                    wv[1] * __builtin_nontemporal_load(&U[(size_t)v * stride + cn + 1]);
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

// phi += sum_v y_v z_v with z_v colour-split (z promoted to float64); set:
// phi = 0 + sum_v y_v z_v, without reading phi (the first update of a solve
// from a zero guess).
template <typename TZ, int NV>
__global__ __launch_bounds__(NTHREADS) void k_update_split(double* __restrict__ phi, const TZ* __restrict__ Z,
                                                           size_t hn, size_t stride, Coeffs16 y, Geom g, int kc,
                                                           int set) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (m >= H || j >= g.ny) return;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int k = k0; k < k1; ++k) {
    const size_t q = sidx(g, m, j, k), cn = 2 * q;
    const int p = (j + k) & 1;
    double l = 0.0, r = 0.0;
    if (!set) {
      l = phi[cn];
      r = phi[cn + 1];
    }
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
