// gmg_kernels.hpp -- gfx950 kernels of the GMG-preconditioned FGMRES solve.
//
// Grid layout: (nz, ny, nx), x fastest.  Every stencil kernel maps a block
// of 64 x 4 threads onto 64 consecutive x-cells of 4 rows and marches each
// thread along z over a chunk of planes; loads along x are coalesced and the
// rows above/below come from the same or neighbouring blocks through L2.
//
// Discrete operator (eq. e18, Sec. 2.2): (A x)_c = sum_f w_f (x_c - x_nb)/h^2.
// On the finest level w_f is the arithmetic mean of the two cells' a; on a
// plate the face coefficient is a_c and the neighbour is the mirrored ghost
// 2 phi_b - x_c; the Neumann sides carry w = 0.  Coarse levels store their
// face coefficients: wx[c] is the face on the -x side of cell c (0 at i = 0),
// wy[c] the -y side (0 at j = 0), wz[c] the -z side (the bottom plate's
// coefficient at k = 0), and tp[j*nx+i] the top plate's coefficient.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmg_common.hpp"

namespace gmg {

struct Coeffs16 {
  double v[MAXV];
};

__device__ __forceinline__ size_t cidx(const Geom& g, int i, int j, int k) {
  return ((size_t)k * g.ny + j) * g.nx + i;
}

// Face weights of one cell, already divided by h_d^2.
template <typename T>
struct Stencil {
  T ww, we, ws, wn, wb, wt;
};

// Finest level: coefficient per cell, face = arithmetic mean.
template <typename T>
struct CellCoef {
  const T* __restrict__ a;
  __device__ __forceinline__ Stencil<T> load(const Geom& g, int i, int j, int k, size_t c) const {
    const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
    const T ac = a[c];
    const T hx = (T)(0.5 * g.ihx2), hy = (T)(0.5 * g.ihy2), hz = (T)(0.5 * g.ihz2);
    Stencil<T> s;
    s.ww = i > 0 ? (ac + a[c - 1]) * hx : T(0);
    s.we = i < g.nx - 1 ? (ac + a[c + 1]) * hx : T(0);
    s.ws = j > 0 ? (ac + a[c - sy]) * hy : T(0);
    s.wn = j < g.ny - 1 ? (ac + a[c + sy]) * hy : T(0);
    s.wb = k > 0 ? (ac + a[c - sz]) * hz : ac * (T)g.ihz2;
    s.wt = k < g.nz - 1 ? (ac + a[c + sz]) * hz : ac * (T)g.ihz2;
    return s;
  }
};

// Coarse levels: stored face coefficients.
template <typename T>
struct FaceCoef {
  const T* __restrict__ wx;
  const T* __restrict__ wy;
  const T* __restrict__ wz;
  const T* __restrict__ tp;
  __device__ __forceinline__ Stencil<T> load(const Geom& g, int i, int j, int k, size_t c) const {
    const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
    const T ix = (T)g.ihx2, iy = (T)g.ihy2, iz = (T)g.ihz2;
    Stencil<T> s;
    s.ww = wx[c] * ix;
    s.we = i < g.nx - 1 ? wx[c + 1] * ix : T(0);
    s.ws = wy[c] * iy;
    s.wn = j < g.ny - 1 ? wy[c + sy] * iy : T(0);
    s.wb = wz[c] * iz;
    s.wt = k < g.nz - 1 ? wz[c + sz] * iz : tp[(size_t)j * g.nx + i] * iz;
    return s;
  }
};

// Values of x at the 6 neighbours (x_c where the face has weight 0; the
// mirrored ghost 2 pb - x_c / 2 pt - x_c through the plates).
template <typename T>
struct Nbrs {
  T c, w, e, s, n, b, t;
};

template <typename T, typename TX>
__device__ __forceinline__ Nbrs<T> load_nbrs(const TX* __restrict__ x, const Geom& g, int i, int j,
                                             int k, size_t c, T pb2, T pt2) {
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  Nbrs<T> v;
  v.c = (T)x[c];
  v.w = i > 0 ? (T)x[c - 1] : v.c;
  v.e = i < g.nx - 1 ? (T)x[c + 1] : v.c;
  v.s = j > 0 ? (T)x[c - sy] : v.c;
  v.n = j < g.ny - 1 ? (T)x[c + sy] : v.c;
  v.b = k > 0 ? (T)x[c - sz] : pb2 - v.c;
  v.t = k < g.nz - 1 ? (T)x[c + sz] : pt2 - v.c;
  return v;
}

template <typename T>
__device__ __forceinline__ T apply_cell(const Stencil<T>& s, const Nbrs<T>& v) {
  return s.ww * (v.c - v.w) + s.we * (v.c - v.e) + s.ws * (v.c - v.s) + s.wn * (v.c - v.n) +
         s.wb * (v.c - v.b) + s.wt * (v.c - v.t);
}

// Diagonal of A (a plate face counts twice through its mirrored ghost).
template <typename T>
__device__ __forceinline__ T diag_cell(const Stencil<T>& s, const Geom& g, int k) {
  return s.ww + s.we + s.ws + s.wn + (k > 0 ? s.wb : T(2) * s.wb) + (k < g.nz - 1 ? s.wt : T(2) * s.wt);
}

// ---------------------------------------------------------------------------
// Deterministic block reductions: 64-lane wavefront shuffles, then the 4
// wave sums in a fixed order; one partial per block and vector.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_store_partials(double (&acc)[NV], int nv, double* __restrict__ partials,
                                                     int nblocks) {
  __shared__ double sm[NV][NWAVES];
  const int tid = threadIdx.y * BX + threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < nv) {
      const double s = wave_sum(acc[v]);
      if (lane == 0) sm[v][wave] = s;
    }
  }
  __syncthreads();
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  if (tid < nv) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) s += sm[tid][w];
    partials[(size_t)tid * nblocks + bid] = s;
  }
}

// ---------------------------------------------------------------------------
// V-cycle kernels (T = float for the mixed-precision preconditioner, double
// otherwise).
// ---------------------------------------------------------------------------

// First pre-smoothing half-sweep from x = 0: red cells x = b / D, black cells
// x = 0 (a red Gauss-Seidel step on a zero guess); with red == 0 (no
// pre-smoothing) x = 0 everywhere.  b is read as b_in * (*bscale) (the lazily
// normalised Krylov vector on the finest level) and, when b_out is given,
// stored there in T (the float32 copy of v_j).
template <typename T, typename TIn, typename Coef>
__global__ __launch_bounds__(NTHREADS) void k_gs_first(T* __restrict__ x, const TIn* __restrict__ b_in,
                                                       const double* __restrict__ bscale,
                                                       T* __restrict__ b_out, Coef co, Geom g, int kc,
                                                       int red) {
  const Tile tl = xcd_tile();
  const int i = tl.x * BX + threadIdx.x;
  if (i >= g.nx) return;
  const double s = bscale ? *bscale : 1.0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
    for (int k = k0; k < k1; ++k) {
      const size_t c = cidx(g, i, j, k);
      const T bv = (T)((double)b_in[c] * s);
      if (b_out) b_out[c] = bv;
      if (((i + j + k) & 1) || !red) {
        x[c] = T(0);
      } else {
        const Stencil<T> st = co.load(g, i, j, k, c);
        x[c] = bv / diag_cell(st, g, k);
      }
    }
  }
}

// Red-black half-sweep of one colour on a coarse level (stored face
// coefficients; even nx).  Lane tx owns the x-pair (2m, 2m+1) of row j; on
// every plane exactly one cell of the pair has the colour being updated.
// The thread marches its z-chunk keeping x and the bottom faces of the pair
// in registers; the loads of two planes are issued in one branch-free group
// with clamped addresses (values behind a missing face get zero weight).
// Only cells of the other colour are read and none of them is written, so
// the update is order-free.  FIRST: the first pre-smoothing half-sweep from
// x = 0 (cells of the colour get b / D, the others 0; x is not read).
template <typename T>
struct FaceSide {
  T xt0, xt1;        // x of the pair on plane k+1
  T wt0, wt1;        // top faces of the pair (wz on plane k+1, or the top plate's)
  T wx0, wx1, wxe;   // x-faces: west of cell 2m, between, east of cell 2m+1
  T xw, xe;          // x of cells 2m-1 and 2m+2
  T ws, wn, xs, xn;  // y-faces and y-neighbours of the updated cell
  T b;               // right side of the updated cell
};

template <typename T, bool FIRST>
__device__ __forceinline__ void face_side_load(FaceSide<T>& S, const T* __restrict__ x, const T* __restrict__ b,
                                               const FaceCoef<T>& co, const Geom& g, int i0, int j, int k,
                                               int colour, bool act) {
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const int kk = act ? k : 0, jj = act ? j : 0, ii = act ? i0 : 0;
  const size_t c = ((size_t)kk * g.ny + jj) * g.nx + ii;
  const int e = (colour + ii + jj + kk) & 1;
  const size_t ce = c + e;
  const bool up = kk + 1 < g.nz;
  const T* wtp = up ? co.wz + c + sz : co.tp + (size_t)jj * g.nx + ii;
  S.wt0 = wtp[0];
  S.wt1 = wtp[1];
  S.wx0 = co.wx[c];
  S.wx1 = co.wx[c + 1];
  S.wxe = co.wx[ii + 2 < g.nx ? c + 2 : c + 1];
  S.ws = co.wy[ce];
  S.wn = co.wy[jj < g.ny - 1 ? ce + sy : ce];
  S.b = b[ce];
  if (!FIRST) {
    const size_t ct = up ? c + sz : c;
    S.xt0 = x[ct];
    S.xt1 = x[ct + 1];
    S.xw = x[ii > 0 ? c - 1 : c];
    S.xe = x[ii + 2 < g.nx ? c + 2 : c];
    S.xs = x[jj > 0 ? ce - sy : ce];
    S.xn = x[jj < g.ny - 1 ? ce + sy : ce];
  } else {
    S.xt0 = S.xt1 = S.xw = S.xe = S.xs = S.xn = T(0);
  }
}

template <typename T, bool FIRST>
__global__ __launch_bounds__(NTHREADS) void k_gs_pair_face(T* __restrict__ x, const T* __restrict__ b,
                                                           FaceCoef<T> co, Geom g, int kc, int colour) {
  const Tile tl = xcd_tile();
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  const int i0 = 2 * m;
  const bool act = i0 < g.nx && j < g.ny;
  const size_t sz = (size_t)g.nx * g.ny;
  const T ix = (T)g.ihx2, iy = (T)g.ihy2, iz = (T)g.ihz2;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  const bool hs = j > 0, hn = j < g.ny - 1;
  const bool hwo = i0 > 0, heo = i0 + 2 < g.nx;
  // x of the pair on planes k-1, k and the pair's bottom faces on plane k
  T xb0 = T(0), xb1 = T(0), xc0 = T(0), xc1 = T(0), wb0, wb1;
  {
    const size_t c = act ? ((size_t)k0 * g.ny + j) * g.nx + i0 : 0;
    const size_t cb = (act && k0 > 0) ? c - sz : c;
    wb0 = co.wz[c];
    wb1 = co.wz[c + 1];
    if (!FIRST) {
      xc0 = x[c];
      xc1 = x[c + 1];
      xb0 = x[cb];
      xb1 = x[cb + 1];
    }
  }
  auto plane = [&](int k, const FaceSide<T>& S) {
    const bool top = k == g.nz - 1;
    const int e = (colour + i0 + j + k) & 1;
    const T ww = e ? S.wx1 : (hwo ? S.wx0 : T(0)), we = e ? (heo ? S.wxe : T(0)) : S.wx1;
    const T ws = hs ? S.ws : T(0), wn = hn ? S.wn : T(0);
    const T wb = e ? wb1 : wb0, wt = e ? S.wt1 : S.wt0;
    const T D = (ww + we) * ix + (ws + wn) * iy + (k > 0 ? wb : T(2) * wb) * iz + (top ? T(2) * wt : wt) * iz;
    if (act) {
      const size_t c = ((size_t)k * g.ny + j) * g.nx + i0;
      if (FIRST) {
        x[c + e] = S.b * recip(D);
        x[c + 1 - e] = T(0);
      } else {
        const T xw = e ? xc0 : S.xw, xe = e ? S.xe : xc1;
        const T xbv = e ? xb1 : xb0, xtv = e ? S.xt1 : S.xt0;
        T off = (ww * xw + we * xe) * ix + (ws * S.xs + wn * S.xn) * iy;
        off += k > 0 ? wb * iz * xbv : T(0);
        off += !top ? wt * iz * xtv : T(0);
        x[c + e] = (S.b + off) * recip(D);
      }
    }
    xb0 = xc0;
    xb1 = xc1;
    xc0 = S.xt0;
    xc1 = S.xt1;
    wb0 = S.wt0;
    wb1 = S.wt1;
  };
  for (int k = k0; k < k1; k += 2) {
    FaceSide<T> S0, S1;
    face_side_load<T, FIRST>(S0, x, b, co, g, i0, j, k, colour, act);
    face_side_load<T, FIRST>(S1, x, b, co, g, i0, j, min(k + 1, k1 - 1), colour, act);
    plane(k, S0);
    if (k + 1 < k1) plane(k + 1, S1);
  }
}

// Residual and restriction on a coarse level (stored face coefficients):
// b_coarse = mean over the 8 children of (b - A x).  Lane tx owns the fine
// x-pair (2I, 2I+1) of fine row j = 4 by + ty and marches the fine planes of
// its z-chunk, 2 per coarse plane, their loads issued in one branch-free
// group with clamped addresses; the two fine rows of a coarse row are summed
// through LDS.  Needs even nx, ny, nz; kc counts coarse planes.
template <typename T>
struct FaceResidSide {
  T xt0, xt1, wt0, wt1;      // x of the pair on plane k+1; top faces of the pair
  T wx0, wx1, wxe, xw, xe;   // x-faces west / between / east; x of cells 2I-1, 2I+2
  T ws0, ws1, xs0, xs1;      // south faces and neighbours of both cells
  T wn0, wn1, xn0, xn1;      // north faces and neighbours of both cells
  T b0, b1;
};

template <typename T>
__device__ __forceinline__ void face_resid_load(FaceResidSide<T>& S, const T* __restrict__ x,
                                                const T* __restrict__ b, const FaceCoef<T>& co, const Geom& g,
                                                int i0, int j, int k, bool act) {
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const int kk = act ? k : 0, jj = act ? j : 0, ii = act ? i0 : 0;
  const size_t c = ((size_t)kk * g.ny + jj) * g.nx + ii;
  const bool up = kk + 1 < g.nz;
  const size_t ct = up ? c + sz : c;
  const T* wtp = up ? co.wz + c + sz : co.tp + (size_t)jj * g.nx + ii;
  const size_t cs = jj > 0 ? c - sy : c, cn = jj < g.ny - 1 ? c + sy : c;
  S.xt0 = x[ct];
  S.xt1 = x[ct + 1];
  S.wt0 = wtp[0];
  S.wt1 = wtp[1];
  S.wx0 = co.wx[c];
  S.wx1 = co.wx[c + 1];
  S.wxe = co.wx[ii + 2 < g.nx ? c + 2 : c + 1];
  S.xw = x[ii > 0 ? c - 1 : c];
  S.xe = x[ii + 2 < g.nx ? c + 2 : c];
  S.ws0 = co.wy[c];
  S.ws1 = co.wy[c + 1];
  S.xs0 = x[cs];
  S.xs1 = x[cs + 1];
  S.wn0 = co.wy[cn];
  S.wn1 = co.wy[cn + 1];
  S.xn0 = x[cn];
  S.xn1 = x[cn + 1];
  S.b0 = b[c];
  S.b1 = b[c + 1];
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_resid_restrict_face(const T* __restrict__ x, const T* __restrict__ b,
                                                                  FaceCoef<T> co, Geom g, T* __restrict__ bc,
                                                                  int kc) {
  __shared__ T part[BY][BX];
  const Tile tl = xcd_tile();
  const int NX = g.nx >> 1, NY = g.ny >> 1, NZ = g.nz >> 1;
  const int I = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  const bool act = I < NX && j < g.ny;
  const int i0 = 2 * I;
  const size_t sz = (size_t)g.nx * g.ny;
  const T ix = (T)g.ihx2, iy = (T)g.ihy2, iz = (T)g.ihz2;
  const int K0 = tl.z * kc, K1 = min(NZ, K0 + kc);
  const bool hw = i0 > 0, he = i0 + 2 < g.nx, hs = j > 0, hn = j < g.ny - 1;
  T xb[2], xc[2], wb[2];
  {
    const int k0 = 2 * K0;
    const size_t c = act ? ((size_t)k0 * g.ny + j) * g.nx + i0 : 0;
    const size_t cb = (act && k0 > 0) ? c - sz : c;
    xc[0] = x[c];
    xc[1] = x[c + 1];
    xb[0] = x[cb];
    xb[1] = x[cb + 1];
    wb[0] = co.wz[c];
    wb[1] = co.wz[c + 1];
  }
  auto plane = [&](int k, const FaceResidSide<T>& S) -> T {
    const bool top = k == g.nz - 1;
    const T xt[2] = {S.xt0, S.xt1}, wt[2] = {S.wt0, S.wt1};
    const T wsv[2] = {S.ws0, S.ws1}, xs[2] = {S.xs0, S.xs1};
    const T wnv[2] = {S.wn0, S.wn1}, xn[2] = {S.xn0, S.xn1};
    const T bv[2] = {S.b0, S.b1};
    T rsum = T(0);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const T xcv = xc[e];
      T Ax = e == 0 ? (hw ? S.wx0 * ix * (xcv - S.xw) : T(0)) + S.wx1 * ix * (xcv - xc[1])
                    : S.wx1 * ix * (xcv - xc[0]) + (he ? S.wxe * ix * (xcv - S.xe) : T(0));
      Ax += hs ? wsv[e] * iy * (xcv - xs[e]) : T(0);
      Ax += hn ? wnv[e] * iy * (xcv - xn[e]) : T(0);
      Ax += k > 0 ? wb[e] * iz * (xcv - xb[e]) : T(2) * wb[e] * iz * xcv;
      Ax += !top ? wt[e] * iz * (xcv - xt[e]) : T(2) * wt[e] * iz * xcv;
      rsum += bv[e] - Ax;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      xb[e] = xc[e];
      xc[e] = xt[e];
      wb[e] = wt[e];
    }
    return rsum;
  };
  for (int K = K0; K < K1; ++K) {
    FaceResidSide<T> S0, S1;
    face_resid_load(S0, x, b, co, g, i0, j, 2 * K, act);
    face_resid_load(S1, x, b, co, g, i0, j, 2 * K + 1, act);
    T acc = plane(2 * K, S0);
    acc += plane(2 * K + 1, S1);
    part[threadIdx.y][threadIdx.x] = acc;
    __syncthreads();
    if (!(threadIdx.y & 1) && act) {
      const T tot = acc + part[threadIdx.y + 1][threadIdx.x];
      bc[((size_t)K * NY + (j >> 1)) * NX + I] = tot * T(0.125);
    }
    __syncthreads();
  }
}

// The bottom of the V-cycle in one workgroup: every level from lb down to
// the coarsest (all small) -- smoothing, residual and restriction, the
// direct coarsest solve, prolongation and post-smoothing -- with block
// barriers between the phases instead of kernel launches.  The iterates and
// right sides of these levels live in LDS; the right side of level lb is
// read from b0 and its iterate written to x0 at the end.  The arguments sit
// in device memory (written once at set-up) so that the per-level fields
// are read with scalar loads.
constexpr int BOTTOM_MAX_LEVELS = 10;
// threads of the bottom workgroup: 1024 in float32; 512 in float64, where
// 1024 threads would leave too few registers per thread
template <typename T>
struct BottomThreads {
  static constexpr int value = sizeof(T) == 4 ? 1024 : 512;
};
constexpr int BOTTOM_LDS_CELLS = 4704;  // >= 4096 * (1 + 1/8 + 1/64 + ...)

template <typename T>
struct BottomArgs {
  FaceCoef<T> co[BOTTOM_MAX_LEVELS];
  Geom g[BOTTOM_MAX_LEVELS];
  T* x0;
  const T* b0;
  const T* Ainv;
  int nlev;  // levels handled, the last one the coarsest
  int nu_pre, nu_post;
  int coff[BOTTOM_MAX_LEVELS];   // offset of each level's cells in the LDS arrays
  int tpoff[BOTTOM_MAX_LEVELS];  // offset of each level's top-plate faces
};

// Face coefficients of the bottom levels are staged in LDS in float32 (the
// sweeps then wait on LDS instead of global memory); in float64 they would
// not fit beside the iterates and stay in global memory.
template <typename T>
struct BottomFaces {
  static constexpr bool staged = sizeof(T) == 4;
  static constexpr int size = staged ? 4 * BOTTOM_LDS_CELLS : 1;
};

template <typename T>
__device__ __forceinline__ FaceCoef<T> bottom_co(const BottomArgs<T>* __restrict__ A, const T* lf, int l) {
  if (!BottomFaces<T>::staged) return A->co[l];
  const int o = A->coff[l];
  return FaceCoef<T>{lf + o, lf + BOTTOM_LDS_CELLS + o, lf + 2 * BOTTOM_LDS_CELLS + o,
                     lf + 3 * BOTTOM_LDS_CELLS + A->tpoff[l]};
}

__device__ __forceinline__ int geom_cells(const Geom& g) { return g.nx * g.ny * g.nz; }

// a / d for 0 <= a < 8192 and 1 <= d <= 1024 with rd = 1.0f / d: the
// float product lies within 1e-3 of the quotient plus 1/(2d), away from an
// integer by at least 1/(2d), so truncation gives the exact quotient (checked
// for every such a and d).  Integer division is the slowest part of the
// bottom kernel's index arithmetic otherwise.
__device__ __forceinline__ int small_div(int a, float rd) { return (int)(((float)a + 0.5f) * rd); }

// Half-sweep of one colour on a level whose dimensions are all even (every
// level that is smoothed): each row holds nx/2 cells of each colour, one in
// each x-pair; thread work items run over those cells only.  from_zero: the
// other colour is set to 0 and the iterate is not read.
template <typename T>
__device__ __forceinline__ void bottom_half_sweep(T* __restrict__ x, const T* __restrict__ b, const FaceCoef<T>& co,
                                                  const Geom& g, int colour, bool from_zero) {
  const int H = g.nx >> 1, nh = geom_cells(g) >> 1;
  const float rH = 1.0f / (float)H, rY = 1.0f / (float)g.ny;
  for (int r = threadIdx.x; r < nh; r += BottomThreads<T>::value) {
    const int row = small_div(r, rH), m = r - row * H;
    const int k = small_div(row, rY), j = row - k * g.ny;
    const int e = (colour + j + k) & 1;  // element of pair m with this colour
    const int i = 2 * m + e;
    const size_t c = cidx(g, i, j, k);
    if (from_zero) x[c + 1 - 2 * e] = T(0);
    const Stencil<T> st = co.load(g, i, j, k, c);
    T off = T(0);
    if (!from_zero) {
      const Nbrs<T> v = load_nbrs<T>(x, g, i, j, k, c, T(0), T(0));
      off = st.ww * v.w + st.we * v.e + st.ws * v.s + st.wn * v.n;
      if (k > 0) off += st.wb * v.b;
      if (k < g.nz - 1) off += st.wt * v.t;
    }
    x[c] = (b[c] + off) * recip(diag_cell(st, g, k));
  }
}

// x += P xc (or x = P xc when set) on level g from the next level in LDS:
// cell-centred trilinear interpolation with mirrored ghosts on the sides and
// negated ones through the plates.
template <typename T>
__device__ __forceinline__ void bottom_prolong(T* __restrict__ x, const T* __restrict__ xc, const Geom& g, bool set) {
  const int n = geom_cells(g);
  const int NX = g.nx >> 1, NY = g.ny >> 1, NZ = g.nz >> 1;
  const float rX = 1.0f / (float)g.nx, rY = 1.0f / (float)g.ny;
  for (int c = threadIdx.x; c < n; c += BottomThreads<T>::value) {
    const int row = small_div(c, rX), i = c - row * g.nx;
    const int k = small_div(row, rY), j = row - k * g.ny;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    int I2 = I + ((i & 1) ? 1 : -1);
    if (I2 < 0 || I2 >= NX) I2 = I;
    int J2 = J + ((j & 1) ? 1 : -1);
    if (J2 < 0 || J2 >= NY) J2 = J;
    int K2 = K + ((k & 1) ? 1 : -1);
    T sk = T(1);
    if (K2 < 0 || K2 >= NZ) {
      K2 = K;
      sk = T(-1);
    }
    const T q3 = T(0.75), q1 = T(0.25);
    const T* p = xc + K * NY * NX;
    const T* q = xc + K2 * NY * NX;
    const T pl = q3 * (q3 * p[J * NX + I] + q1 * p[J * NX + I2]) + q1 * (q3 * p[J2 * NX + I] + q1 * p[J2 * NX + I2]);
    const T ql = q3 * (q3 * q[J * NX + I] + q1 * q[J * NX + I2]) + q1 * (q3 * q[J2 * NX + I] + q1 * q[J2 * NX + I2]);
    const T v = q3 * pl + q1 * sk * ql;
    x[c] = set ? v : x[c] + v;
  }
}

// Coarsest level in LDS: x = A_L^{-1} b.
template <typename T>
__device__ __forceinline__ void bottom_coarsest(T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ Ainv,
                                                int n) {
  for (int r = threadIdx.x; r < n; r += BottomThreads<T>::value) {
    T acc = T(0);
    for (int c = 0; c < n; ++c) acc += Ainv[(size_t)c * n + r] * b[c];
    x[r] = acc;
  }
}

// V-cycle on the levels l0 .. L of the bottom kernel (L the coarsest), right
// side of level l0 in lb + off0; from x = 0, or from the guess in lx + off0
// when from_x (the coarser levels start from 0 either way).  Levels are
// stored one after the other in lx / lb.
template <typename T>
__device__ __forceinline__ void bottom_cycle(T* __restrict__ lx, T* __restrict__ lb, const T* lf,
                                             const BottomArgs<T>* __restrict__ A, int l0, int off0, bool from_x) {
  const int L = A->nlev - 1;
  const int nu_pre = A->nu_pre, nu_post = A->nu_post;
  int off = off0;
  for (int l = l0; l < L; ++l) {
    const Geom g = A->g[l];
    const FaceCoef<T> co = bottom_co<T>(A, lf, l);
    T* x = lx + off;
    T* b = lb + off;
    const bool guess = from_x && l == l0;
    if (!guess) {
      bottom_half_sweep<T>(x, b, co, g, 0, true);  // red from x = 0 (black set to 0)
      if (nu_pre == 0) {
        __syncthreads();
        for (int c = threadIdx.x; c < geom_cells(g); c += BottomThreads<T>::value) x[c] = T(0);
      }
      __syncthreads();
    }
    for (int it = 0; it < nu_pre; ++it) {
      if (it > 0 || guess) {
        bottom_half_sweep<T>(x, b, co, g, 0, false);
        __syncthreads();
      }
      bottom_half_sweep<T>(x, b, co, g, 1, false);
      __syncthreads();
    }
    // residual and restriction into b of level l+1
    const Geom gc = A->g[l + 1];
    T* bc = lb + off + geom_cells(g);
    const int nc = geom_cells(gc);
    const float rX = 1.0f / (float)gc.nx, rY = 1.0f / (float)gc.ny;
    for (int C = threadIdx.x; C < nc; C += BottomThreads<T>::value) {
      const int row = small_div(C, rX), I = C - row * gc.nx;
      const int K = small_div(row, rY), J = row - K * gc.ny;
      T sum = T(0);
      for (int d = 0; d < 8; ++d) {
        const int i = 2 * I + (d & 1), j = 2 * J + ((d >> 1) & 1), k = 2 * K + (d >> 2);
        const size_t c = cidx(g, i, j, k);
        const Stencil<T> st = co.load(g, i, j, k, c);
        const Nbrs<T> v = load_nbrs<T>(x, g, i, j, k, c, T(0), T(0));
        sum += b[c] - apply_cell(st, v);
      }
      bc[C] = sum * T(0.125);
    }
    __syncthreads();
    off += geom_cells(g);
  }
  bottom_coarsest<T>(lx + off, lb + off, A->Ainv, geom_cells(A->g[L]));
  __syncthreads();
  for (int l = L - 1; l >= l0; --l) {
    const Geom g = A->g[l];
    const FaceCoef<T> co = bottom_co<T>(A, lf, l);
    const int offc = off;  // level l+1
    off -= geom_cells(g);  // level l
    T* x = lx + off;
    const T* b = lb + off;
    bottom_prolong<T>(x, lx + offc, g, false);
    __syncthreads();
    for (int it = 0; it < nu_post; ++it) {
      bottom_half_sweep<T>(x, b, co, g, 1, false);
      __syncthreads();
      bottom_half_sweep<T>(x, b, co, g, 0, false);
      __syncthreads();
    }
  }
}

// The levels from the first bottom level (<= 4096 cells) to the coarsest in
// one workgroup, iterates and right sides in LDS.  FMG false: one V-cycle
// from zero for the right side b0.  FMG true: the full multigrid cycle over these
// levels: b0 restricted (mean of 8) to every level, the coarsest solved, then
// on each finer level one V-cycle from the interpolated coarser solution.
// The result of the first bottom level goes to x0.  (Two instantiations, so
// that each inlines the V-cycle once: register pressure.)
template <typename T, bool FMG>
__global__ __launch_bounds__(BottomThreads<T>::value) void k_vcycle_bottom(const BottomArgs<T>* __restrict__ A) {
  __shared__ T lx[BOTTOM_LDS_CELLS], lb[BOTTOM_LDS_CELLS];
  __shared__ T lf[BottomFaces<T>::size];
  const int L = A->nlev - 1;  // index of the coarsest level
  {
    const int n0 = geom_cells(A->g[0]);
    for (int c = threadIdx.x; c < n0; c += BottomThreads<T>::value) lb[c] = A->b0[c];
    if (BottomFaces<T>::staged) {
      for (int l = 0; l <= L; ++l) {
        const FaceCoef<T> co = A->co[l];
        const int n = geom_cells(A->g[l]), o = A->coff[l];
        for (int c = threadIdx.x; c < n; c += BottomThreads<T>::value) {
          lf[o + c] = co.wx[c];
          lf[BOTTOM_LDS_CELLS + o + c] = co.wy[c];
          lf[2 * BOTTOM_LDS_CELLS + o + c] = co.wz[c];
        }
        const int np = A->g[l].nx * A->g[l].ny, op = 3 * BOTTOM_LDS_CELLS + A->tpoff[l];
        for (int c = threadIdx.x; c < np; c += BottomThreads<T>::value) lf[op + c] = co.tp[c];
      }
    }
    __syncthreads();
  }
  if (!FMG) {
    bottom_cycle<T>(lx, lb, lf, A, 0, 0, false);
  } else {
    int off = 0;
    for (int l = 0; l < L; ++l) {  // right sides of every level
      const Geom g = A->g[l], gc = A->g[l + 1];
      const T* b = lb + off;
      T* bc = lb + off + geom_cells(g);
      const int nc = geom_cells(gc);
      const float rX = 1.0f / (float)gc.nx, rY = 1.0f / (float)gc.ny;
      for (int C = threadIdx.x; C < nc; C += BottomThreads<T>::value) {
        const int row = small_div(C, rX), I = C - row * gc.nx;
        const int K = small_div(row, rY), J = row - K * gc.ny;
        T sum = T(0);
        for (int d = 0; d < 8; ++d)
          sum += b[cidx(g, 2 * I + (d & 1), 2 * J + ((d >> 1) & 1), 2 * K + (d >> 2))];
        bc[C] = sum * T(0.125);
      }
      __syncthreads();
      off += geom_cells(g);
    }
    bottom_coarsest<T>(lx + off, lb + off, A->Ainv, geom_cells(A->g[L]));
    __syncthreads();
    for (int l = L - 1; l >= 0; --l) {
      const int offc = off;
      off -= geom_cells(A->g[l]);
      bottom_prolong<T>(lx + off, lx + offc, A->g[l], true);
      __syncthreads();
      bottom_cycle<T>(lx, lb, lf, A, l, off, true);
    }
  }
  {
    const int n0 = geom_cells(A->g[0]);
    for (int c = threadIdx.x; c < n0; c += BottomThreads<T>::value) A->x0[c] = lx[c];
  }
}


// Coarsest level: x = A_L^{-1} b with the precomputed (symmetric) inverse;
// thread r forms row r, reading column r of the symmetric inverse so that a
// wavefront's loads are contiguous.
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_coarse_solve(const T* __restrict__ Ainv, const T* __restrict__ b,
                                                           T* __restrict__ x, int n) {
  const int r = blockIdx.x * NTHREADS + threadIdx.y * BX + threadIdx.x;
  if (r >= n) return;
  T acc = T(0);
  for (int c = 0; c < n; ++c) acc += Ainv[(size_t)c * n + r] * b[c];
  x[r] = acc;
}

// ---------------------------------------------------------------------------
// Outer FGMRES kernels (float64).
// ---------------------------------------------------------------------------

// b = f + lifting, r = b - A x0 (r = b without x0); partial sums of ||b||^2
// and ||r||^2; r stored when r_out is given.
__global__ __launch_bounds__(NTHREADS) void k_init_residual(const double* __restrict__ f,
                                                            const double* __restrict__ a,
                                                            const double* __restrict__ x0, Geom g, double pb,
                                                            double pt, double* __restrict__ r_out,
                                                            double* __restrict__ partials, int kc) {
  // z-marching columns: x0 and a of the planes below / above in registers,
  // x- and y-neighbours from clamped addresses (zero flux through the sides)
  const Tile tl = xcd_tile();
  double acc[2] = {0.0, 0.0};
  const int i = tl.x * BX + threadIdx.x;
  if (i < g.nx) {
    const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
    const double hx = 0.5 * g.ihx2, hy = 0.5 * g.ihy2, hz = 0.5 * g.ihz2, pz = 2.0 * g.ihz2;
    const size_t dw = i > 0 ? 1 : 0, de = i < g.nx - 1 ? 1 : 0;
    const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
    for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
      const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
      size_t c = cidx(g, i, j, k0);
      double ac = a[c], ab = a[k0 > 0 ? c - sz : c];
      double xc = 0.0, xb = 0.0;
      if (x0) {
        xc = x0[c];
        xb = x0[k0 > 0 ? c - sz : c];
      }
      for (int k = k0; k < k1; ++k, c += sz) {
        const bool top = k == g.nz - 1;
        const size_t ct = top ? c : c + sz;
        const double at = a[ct];
        double bv = f[c];
        if (k == 0) bv += 2.0 * ac * pb * g.ihz2;
        if (top) bv += 2.0 * ac * pt * g.ihz2;
        double r = bv, xt = 0.0;
        if (x0) {
          xt = x0[ct];
          const double xw = x0[c - dw], aw = a[c - dw], xe = x0[c + de], ae = a[c + de];
          const double xs = x0[c - ds], as = a[c - ds], xn = x0[c + dn], an = a[c + dn];
          double s = (ac + aw) * hx * (xc - xw);
          s += (ac + ae) * hx * (xc - xe);
          s += (ac + as) * hy * (xc - xs);
          s += (ac + an) * hy * (xc - xn);
          s += k > 0 ? (ac + ab) * hz * (xc - xb) : pz * ac * xc;
          s += !top ? (ac + at) * hz * (xc - xt) : pz * ac * xc;
          r -= s;
        }
        if (r_out) r_out[c] = r;
        acc[0] += bv * bv;
        acc[1] += r * r;
        xb = xc;
        xc = xt;
        ab = ac;
        ac = at;
      }
    }
  }
  block_store_partials<2>(acc, 2, partials, gridDim.x * gridDim.y * gridDim.z);
}

// The operator of e18 (homogeneous plates) on natural-layout float64
// fields with one lane per x-pair (cells 2m, 2m + 1; nx even).  Each lane
// marches its pair through a z-chunk with x and a of the planes below and
// above in registers, loads the pair and its y-neighbours as 16-byte
// vectors and takes the x-neighbours from the adjacent lanes (the block's
// edge lanes load them).  PairOp::apply returns A x on both cells of plane
// k, summed in the order of the one-cell kernels (west, east, south,
// north, bottom, top), so the values are the same to the bit.  Lanes past
// the row's end (m >= H) run with clamped addresses so that every lane of
// a wave takes part in the exchange; their results are not used.
struct PairOp {
  double hx, hy, hz, pz;
  bool hw, he;  // x-faces of the pair outside it are interior faces
  __device__ explicit PairOp(const Geom& g, int m) {
    hx = 0.5 * g.ihx2;
    hy = 0.5 * g.ihy2;
    hz = 0.5 * g.ihz2;
    pz = 2.0 * g.ihz2;
    const int H = g.nx >> 1;
    hw = m > 0 && m < H;
    he = m < H - 1;
  }
  __device__ __forceinline__ double cell(double xc, double ac, bool hwest, double xw, double aw, bool heast,
                                         double xe, double ae, bool hs, double xs, double as, bool hn, double xn,
                                         double an, bool bot, double xb, double ab, bool top, double xt,
                                         double at) const {
    double s = hwest ? (ac + aw) * hx * (xc - xw) : 0.0;
    s += heast ? (ac + ae) * hx * (xc - xe) : 0.0;
    s += hs ? (ac + as) * hy * (xc - xs) : 0.0;
    s += hn ? (ac + an) * hy * (xc - xn) : 0.0;
    s += bot ? (ac + ab) * hz * (xc - xb) : pz * ac * xc;
    s += !top ? (ac + at) * hz * (xc - xt) : pz * ac * xc;
    return s;
  }
};

// March state and loads of one lane: X (scaled by sv as it is read) and a.
struct PairMarch {
  const double* __restrict__ x;
  const double* __restrict__ a;
  double sv;
  size_t sy, sz;
  __device__ __forceinline__ double2 ld2(const double* __restrict__ p, size_t c) const {
    return *reinterpret_cast<const double2*>(p + c);
  }
  __device__ __forceinline__ double2 lx2(size_t c) const {
    const double2 v = ld2(x, c);
    return make_double2(v.x * sv, v.y * sv);
  }
};

// Runs fn(c, s0, s1) for every pair of the lane's rows and z-chunk with
// s = A (sv x) on its two cells (c = natural index of cell 2m).
template <typename F>
__device__ __forceinline__ void pair_op_march(const double* __restrict__ x, double sv,
                                              const double* __restrict__ a, const Geom& g, int kc, F&& fn) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int lane = threadIdx.x;
  const int m = tl.x * BX + lane;
  const bool act = m < H;
  const int mm = act ? m : H - 1;
  const PairOp op(g, m);
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const PairMarch pm{x, a, sv, sy, sz};
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
    const bool hs = j > 0, hn = j < g.ny - 1;
    size_t c = ((size_t)k0 * g.ny + j) * g.nx + 2 * mm;
    double2 xc = pm.lx2(c), ac = pm.ld2(a, c);
    double2 xb = xc, ab = ac;
    if (k0 > 0) {
      xb = pm.lx2(c - sz);
      ab = pm.ld2(a, c - sz);
    }
    for (int k = k0; k < k1; ++k, c += sz) {
      const bool top = k == g.nz - 1, bot = k > 0;
      const double2 xt = top ? xc : pm.lx2(c + sz), at = top ? ac : pm.ld2(a, c + sz);
      const double2 xs = hs ? pm.lx2(c - sy) : xc, as = hs ? pm.ld2(a, c - sy) : ac;
      const double2 xn = hn ? pm.lx2(c + sy) : xc, an = hn ? pm.ld2(a, c + sy) : ac;
      double xw = __shfl_up(xc.y, 1, 64), aw = __shfl_up(ac.y, 1, 64);
      double xe = __shfl_down(xc.x, 1, 64), ae = __shfl_down(ac.x, 1, 64);
      if (lane == 0 && op.hw) {
        xw = x[c - 1] * sv;
        aw = a[c - 1];
      }
      if (lane == BX - 1 && op.he) {
        xe = x[c + 2] * sv;
        ae = a[c + 2];
      }
      const double s0 = op.cell(xc.x, ac.x, op.hw, xw, aw, true, xc.y, ac.y, hs, xs.x, as.x, hn, xn.x, an.x, bot,
                                xb.x, ab.x, top, xt.x, at.x);
      const double s1 = op.cell(xc.y, ac.y, true, xc.x, ac.x, op.he, xe, ae, hs, xs.y, as.y, hn, xn.y, an.y, bot,
                                xb.y, ab.y, top, xt.y, at.y);
      if (act) fn(c, k, s0, s1, ac);
      xb = xc;
      ab = ac;
      xc = xt;
      ac = at;
    }
  }
}

// w = A (s x) (s = *xscale, 1 when null) on natural-layout float64 vectors,
// one lane per x-pair (nx even), and the dots (w, u_v), v < NV (none when
// NV = 0): the values of k_op_natural.
template <int NV>
__global__ __launch_bounds__(NTHREADS) void k_op_pair(const double* __restrict__ x,
                                                      const double* __restrict__ xscale,
                                                      const double* __restrict__ a, Geom g,
                                                      double* __restrict__ w, const double* __restrict__ U,
                                                      size_t stride, double* __restrict__ partials, int kc) {
  double acc[NV > 0 ? NV : 1];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const double sv = xscale ? *xscale : 1.0;
  pair_op_march(x, sv, a, g, kc, [&](size_t c, int, double s0, double s1, const double2&) {
    *reinterpret_cast<double2*>(w + c) = make_double2(s0, s1);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double2 u = *reinterpret_cast<const double2*>(U + (size_t)q * stride + c);
      acc[q] += s0 * u.x + s1 * u.y;
    }
  });
  if constexpr (NV > 0) block_store_partials<NV>(acc, NV, partials, gridDim.x * gridDim.y * gridDim.z);
}

// k_init_residual with one lane per x-pair (nx even): b = f + lifting, r =
// b - A x0 (r = b without x0, which then reads a on the plates only), the
// same values; partial sums of ||b||^2 and ||r||^2; r stored when r_out is
// given.
template <bool HAS_X>
__global__ __launch_bounds__(NTHREADS) void k_init_residual_pair(const double* __restrict__ f,
                                                                 const double* __restrict__ a,
                                                                 const double* __restrict__ x0, Geom g, double pb,
                                                                 double pt, double* __restrict__ r_out,
                                                                 double* __restrict__ partials, int kc) {
  double acc[2] = {0.0, 0.0};
  auto rhs = [&](size_t c, int k, double& b0, double& b1, const double2& ac) {
    const double2 fv = *reinterpret_cast<const double2*>(f + c);
    b0 = fv.x;
    b1 = fv.y;
    if (k == 0) {
      b0 += 2.0 * ac.x * pb * g.ihz2;
      b1 += 2.0 * ac.y * pb * g.ihz2;
    }
    if (k == g.nz - 1) {
      b0 += 2.0 * ac.x * pt * g.ihz2;
      b1 += 2.0 * ac.y * pt * g.ihz2;
    }
  };
  if constexpr (HAS_X) {
    pair_op_march(x0, 1.0, a, g, kc, [&](size_t c, int k, double s0, double s1, const double2& ac) {
      double b0, b1;
      rhs(c, k, b0, b1, ac);
      const double r0 = b0 - s0, r1 = b1 - s1;
      if (r_out) *reinterpret_cast<double2*>(r_out + c) = make_double2(r0, r1);
      acc[0] += b0 * b0 + b1 * b1;
      acc[1] += r0 * r0 + r1 * r1;
    });
  } else {
    const Tile tl = xcd_tile();
    const int m = tl.x * BX + threadIdx.x;
    if (m < (g.nx >> 1)) {
      const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
      for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
        for (int k = k0; k < k1; ++k) {
          const size_t c = ((size_t)k * g.ny + j) * g.nx + 2 * m;
          const double2 ac = (k == 0 || k == g.nz - 1) ? *reinterpret_cast<const double2*>(a + c)
                                                      : make_double2(0.0, 0.0);
          double b0, b1;
          rhs(c, k, b0, b1, ac);
          if (r_out) *reinterpret_cast<double2*>(r_out + c) = make_double2(b0, b1);
          acc[0] += b0 * b0 + b1 * b1;
          acc[1] += b0 * b0 + b1 * b1;
        }
      }
    }
  }
  block_store_partials<2>(acc, 2, partials, gridDim.x * gridDim.y * gridDim.z);
}

// Flat grid-stride loop over n cells, block size NTHREADS.
#define GMG_FLAT_LOOP(c, n)                                                                        \
  for (size_t c = (size_t)blockIdx.x * NTHREADS + threadIdx.y * BX + threadIdx.x; c < (n);       \
       c += (size_t)gridDim.x * NTHREADS)

// w = A z (z promoted to float64) and the dots (w, u_v), v < NV.  Each
// thread marches one (i, j) column through its z-chunk and keeps the values
// of z and a on the planes below / above in registers.
template <typename TZ, int NV>
__global__ __launch_bounds__(NTHREADS) void k_op_multidot(const TZ* __restrict__ z, const double* __restrict__ a,
                                                          Geom g, double* __restrict__ w,
                                                          const double* __restrict__ U, size_t stride,
                                                          double* __restrict__ partials, int kc) {
  const Tile tl = xcd_tile();
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const int i = tl.x * BX + threadIdx.x;
  if (i < g.nx) {
    const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
    const double hx = 0.5 * g.ihx2, hy = 0.5 * g.ihy2, hz = 0.5 * g.ihz2, pz = 2.0 * g.ihz2;
    const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
    for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
      size_t c = cidx(g, i, j, k0);
      double zc = (double)z[c], ac = a[c];
      double zb = k0 > 0 ? (double)z[c - sz] : 0.0;
      double ab = k0 > 0 ? a[c - sz] : 0.0;
      for (int k = k0; k < k1; ++k, c += sz) {
        const bool top = k == g.nz - 1;
        const double zt = top ? 0.0 : (double)z[c + sz];
        const double at = top ? 0.0 : a[c + sz];
        double s = 0.0;
        if (i > 0) s += (ac + a[c - 1]) * hx * (zc - (double)z[c - 1]);
        if (i < g.nx - 1) s += (ac + a[c + 1]) * hx * (zc - (double)z[c + 1]);
        if (j > 0) s += (ac + a[c - sy]) * hy * (zc - (double)z[c - sy]);
        if (j < g.ny - 1) s += (ac + a[c + sy]) * hy * (zc - (double)z[c + sy]);
        s += k > 0 ? (ac + ab) * hz * (zc - zb) : pz * ac * zc;
        s += !top ? (ac + at) * hz * (zc - zt) : pz * ac * zc;
        w[c] = s;
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += s * U[(size_t)q * stride + c];
        zb = zc;
        zc = zt;
        ab = ac;
        ac = at;
      }
    }
  }
  block_store_partials<NV>(acc, NV, partials, gridDim.x * gridDim.y * gridDim.z);
}

// Dots (w, u_v), v < NV (flat launch).
template <int NV>
__global__ __launch_bounds__(NTHREADS) void k_multidot(const double* __restrict__ w, size_t n,
                                                       const double* __restrict__ U, size_t stride,
                                                       double* __restrict__ partials) {
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  GMG_FLAT_LOOP(c, n) {
    const double wv = w[c];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] += wv * U[(size_t)q * stride + c];
  }
  block_store_partials<NV>(acc, NV, partials, gridDim.x);
}

// w -= sum_v (h_v * s_v) u_v (h_v = (w, v_v) with v_v = s_v u_v), and the
// partial sums of ||w||^2 when want_norm (flat launch).
template <int NV>
__global__ __launch_bounds__(NTHREADS) void k_axpy_norm(double* __restrict__ w, size_t n,
                                                        const double* __restrict__ U, size_t stride,
                                                        const double* __restrict__ hcol,
                                                        const double* __restrict__ vscale, int want_norm,
                                                        double* __restrict__ partials) {
  double cf[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) cf[q] = hcol[q] * vscale[q];
  double acc[1] = {0.0};
  GMG_FLAT_LOOP(c, n) {
    double wv = w[c];
#pragma unroll
    for (int q = 0; q < NV; ++q) wv -= cf[q] * U[(size_t)q * stride + c];
    w[c] = wv;
    acc[0] += wv * wv;
  }
  if (want_norm) block_store_partials<1>(acc, 1, partials, gridDim.x);
}

// phi += sum_v y_v z_v (z promoted to float64; flat launch); set: phi = 0 +
// sum_v y_v z_v, without reading phi.
template <typename TZ, int NV>
__global__ __launch_bounds__(NTHREADS) void k_update(double* __restrict__ phi, size_t n, const TZ* __restrict__ Z,
                                                     size_t stride, Coeffs16 y, int set) {
  GMG_FLAT_LOOP(c, n) {
    double p = set ? 0.0 : phi[c];
#pragma unroll
    for (int q = 0; q < NV; ++q) p += y.v[q] * (double)Z[(size_t)q * stride + c];
    phi[c] = p;
  }
}

// Second reduction stage, one block: sum the per-block partials of nv
// vectors in a fixed order.  mode 0: out[v] = sum; mode 1: out[v] = sum *
// scale[v] (dots against lazily normalised vectors); mode 2 (nv = 1):
// out[0] = sqrt(sum), out2[0] = 1 / sqrt(sum) (0 if the sum is 0).
constexpr int FIN_THREADS = 1024;
constexpr int FIN_BATCH = 8;  // partials of one vector a thread loads per wait

__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const double* __restrict__ partials, int nblocks, int nv,
                                                          int mode, double* __restrict__ out,
                                                          const double* __restrict__ scale,
                                                          double* __restrict__ out2) {
  __shared__ double sm[MAXV][FIN_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // vector by vector, each thread adds its partials b = tid, tid +
  // FIN_THREADS, ... in that order, FIN_BATCH of them loaded before it waits
  // (one pass over b with every vector's partial per step waited for each
  // load: 17 us for five vectors of 16384 partials)
  for (int v = 0; v < nv; ++v) {
    const double* __restrict__ pv = partials + (size_t)v * nblocks;
    double sv = 0.0;
    for (int b0 = tid; b0 < nblocks; b0 += FIN_BATCH * FIN_THREADS) {
      double q[FIN_BATCH];
#pragma unroll
      for (int u = 0; u < FIN_BATCH; ++u) {
        const int b = b0 + u * FIN_THREADS;
        q[u] = pv[b < nblocks ? b : b0];
      }
#pragma unroll
      for (int u = 0; u < FIN_BATCH; ++u)
        if (b0 + u * FIN_THREADS < nblocks) sv += q[u];
    }
    const double t = wave_sum(sv);
    if (lane == 0) sm[v][wave] = t;
  }
  __syncthreads();
  if (tid < nv) {
    double t = 0.0;
    for (int w = 0; w < FIN_THREADS / 64; ++w) t += sm[tid][w];
    if (mode == 0) {
      out[tid] = t;
    } else if (mode == 1) {
      out[tid] = t * scale[tid];
    } else {
      const double r = sqrt(t);
      out[0] = r;
      out2[0] = r > 0.0 ? 1.0 / r : 0.0;
    }
  }
}

// y = A x - lifting (left side of e18 with plate values pb, pt).
__global__ __launch_bounds__(NTHREADS) void k_apply_bc(const double* __restrict__ x, const double* __restrict__ a,
                                                       Geom g, double pb, double pt, double* __restrict__ y,
                                                       int kc) {
  const Tile tl = xcd_tile();
  const int i = tl.x * BX + threadIdx.x;
  if (i >= g.nx) return;
  const CellCoef<double> co{a};
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
    for (int k = k0; k < k1; ++k) {
      const size_t c = cidx(g, i, j, k);
      const Stencil<double> st = co.load(g, i, j, k, c);
      const Nbrs<double> v = load_nbrs<double>(x, g, i, j, k, c, 2.0 * pb, 2.0 * pt);
      y[c] = apply_cell(st, v);
    }
  }
}

// dL/da_c = -1/2 sum_faces (d phi)_f (d lam)_f (see gmg_face_flux_grad).
__global__ __launch_bounds__(NTHREADS) void k_face_grad(const double* __restrict__ phi,
                                                        const double* __restrict__ lam, Geom g, double pb,
                                                        double pt, double* __restrict__ out, int kc) {
  // z-marching columns with the planes below / above in registers; x- and
  // y-neighbours from clamped addresses, whose terms vanish on the sides
  const Tile tl = xcd_tile();
  const int i = tl.x * BX + threadIdx.x;
  if (i >= g.nx) return;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const size_t dw = i > 0 ? 1 : 0, de = i < g.nx - 1 ? 1 : 0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
    const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
    size_t c = cidx(g, i, j, k0);
    double pc = phi[c], lc = lam[c];
    double pbv = phi[k0 > 0 ? c - sz : c], lbv = lam[k0 > 0 ? c - sz : c];
    for (int k = k0; k < k1; ++k, c += sz) {
      const bool top = k == g.nz - 1;
      const size_t ct = top ? c : c + sz;
      const double ptv = phi[ct], ltv = lam[ct];
      double s = (phi[c - dw] - pc) * (lam[c - dw] - lc) * g.ihx2;
      s += (phi[c + de] - pc) * (lam[c + de] - lc) * g.ihx2;
      s += (phi[c - ds] - pc) * (lam[c - ds] - lc) * g.ihy2;
      s += (phi[c + dn] - pc) * (lam[c + dn] - lc) * g.ihy2;
      s += (pbv - pc) * (lbv - lc) * g.ihz2;  // zero at k = 0 (clamped to the cell)
      s += (ptv - pc) * (ltv - lc) * g.ihz2;  // zero on the top layer
      double gsum = -0.5 * s;
      if (k == 0) gsum -= 2.0 * (pc - pb) * lc * g.ihz2;
      if (top) gsum -= 2.0 * (pc - pt) * lc * g.ihz2;
      out[c] = gsum;
      pbv = pc;
      lbv = lc;
      pc = ptv;
      lc = ltv;
    }
  }
}

// k_face_grad with one lane per x-pair (nx even): phi and lam of the pair
// and of its y-neighbours as 16-byte loads, the x-neighbours outside the
// pair from the adjacent lanes (the block's edge lanes load them), the same
// arithmetic in the same order (a missing neighbour is the cell itself, so
// its term is zero).  Lanes past the row's end run clamped, for the
// exchange, and store nothing.
__global__ __launch_bounds__(NTHREADS) void k_face_grad_pair(const double* __restrict__ phi,
                                                             const double* __restrict__ lam, Geom g, double pb,
                                                             double pt, double* __restrict__ out, int kc) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int lane = threadIdx.x;
  const int m = tl.x * BX + lane;
  const bool act = m < H;
  const int mm = act ? m : H - 1;
  const bool hw = mm > 0, he = mm < H - 1;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  auto ld2 = [](const double* __restrict__ p, size_t c) { return *reinterpret_cast<const double2*>(p + c); };
  for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
    const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
    size_t c = ((size_t)k0 * g.ny + j) * g.nx + 2 * mm;
    double2 pc = ld2(phi, c), lc = ld2(lam, c);
    double2 pbv = k0 > 0 ? ld2(phi, c - sz) : pc, lbv = k0 > 0 ? ld2(lam, c - sz) : lc;
    for (int k = k0; k < k1; ++k, c += sz) {
      const bool top = k == g.nz - 1;
      const size_t ct = top ? c : c + sz;
      const double2 ptv = ld2(phi, ct), ltv = ld2(lam, ct);
      const double2 ps = ld2(phi, c - ds), ls = ld2(lam, c - ds), pn = ld2(phi, c + dn), ln = ld2(lam, c + dn);
      double pw = __shfl_up(pc.y, 1, 64), lw = __shfl_up(lc.y, 1, 64);
      double pe = __shfl_down(pc.x, 1, 64), le = __shfl_down(lc.x, 1, 64);
      if (lane == 0 && hw) {
        pw = phi[c - 1];
        lw = lam[c - 1];
      }
      if (lane == BX - 1 && he) {
        pe = phi[c + 2];
        le = lam[c + 2];
      }
      if (!hw) {
        pw = pc.x;
        lw = lc.x;
      }
      if (!he) {
        pe = pc.y;
        le = lc.y;
      }
      auto cell = [&](double p0, double l0, double pwv, double lwv, double pev, double lev, double psv, double lsv,
                      double pnv, double lnv, double pbc, double lbc, double ptc, double ltc) {
        double s = (pwv - p0) * (lwv - l0) * g.ihx2;
        s += (pev - p0) * (lev - l0) * g.ihx2;
        s += (psv - p0) * (lsv - l0) * g.ihy2;
        s += (pnv - p0) * (lnv - l0) * g.ihy2;
        s += (pbc - p0) * (lbc - l0) * g.ihz2;  // zero at k = 0 (the cell itself)
        s += (ptc - p0) * (ltc - l0) * g.ihz2;  // zero on the top layer
        double gsum = -0.5 * s;
        if (k == 0) gsum -= 2.0 * (p0 - pb) * l0 * g.ihz2;
        if (top) gsum -= 2.0 * (p0 - pt) * l0 * g.ihz2;
        return gsum;
      };
      const double g0 = cell(pc.x, lc.x, pw, lw, pc.y, lc.y, ps.x, ls.x, pn.x, ln.x, pbv.x, lbv.x, ptv.x, ltv.x);
      const double g1 = cell(pc.y, lc.y, pc.x, lc.x, pe, le, ps.y, ls.y, pn.y, ln.y, pbv.y, lbv.y, ptv.y, ltv.y);
      if (act) *reinterpret_cast<double2*>(out + c) = make_double2(g0, g1);
      pbv = pc;
      lbv = lc;
      pc = ptv;
      lc = ltv;
    }
  }
}

// In-place Gauss-Jordan inversion of an SPD matrix A (n x n, row-major),
// step k: k_gj_save copies row k and column k, then k_gj_step updates every
// element from the copies (pivot p = A[k][k]): A[k][k] = 1/p, row k / p,
// column k / -p, A[i][j] -= A[i][k] A[k][j] / p elsewhere.  After steps 0 ..
// n-1, A holds A^{-1}.  Grid of k_gj_step: x over columns, y over rows.
__global__ __launch_bounds__(256) void k_gj_save(const double* __restrict__ A, int n, int k,
                                                 double* __restrict__ rk, double* __restrict__ ck) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    rk[i] = A[(size_t)k * n + i];
    ck[i] = A[(size_t)i * n + k];
  }
}

__global__ __launch_bounds__(256) void k_gj_step(double* __restrict__ A, int n, int k,
                                                 const double* __restrict__ rk, const double* __restrict__ ck) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  if (j >= n) return;
  const double ip = 1.0 / rk[k];
  double v;
  if (i == k)
    v = j == k ? ip : rk[j] * ip;
  else if (j == k)
    v = -ck[i] * ip;
  else
    v = A[(size_t)i * n + j] - ck[i] * (rk[j] * ip);
  A[(size_t)i * n + j] = v;
}

__global__ __launch_bounds__(256) void k_gj_diag(const double* __restrict__ A, int n, double* __restrict__ d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = A[(size_t)i * n + i];
}

// ---------------------------------------------------------------------------
// Setup kernels (hierarchy of face coefficients, float64).
// ---------------------------------------------------------------------------

// Level-1 faces from the finest cell coefficient: mean of the 4 finest faces
// (each the arithmetic mean of its two cells) on every coarse face; plate
// faces from the plate coefficients a_c of the first / last layer.
__global__ __launch_bounds__(NTHREADS) void k_faces_from_cells(const double* __restrict__ a, Geom g,
                                                               double* __restrict__ wx, double* __restrict__ wy,
                                                               double* __restrict__ wz, double* __restrict__ tp,
                                                               int kc) {
  const int NX = g.nx >> 1, NY = g.ny >> 1, NZ = g.nz >> 1;
  const int I = blockIdx.x * BX + threadIdx.x;
  if (I >= NX) return;
  const int K0 = blockIdx.z * kc, K1 = min(NZ, K0 + kc);
  auto A = [&](int i, int j, int k) { return a[cidx(g, i, j, k)]; };
  for (int J = blockIdx.y * BY + threadIdx.y; J < NY; J += gridDim.y * BY) {
    for (int K = K0; K < K1; ++K) {
      const size_t C = ((size_t)K * NY + J) * NX + I;
      double sx = 0.0, sy = 0.0, sz = 0.0;
      for (int p = 0; p < 2; ++p) {
        for (int q = 0; q < 2; ++q) {
          if (I > 0) sx += 0.5 * (A(2 * I - 1, 2 * J + p, 2 * K + q) + A(2 * I, 2 * J + p, 2 * K + q));
          if (J > 0) sy += 0.5 * (A(2 * I + p, 2 * J - 1, 2 * K + q) + A(2 * I + p, 2 * J, 2 * K + q));
          if (K > 0)
            sz += 0.5 * (A(2 * I + p, 2 * J + q, 2 * K - 1) + A(2 * I + p, 2 * J + q, 2 * K));
          else
            sz += A(2 * I + p, 2 * J + q, 0);
        }
      }
      wx[C] = 0.25 * sx;
      wy[C] = 0.25 * sy;
      wz[C] = 0.25 * sz;
      if (K == NZ - 1) {
        double st = 0.0;
        for (int p = 0; p < 2; ++p)
          for (int q = 0; q < 2; ++q) st += A(2 * I + p, 2 * J + q, g.nz - 1);
        tp[(size_t)J * NX + I] = 0.25 * st;
      }
    }
  }
}

// Level l+1 faces from level l faces (g = level l grid).
__global__ __launch_bounds__(NTHREADS) void k_coarsen_faces(const double* __restrict__ wx,
                                                            const double* __restrict__ wy,
                                                            const double* __restrict__ wz,
                                                            const double* __restrict__ tp, Geom g,
                                                            double* __restrict__ cwx, double* __restrict__ cwy,
                                                            double* __restrict__ cwz, double* __restrict__ ctp,
                                                            int kc) {
  const int NX = g.nx >> 1, NY = g.ny >> 1, NZ = g.nz >> 1;
  const int I = blockIdx.x * BX + threadIdx.x;
  if (I >= NX) return;
  const int K0 = blockIdx.z * kc, K1 = min(NZ, K0 + kc);
  for (int J = blockIdx.y * BY + threadIdx.y; J < NY; J += gridDim.y * BY) {
    for (int K = K0; K < K1; ++K) {
      const size_t C = ((size_t)K * NY + J) * NX + I;
      double sx = 0.0, sy = 0.0, sz = 0.0;
      for (int p = 0; p < 2; ++p) {
        for (int q = 0; q < 2; ++q) {
          sx += wx[cidx(g, 2 * I, 2 * J + p, 2 * K + q)];
          sy += wy[cidx(g, 2 * I + p, 2 * J, 2 * K + q)];
          sz += wz[cidx(g, 2 * I + p, 2 * J + q, 2 * K)];
        }
      }
      cwx[C] = 0.25 * sx;
      cwy[C] = 0.25 * sy;
      cwz[C] = 0.25 * sz;
      if (K == NZ - 1) {
        double st = 0.0;
        for (int p = 0; p < 2; ++p)
          for (int q = 0; q < 2; ++q) st += tp[(size_t)(2 * J + p) * g.nx + 2 * I + q];
        ctp[(size_t)J * NX + I] = 0.25 * st;
      }
    }
  }
}

// Per-block minimum of a and count of non-finite entries (flat grid-stride).
__global__ __launch_bounds__(NTHREADS) void k_check_coef(const double* __restrict__ a, size_t n,
                                                         double* __restrict__ partials) {
  __shared__ double smin[NTHREADS];
  __shared__ double sbad[NTHREADS];
  const int tid = threadIdx.y * BX + threadIdx.x;
  double mn = 1.0e308, bad = 0.0;
  for (size_t c = (size_t)blockIdx.x * NTHREADS + tid; c < n; c += (size_t)gridDim.x * NTHREADS) {
    const double v = a[c];
    if (!isfinite(v)) bad += 1.0;
    else mn = fmin(mn, v);
  }
  smin[tid] = mn;
  sbad[tid] = bad;
  __syncthreads();
  for (int s = NTHREADS / 2; s > 0; s >>= 1) {
    if (tid < s) {
      smin[tid] = fmin(smin[tid], smin[tid + s]);
      sbad[tid] += sbad[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[2 * blockIdx.x] = smin[0];
    partials[2 * blockIdx.x + 1] = sbad[0];
  }
}

template <typename TO, typename TI>
__global__ __launch_bounds__(NTHREADS) void k_convert(const TI* __restrict__ in, TO* __restrict__ out, size_t n) {
  for (size_t c = (size_t)blockIdx.x * NTHREADS + threadIdx.y * BX + threadIdx.x; c < n;
       c += (size_t)gridDim.x * NTHREADS)
    out[c] = (TO)in[c];
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_fill(T* __restrict__ out, T v, size_t n) {
  for (size_t c = (size_t)blockIdx.x * NTHREADS + threadIdx.y * BX + threadIdx.x; c < n;
       c += (size_t)gridDim.x * NTHREADS)
    out[c] = v;
}

}  // namespace gmg
