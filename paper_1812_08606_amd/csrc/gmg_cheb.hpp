// Kernels of the Chebyshev(2)+SSOR smoother (Sec. 3.2, eq. qntn) and of the
// Arnoldi estimate of its bounds.  The SSOR steps themselves are the
// red-black half-sweep kernels of the Gauss-Seidel smoother (one symmetric
// sweep from zero: red, black, red); these kernels add the residuals the
// Chebyshev recurrence needs, its vector update, and the start vector and
// coarse-level vector passes of the estimate.  All are single streaming
// passes bound by HBM bandwidth.
#pragma once

#include "gmg_fine.hpp"

namespace gmg {

// SplitMix64 (Steele, Lea and Flood 2014; output function of Vigna's
// reference version): output k >= 1 of the generator seeded with s is the
// mix of the state s + k * 0x9E3779B97F4A7C15 (mod 2^64).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long s, unsigned long long k) {
  unsigned long long z = s + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Arnoldi start vector: out[c] = 2 (z >> 11) 2^-53 - 1, z = output c + 1 of
// SplitMix64 seeded with s (flat launch; exact in float64).
__global__ __launch_bounds__(NTHREADS) void k_uniform_start(double* __restrict__ out, size_t n,
                                                            unsigned long long s) {
  GMG_FLAT_LOOP(c, n) {
    const unsigned long long z = splitmix64(s, (unsigned long long)c + 1ull);
    out[c] = 2.0 * ((double)(z >> 11) * 1.1102230246251565e-16) - 1.0;
  }
}

// r = b - A x on a coarse level (natural layout, stored face coefficients;
// homogeneous plates), or r = A x when b is null.  One lane per cell of a
// row, marching a z-chunk with x of the planes below and above in
// registers; neighbours behind a Neumann side come from clamped (valid)
// addresses and get zero weight.
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_resid_face(const T* __restrict__ x, const T* __restrict__ b,
                                                         FaceCoef<T> co, Geom g, T* __restrict__ r, int kc) {
  const Tile tl = xcd_tile();
  const int i = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const T ix = (T)g.ihx2, iy = (T)g.ihy2, iz = (T)g.ihz2;
  const bool hw = i > 0, he = i < g.nx - 1, hs = j > 0, hn = j < g.ny - 1;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  size_t c = cidx(g, i, j, k0);
  T xc = x[c], xb = x[k0 > 0 ? c - sz : c];
  for (int k = k0; k < k1; ++k, c += sz) {
    const bool top = k == g.nz - 1;
    const T xt = x[top ? c : c + sz];
    const T ww = co.wx[c], we = co.wx[he ? c + 1 : c];
    const T ws = co.wy[c], wn = co.wy[hn ? c + sy : c];
    const T wb = co.wz[c], wt = top ? co.tp[(size_t)j * g.nx + i] : co.wz[c + sz];
    const T xw = x[hw ? c - 1 : c], xe = x[he ? c + 1 : c];
    const T xs = x[hs ? c - sy : c], xn = x[hn ? c + sy : c];
    const T ax = (hw ? ww * (xc - xw) : T(0)) + (he ? we * (xc - xe) : T(0));
    const T ay = (hs ? ws * (xc - xs) : T(0)) + (hn ? wn * (xc - xn) : T(0));
    const T az = (k > 0 ? wb * (xc - xb) : T(2) * wb * xc) + (!top ? wt * (xc - xt) : T(2) * wt * xc);
    const T Ax = ax * ix + ay * iy + az * iz;
    r[c] = b ? b[c] - Ax : Ax;
    xb = xc;
    xc = xt;
  }
}

// Finest level: r = s u - A x in the natural layout, float64, with x
// colour-split (precision T, promoted), u the natural float64 right side
// scaled by s = *bscale (1 when null) and the operator of the finest level
// (cell coefficient a of precision T, face = mean of the two cells,
// homogeneous plates).  x null: x = 0.  One lane per x-pair of a row,
// marching a z-chunk; every load has a clamped (valid) address.
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_resid_split(const T* __restrict__ X, const double* __restrict__ u,
                                                          const double* __restrict__ bscale,
                                                          const T* __restrict__ a, Geom g, size_t hn,
                                                          double* __restrict__ r, int kc) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (m >= H || j >= g.ny) return;
  const double s = bscale ? *bscale : 1.0;
  const double hx = 0.5 * g.ihx2, hy = 0.5 * g.ihy2, hz = 0.5 * g.ihz2, pz = 2.0 * g.ihz2;
  const size_t ty = (size_t)H, tz = (size_t)H * g.ny;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const bool hw = m > 0, he = m < H - 1, hs = j > 0, hn_ = j < g.ny - 1;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int k = k0; k < k1; ++k) {
    const bool hb = k > 0, ht = k < g.nz - 1;
    const size_t q = sidx(g, m, j, k);
    const size_t cn = ((size_t)k * g.ny + j) * g.nx + 2 * m;
    // pairs (left = cell 2m, right = 2m+1) of this row and of the rows and
    // planes around it; the colour of cell 2m is the parity of j + k
    double l0 = 0.0, r0 = 0.0, lw = 0.0, rw = 0.0, le = 0.0, re = 0.0, ls = 0.0, rs = 0.0;
    double ln = 0.0, rn = 0.0, lb = 0.0, rb = 0.0, lt = 0.0, rt = 0.0;
    if (X) {
      const int p = (j + k) & 1;
      split_pair<double>(X, hn, q, p, l0, r0);
      split_pair<double>(X, hn, hw ? q - 1 : q, p, lw, rw);
      split_pair<double>(X, hn, he ? q + 1 : q, p, le, re);
      split_pair<double>(X, hn, hs ? q - ty : q, hs ? 1 - p : p, ls, rs);
      split_pair<double>(X, hn, hn_ ? q + ty : q, hn_ ? 1 - p : p, ln, rn);
      split_pair<double>(X, hn, hb ? q - tz : q, hb ? 1 - p : p, lb, rb);
      split_pair<double>(X, hn, ht ? q + tz : q, ht ? 1 - p : p, lt, rt);
    }
    const double a0 = (double)a[cn], a1 = (double)a[cn + 1];
    const double aw = (double)a[hw ? cn - 1 : cn], ae = (double)a[he ? cn + 2 : cn + 1];
    const double as0 = (double)a[hs ? cn - sy : cn], as1 = (double)a[hs ? cn + 1 - sy : cn + 1];
    const double an0 = (double)a[hn_ ? cn + sy : cn], an1 = (double)a[hn_ ? cn + 1 + sy : cn + 1];
    const double ab0 = (double)a[hb ? cn - sz : cn], ab1 = (double)a[hb ? cn + 1 - sz : cn + 1];
    const double at0 = (double)a[ht ? cn + sz : cn], at1 = (double)a[ht ? cn + 1 + sz : cn + 1];
    // cell 2m: west neighbour is the right cell of pair m-1, east the pair's right cell
    double A0 = (hw ? (a0 + aw) * hx * (l0 - rw) : 0.0) + (a0 + a1) * hx * (l0 - r0);
    A0 += (hs ? (a0 + as0) * hy * (l0 - ls) : 0.0) + (hn_ ? (a0 + an0) * hy * (l0 - ln) : 0.0);
    A0 += (hb ? (a0 + ab0) * hz * (l0 - lb) : pz * a0 * l0) + (ht ? (a0 + at0) * hz * (l0 - lt) : pz * a0 * l0);
    // cell 2m+1: west is the pair's left cell, east the left cell of pair m+1
    double A1 = (a1 + a0) * hx * (r0 - l0) + (he ? (a1 + ae) * hx * (r0 - le) : 0.0);
    A1 += (hs ? (a1 + as1) * hy * (r0 - rs) : 0.0) + (hn_ ? (a1 + an1) * hy * (r0 - rn) : 0.0);
    A1 += (hb ? (a1 + ab1) * hz * (r0 - rb) : pz * a1 * r0) + (ht ? (a1 + at1) * hz * (r0 - rt) : pz * a1 * r0);
    const double2 uv = *reinterpret_cast<const double2*>(u + cn);
    *reinterpret_cast<double2*>(r + cn) = make_double2(s * uv.x - A0, s * uv.y - A1);
  }
}

// One step of the Chebyshev recurrence on gridDim.y ranges of n elements
// (range y starts at y * stride: both colours of a colour-split array, or
// one natural array): d = c1 d + c2 e (mode bit 0: d = c2 e), then x += d
// (mode bit 1: x = d).  Coefficients in float64, stored in T.
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_cheb_update(T* __restrict__ x, T* __restrict__ d,
                                                          const T* __restrict__ e, double c1, double c2, size_t n,
                                                          size_t stride, int mode) {
  const size_t off = (size_t)blockIdx.y * stride;
  GMG_FLAT_LOOP(c, n) {
    const size_t q = off + c;
    const double dv = (mode & 1) ? c2 * (double)e[q] : c1 * (double)d[q] + c2 * (double)e[q];
    const T dt = (T)dv;
    d[q] = dt;
    x[q] = (mode & 2) ? dt : (T)((double)x[q] + (double)dt);
  }
}

// Bound estimate, coarse levels: y = x * (*s) (the lazily normalised
// Arnoldi vector made explicit for the operator kernel; flat launch).
__global__ __launch_bounds__(NTHREADS) void k_scale_by(double* __restrict__ y, const double* __restrict__ x,
                                                       const double* __restrict__ s, size_t n) {
  const double sv = *s;
  GMG_FLAT_LOOP(c, n) { y[c] = x[c] * sv; }
}

// Bound estimate, coarse levels: out = x promoted to float64 and the
// per-block partial sums of the dots (out, u_v), v < NV (flat launch).
template <typename T, int NV>
__global__ __launch_bounds__(NTHREADS) void k_convert_dots(const T* __restrict__ x, double* __restrict__ out,
                                                           size_t n, const double* __restrict__ U, size_t stride,
                                                           double* __restrict__ partials) {
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  GMG_FLAT_LOOP(c, n) {
    const double v = (double)x[c];
    out[c] = v;
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] += v * U[(size_t)q * stride + c];
  }
  block_store_partials<NV>(acc, NV, partials, gridDim.x);
}

}  // namespace gmg
