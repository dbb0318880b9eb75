// Vector kernels of the other Krylov methods compared with FGMRES (GMRES,
// CG, FCG, CGS, BiCGSTAB; Sec. 5.3, Table t1).  They work on natural-layout
// float64 vectors; the preconditioner's output is converted once.
#pragma once

#include "gmg_fine.hpp"

namespace gmg {

// out = z promoted to float64 in the natural layout, z colour-split (colour
// c at offset c * hn).  One lane per x-pair of a row, z-chunks of kc planes.
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_split_to_natural(const T* __restrict__ Z, size_t hn, Geom g,
                                                               double* __restrict__ out, int kc) {
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (m >= H || j >= g.ny) return;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  for (int k = k0; k < k1; ++k) {
    const size_t q = sidx(g, m, j, k);
    const int e = (j + k) & 1;  // colour of cell 2m
    const double2 v = make_double2((double)Z[(size_t)e * hn + q], (double)Z[(size_t)(1 - e) * hn + q]);
    *reinterpret_cast<double2*>(out + ((size_t)k * g.ny + j) * g.nx + 2 * m) = v;
  }
}

// y = c0 x0 + c1 x1 + c2 x2 (x1, x2 may be null and are then skipped) and,
// when want_norm, the per-block partial sums of ||y||^2 (flat launch).  y may
// be one of the inputs: every element is read before it is written, by the
// same thread.
__global__ __launch_bounds__(NTHREADS) void k_lincomb3(double* y, const double* x0, const double* x1,
                                                       const double* x2, double c0, double c1, double c2, size_t n,
                                                       int want_norm, double* __restrict__ partials) {
  double acc[1] = {0.0};
  GMG_FLAT_LOOP(c, n) {
    double v = c0 * x0[c];
    if (x1) v += c1 * x1[c];
    if (x2) v += c2 * x2[c];
    y[c] = v;
    acc[0] += v * v;
  }
  if (want_norm) block_store_partials<1>(acc, 1, partials, gridDim.x);
}

// w = A (s x) on natural float64 vectors (the operator of e18 with
// homogeneous plate values; s = *xscale, 1 when xscale is null, applied to
// every value of x as it is read) and the dots (w, u_v), v < NV (none when
// NV = 0).  Each thread marches one (i, j) column through its z-chunk (rows
// strided when the grid has more columns than blocks allow), x and a of the
// planes below / above in registers; x- and y-neighbours are loaded from
// clamped addresses, which make the flux through a side face exactly zero
// (Neumann).
template <int NV>
__global__ __launch_bounds__(NTHREADS) void k_op_natural(const double* __restrict__ xr,
                                                         const double* __restrict__ xscale,
                                                         const double* __restrict__ a, Geom g,
                                                         double* __restrict__ w, const double* __restrict__ U,
                                                         size_t stride, double* __restrict__ partials, int kc) {
  const Tile tl = xcd_tile();
  double acc[NV > 0 ? NV : 1];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const double sv = xscale ? *xscale : 1.0;
  auto x = [&](size_t c) { return xr[c] * sv; };
  const int i = tl.x * BX + threadIdx.x;
  if (i < g.nx) {
    const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
    const double hx = 0.5 * g.ihx2, hy = 0.5 * g.ihy2, hz = 0.5 * g.ihz2, pz = 2.0 * g.ihz2;
    const size_t dw = i > 0 ? 1 : 0, de = i < g.nx - 1 ? 1 : 0;
    const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
    for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
      const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
      size_t c = cidx(g, i, j, k0);
      double xc = x(c), ac = a[c];
      double xb = x(k0 > 0 ? c - sz : c), ab = a[k0 > 0 ? c - sz : c];
      for (int k = k0; k < k1; ++k, c += sz) {
        const bool top = k == g.nz - 1;
        const size_t ct = top ? c : c + sz;
        const double xt = x(ct), at = a[ct];
        const double xw = x(c - dw), aw = a[c - dw], xe = x(c + de), ae = a[c + de];
        const double xs = x(c - ds), as = a[c - ds], xn = x(c + dn), an = a[c + dn];
        double s = (ac + aw) * hx * (xc - xw);
        s += (ac + ae) * hx * (xc - xe);
        s += (ac + as) * hy * (xc - xs);
        s += (ac + an) * hy * (xc - xn);
        s += k > 0 ? (ac + ab) * hz * (xc - xb) : pz * ac * xc;
        s += !top ? (ac + at) * hz * (xc - xt) : pz * ac * xc;
        w[c] = s;
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += s * U[(size_t)q * stride + c];
        xb = xc;
        xc = xt;
        ab = ac;
        ac = at;
      }
    }
  }
  if constexpr (NV > 0) block_store_partials<NV>(acc, NV, partials, gridDim.x * gridDim.y * gridDim.z);
}

// out = z promoted to float64 in the natural layout (z colour-split, colour
// c at offset c * hn) and the per-block partial sums of the dots (out, u_v),
// v < NV.  One lane per x-pair of a row, rows strided when the grid has
// fewer rows than the level, z-chunks of kc planes.
template <typename T, int NV>
__global__ __launch_bounds__(NTHREADS) void k_split_to_natural_dots(const T* __restrict__ Z, size_t hn, Geom g,
                                                                    double* __restrict__ out,
                                                                    const double* __restrict__ U, size_t stride,
                                                                    double* __restrict__ partials, int kc) {
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const Tile tl = xcd_tile();
  const int H = g.nx >> 1;
  const int m = tl.x * BX + threadIdx.x;
  if (m < H) {
    const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
    for (int j = tl.y * BY + threadIdx.y; j < g.ny; j += gridDim.y * BY) {
      for (int k = k0; k < k1; ++k) {
        const size_t q = sidx(g, m, j, k);
        const int e = (j + k) & 1;  // colour of cell 2m
        const double v0 = (double)Z[(size_t)e * hn + q], v1 = (double)Z[(size_t)(1 - e) * hn + q];
        const size_t c = ((size_t)k * g.ny + j) * g.nx + 2 * m;
        *reinterpret_cast<double2*>(out + c) = make_double2(v0, v1);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double2 u = *reinterpret_cast<const double2*>(U + (size_t)v * stride + c);
          acc[v] += v0 * u.x + v1 * u.y;
        }
      }
    }
  }
  block_store_partials<NV>(acc, NV, partials, gridDim.x * gridDim.y * gridDim.z);
}

}  // namespace gmg
