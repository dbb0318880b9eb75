// Elliptic side of one semi-implicit time step (Sec. 2.1-2.2): the
// coefficient and right side of the variable-coefficient problem (the
// definition of P^n and the right side of eq. e18), and the electric field
// E = -grad phi by central differences.  Both are single passes bound by HBM
// bandwidth: one lane per cell of a row, marching a z-chunk with the column's
// planes k-1, k, k+1 in registers and branch-free clamped loads of the x and
// y neighbours (the same cache lines the adjacent lanes and rows load).
#pragma once

#include "gmg_kernels.hpp"

namespace gmg {

// P = eps0/e + tau_eff (mu_p n_p + mu_e n_e); cx, cy, cz = D_d / h_d^2.
struct StepCoef {
  double eps0_over_e, tau_eff, mu_e, mu_p, cx, cy, cz;
};

// a = P, f = n_p - n_e - tau_eff (cx dxx n_e + cy dyy n_e + cz dzz n_e), the
// second differences with ghost cells equal to the boundary cells
// (homogeneous Neumann condition of n_e on every boundary, Sec. 1).
__global__ __launch_bounds__(NTHREADS) void k_assemble_step(const double* __restrict__ ne,
                                                            const double* __restrict__ np, Geom g, StepCoef p,
                                                            double* __restrict__ a, double* __restrict__ f,
                                                            int kc) {
  const Tile tl = xcd_tile();
  const int i = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const size_t dw = i > 0 ? 1 : 0, de = i < g.nx - 1 ? 1 : 0;
  const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  size_t c = cidx(g, i, j, k0);
  double eb = ne[k0 > 0 ? c - sz : c], ec = ne[c];
  for (int k = k0; k < k1; ++k, c += sz) {
    const double et = ne[k < g.nz - 1 ? c + sz : c];
    const double ew = ne[c - dw], ee = ne[c + de], es = ne[c - ds], en = ne[c + dn];
    const double pv = np[c];
    const double dxx = ee - 2.0 * ec + ew, dyy = en - 2.0 * ec + es, dzz = et - 2.0 * ec + eb;
    a[c] = p.eps0_over_e + p.tau_eff * (p.mu_p * pv + p.mu_e * ec);
    f[c] = pv - ec - p.tau_eff * (p.cx * dxx + p.cy * dyy + p.cz * dzz);
    eb = ec;
    ec = et;
  }
}

// E = -grad phi by central differences; ghosts equal to the boundary cells on
// the sides (Neumann), mirrored through the plates (2 phi_b - phi_c); and |E|.
__global__ __launch_bounds__(NTHREADS) void k_electric_field(const double* __restrict__ phi, Geom g, double hx,
                                                             double hy, double hz, double pb, double pt,
                                                             double* __restrict__ ex, double* __restrict__ ey,
                                                             double* __restrict__ ez, double* __restrict__ em,
                                                             int kc) {
  const Tile tl = xcd_tile();
  const int i = tl.x * BX + threadIdx.x;
  const int j = tl.y * BY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const size_t dw = i > 0 ? 1 : 0, de = i < g.nx - 1 ? 1 : 0;
  const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  size_t c = cidx(g, i, j, k0);
  double pbv = phi[k0 > 0 ? c - sz : c], pc = phi[c];
  if (k0 == 0) pbv = 2.0 * pb - pc;
  for (int k = k0; k < k1; ++k, c += sz) {
    const double ptl = phi[k < g.nz - 1 ? c + sz : c];
    const double ptv = k < g.nz - 1 ? ptl : 2.0 * pt - pc;
    const double pw = phi[c - dw], pe = phi[c + de], ps = phi[c - ds], pn = phi[c + dn];
    const double vx = -(pe - pw) / (2.0 * hx), vy = -(pn - ps) / (2.0 * hy), vz = -(ptv - pbv) / (2.0 * hz);
    ex[c] = vx;
    ey[c] = vy;
    ez[c] = vz;
    em[c] = sqrt(vx * vx + vy * vy + vz * vz);
    pbv = pc;
    pc = ptl;
  }
}

// Density update of the time step: n_out = n + dt L for both species (the
// predictor of eq. e1 with dt = tau/2, the corrector of eq. e2 and the
// first-order step with dt = tau).  Outputs may be the inputs n (same index
// read, then written), so no restrict qualifiers.
__global__ __launch_bounds__(NTHREADS) void k_density_update(const double* ne, const double* np, const double* le,
                                                             const double* lp, double dt, double* oe, double* op,
                                                             size_t n) {
  GMG_FLAT_LOOP(c, n) {
    const double e = ne[c] + dt * le[c];
    const double p = np[c] + dt * lp[c];
    oe[c] = e;
    op[c] = p;
  }
}

}  // namespace gmg
