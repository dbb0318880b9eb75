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

// The two kernels above with one lane per x-pair (nx even): the pair and
// its y-neighbours as 16-byte loads, the planes below and above in
// registers, the x-neighbours outside the pair from the adjacent lanes (the
// block's edge lanes load them); the same arithmetic.  Lanes past the row's
// end run clamped, for the exchange, and store nothing.
struct PairLane {
  int H, m, mm;
  bool act, hw, he;
  __device__ PairLane(const Geom& g, int m_) : H(g.nx >> 1), m(m_) {
    act = m < H;
    mm = act ? m : H - 1;
    hw = mm > 0;
    he = mm < H - 1;
  }
  // x-neighbours of the pair (cell 2m-1 and 2m+2; the cell itself at a side)
  __device__ __forceinline__ void xnb(const double* __restrict__ v, size_t c, const double2& vc, double& w,
                                      double& e) const {
    w = __shfl_up(vc.y, 1, 64);
    e = __shfl_down(vc.x, 1, 64);
    if (threadIdx.x == 0 && hw) w = v[c - 1];
    if (threadIdx.x == BX - 1 && he) e = v[c + 2];
    if (!hw) w = vc.x;
    if (!he) e = vc.y;
  }
};

__device__ __forceinline__ double2 ldp(const double* __restrict__ p, size_t c) {
  return *reinterpret_cast<const double2*>(p + c);
}

__global__ __launch_bounds__(NTHREADS) void k_assemble_step_pair(const double* __restrict__ ne,
                                                                 const double* __restrict__ np, Geom g, StepCoef p,
                                                                 double* __restrict__ a, double* __restrict__ f,
                                                                 int kc) {
  const Tile tl = xcd_tile();
  const PairLane pl(g, tl.x * BX + threadIdx.x);
  const int j = tl.y * BY + threadIdx.y;
  if (j >= g.ny) return;  // whole waves (a wave is one row)
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  size_t c = cidx(g, 2 * pl.mm, j, k0);
  double2 ec = ldp(ne, c), eb = k0 > 0 ? ldp(ne, c - sz) : ec;
  for (int k = k0; k < k1; ++k, c += sz) {
    const double2 et = ldp(ne, k < g.nz - 1 ? c + sz : c);
    const double2 es = ldp(ne, c - ds), en = ldp(ne, c + dn), pv = ldp(np, c);
    double ew, ee;
    pl.xnb(ne, c, ec, ew, ee);
    auto cell = [&](double e, double w_, double e_, double s_, double n_, double b_, double t_, double pp, double& av,
                    double& fv) {
      const double dxx = e_ - 2.0 * e + w_, dyy = n_ - 2.0 * e + s_, dzz = t_ - 2.0 * e + b_;
      av = p.eps0_over_e + p.tau_eff * (p.mu_p * pp + p.mu_e * e);
      fv = pp - e - p.tau_eff * (p.cx * dxx + p.cy * dyy + p.cz * dzz);
    };
    double a0, a1, f0, f1;
    cell(ec.x, ew, ec.y, es.x, en.x, eb.x, et.x, pv.x, a0, f0);
    cell(ec.y, ec.x, ee, es.y, en.y, eb.y, et.y, pv.y, a1, f1);
    if (pl.act) {
      *reinterpret_cast<double2*>(a + c) = make_double2(a0, a1);
      *reinterpret_cast<double2*>(f + c) = make_double2(f0, f1);
    }
    eb = ec;
    ec = et;
  }
}

__global__ __launch_bounds__(NTHREADS) void k_electric_field_pair(const double* __restrict__ phi, Geom g,
                                                                  double hx, double hy, double hz, double pb,
                                                                  double pt, double* __restrict__ ex,
                                                                  double* __restrict__ ey, double* __restrict__ ez,
                                                                  double* __restrict__ em, int kc) {
  const Tile tl = xcd_tile();
  const PairLane pl(g, tl.x * BX + threadIdx.x);
  const int j = tl.y * BY + threadIdx.y;
  if (j >= g.ny) return;  // whole waves (a wave is one row)
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const size_t ds = j > 0 ? sy : 0, dn = j < g.ny - 1 ? sy : 0;
  const int k0 = tl.z * kc, k1 = min(g.nz, k0 + kc);
  size_t c = cidx(g, 2 * pl.mm, j, k0);
  double2 pc = ldp(phi, c), pbv = k0 > 0 ? ldp(phi, c - sz) : pc;
  if (k0 == 0) pbv = make_double2(2.0 * pb - pc.x, 2.0 * pb - pc.y);
  for (int k = k0; k < k1; ++k, c += sz) {
    const double2 ptl = ldp(phi, k < g.nz - 1 ? c + sz : c);
    const double2 ptv = k < g.nz - 1 ? ptl : make_double2(2.0 * pt - pc.x, 2.0 * pt - pc.y);
    const double2 ps = ldp(phi, c - ds), pn = ldp(phi, c + dn);
    double pw, pe;
    pl.xnb(phi, c, pc, pw, pe);
    auto cell = [&](double w_, double e_, double s_, double n_, double b_, double t_, double& vx, double& vy,
                    double& vz, double& vm) {
      vx = -(e_ - w_) / (2.0 * hx);
      vy = -(n_ - s_) / (2.0 * hy);
      vz = -(t_ - b_) / (2.0 * hz);
      vm = sqrt(vx * vx + vy * vy + vz * vz);
    };
    double x0, y0, z0, m0, x1, y1, z1, m1;
    cell(pw, pc.y, ps.x, pn.x, pbv.x, ptv.x, x0, y0, z0, m0);
    cell(pc.x, pe, ps.y, pn.y, pbv.y, ptv.y, x1, y1, z1, m1);
    if (pl.act) {
      *reinterpret_cast<double2*>(ex + c) = make_double2(x0, x1);
      *reinterpret_cast<double2*>(ey + c) = make_double2(y0, y1);
      *reinterpret_cast<double2*>(ez + c) = make_double2(z0, z1);
      *reinterpret_cast<double2*>(em + c) = make_double2(m0, m1);
    }
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
