// gmg.hip -- host side of the GMG-preconditioned FGMRES solver: workspace
// layout, hierarchy set-up, V-cycle schedule, FGMRES(m) with host Givens
// least squares (Algorithm 1, Sec. 3.1), profiling, and the C ABI of gmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "gmg.h"
#include "gmg_fine.hpp"
#include "gmg_step.hpp"
#include "gmg_krylov.hpp"
#include "gmg_cheb.hpp"
#include "gmg_face_sym.hpp"

using namespace gmg;

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_RESTART = 32;
// coarsest levels of more cells than this are inverted on the GPU
// (Gauss-Jordan), smaller ones on the host (Cholesky)
constexpr int GJ_MIN_CELLS = 1024;
constexpr double BREAKDOWN_TOL = 1e-14;
constexpr int CHEB_ARNOLDI = 10;  // Arnoldi steps of the Chebyshev bound estimate
constexpr int CHEB_DEGREE = 2;    // degree of the Chebyshev smoothing polynomial
// device scalars of level l's bound estimate, CHEB_STRIDE doubles: column j
// of the Hessenberg matrix at j * (CHEB_ARNOLDI + 1) (entries 0 .. j + 1),
// the basis scales at CHEB_SCALES, the start vector's norm at CHEB_NORM0
constexpr int CHEB_SCALES = CHEB_ARNOLDI * (CHEB_ARNOLDI + 1);
constexpr int CHEB_NORM0 = CHEB_SCALES + CHEB_ARNOLDI + 1;
constexpr int CHEB_STRIDE = 128;
static_assert(CHEB_NORM0 < CHEB_STRIDE, "estimate scalars overflow their slot");

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }


struct LevelShape {
  int nx, ny, nz;
  double hx, hy, hz;
  size_t n() const { return (size_t)nx * ny * nz; }
  Geom geom() const { return Geom{nx, ny, nz, 1.0 / (hx * hx), 1.0 / (hy * hy), 1.0 / (hz * hz)}; }
};

// Level shapes: halve all dimensions while every one is even and >= 4.
std::vector<LevelShape> level_shapes(int nx, int ny, int nz, double hx, double hy, double hz) {
  std::vector<LevelShape> v;
  v.push_back({nx, ny, nz, hx, hy, hz});
  while (true) {
    const LevelShape& l = v.back();
    if (l.nx % 2 || l.ny % 2 || l.nz % 2 || l.nx < 4 || l.ny < 4 || l.nz < 4) break;
    v.push_back({l.nx / 2, l.ny / 2, l.nz / 2, 2 * l.hx, 2 * l.hy, 2 * l.hz});
  }
  return v;
}

// Byte offsets of every buffer in the caller's workspace.
struct LevelOffsets {
  size_t wx, wy, wz, tp;          // precision T faces (levels >= 1)
  size_t wx64, wy64, wz64, tp64;  // float64 faces (levels >= 1; == T faces in FP64)
  size_t b, x;                    // precision T right side and iterate
  size_t x2;                      // second iterate: the fused sweeps ping-pong between x and x2
  size_t cr, ce, cd;              // Chebyshev smoother: residual, SSOR output, direction (T)
};

struct Layout {
  std::vector<LevelShape> shapes;
  std::vector<LevelOffsets> lv;
  size_t V, Z, a32, b0, xs, partials, scal, cinv, bargs, total;
  size_t cgjm, cgjb;  // GPU inverse of a large coarsest level: float64 matrix (mixed), row / column buffers
  size_t cr0, cd0;  // Chebyshev smoother, finest level: float64 natural residual, T colour-split direction
  size_t rr;        // transpose restriction: residual of the level being restricted (finest: float64)
  size_t chs;       // Chebyshev smoother: device scalars of every level's bound estimate
  size_t tsize;  // bytes of the V-cycle precision
  size_t ldv;    // elements between consecutive Krylov vectors (v_i and z_i)
  size_t hn;     // elements of one colour array of a colour-split finest-level field
  int m;
};

bool options_valid(const gmg_options* o) {
  if (!o) return false;
  if (o->restart < 1 || o->restart > MAX_RESTART) return false;
  if (o->max_iter < 0) return false;
  if (o->nu_pre < 0 || o->nu_pre > 8 || o->nu_post < 0 || o->nu_post > 8) return false;
  if (o->precision != GMG_FP64 && o->precision != GMG_MIXED) return false;
  if (o->coarse_max_cells < 1 || o->coarse_max_cells > 4096) return false;
  if (o->fine_sweep < GMG_SWEEP_AUTO || o->fine_sweep > GMG_SWEEP_FUSED) return false;
  if (o->cold_cycle != GMG_CYCLE_V && o->cold_cycle != GMG_CYCLE_FMG) return false;
  if (o->graphs != 0 && o->graphs != 1) return false;
  if (o->smoother != GMG_SMOOTH_RBGS && o->smoother != GMG_SMOOTH_CHEBYSHEV) return false;
  if (o->warm_cycle != GMG_CYCLE_V && o->warm_cycle != GMG_CYCLE_FMG) return false;
  if (o->smoother == GMG_SMOOTH_CHEBYSHEV && (o->cold_cycle != GMG_CYCLE_V || o->warm_cycle != GMG_CYCLE_V))
    return false;
  if (o->restriction != GMG_RESTRICT_MEAN && o->restriction != GMG_RESTRICT_TRANSPOSE) return false;
  if (o->restriction == GMG_RESTRICT_TRANSPOSE &&
      (o->smoother != GMG_SMOOTH_RBGS || o->cold_cycle != GMG_CYCLE_V || o->warm_cycle != GMG_CYCLE_V))
    return false;
  return true;
}

int make_layout(int nx, int ny, int nz, double hx, double hy, double hz, const gmg_options* o, Layout* L) {
  if (!options_valid(o)) return GMG_ERR_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20)) return GMG_ERR_SHAPE;
  if ((nx + BX - 1) / BX > MAX_RED_BLOCKS) return GMG_ERR_SHAPE;
  if ((ny + BY - 1) / BY > 65535) return GMG_ERR_SHAPE;  // grid y of the z-marching kernels
  L->shapes = level_shapes(nx, ny, nz, hx, hy, hz);
  const LevelShape& last = L->shapes.back();
  if (last.n() > (size_t)o->coarse_max_cells) return GMG_ERR_SHAPE;
  const bool mixed = o->precision == GMG_MIXED;
  L->tsize = mixed ? 4 : 8;
  L->m = o->restart;
  const size_t N = L->shapes[0].n();
  const int nl = (int)L->shapes.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  // every Krylov vector, and each colour half of a colour-split one, starts
  // 512-byte aligned
  L->hn = ((N + 1) / 2 + 63) / 64 * 64;
  L->ldv = 2 * L->hn;
  // the Chebyshev smoother's bound estimate keeps its Arnoldi basis in the
  // Krylov slots
  const bool cheb = o->smoother == GMG_SMOOTH_CHEBYSHEV;
  const int nvslots = cheb ? std::max(L->m + 1, CHEB_ARNOLDI + 1) : L->m + 1;
  L->V = take((size_t)nvslots * L->ldv * 8);
  L->Z = take((size_t)L->m * L->ldv * L->tsize);
  L->a32 = mixed ? take(N * 4) : 0;
  // finest-level right side in T (colour-split; natural when the finest
  // level is also the coarsest)
  L->b0 = take(L->ldv * L->tsize);
  // second finest-level iterate: the fused symmetric sweeps ping-pong
  // between it and z
  L->xs = nl > 1 ? take(L->ldv * L->tsize) : 0;
  L->lv.assign(nl, LevelOffsets{});
  for (int l = 1; l < nl; ++l) {
    const LevelShape& s = L->shapes[l];
    const size_t n = s.n(), nxy = (size_t)s.nx * s.ny;
    LevelOffsets& lo = L->lv[l];
    lo.wx64 = take(n * 8);
    lo.wy64 = take(n * 8);
    lo.wz64 = take(n * 8);
    lo.tp64 = take(nxy * 8);
    if (mixed) {
      lo.wx = take(n * 4);
      lo.wy = take(n * 4);
      lo.wz = take(n * 4);
      lo.tp = take(nxy * 4);
    } else {
      lo.wx = lo.wx64;
      lo.wy = lo.wy64;
      lo.wz = lo.wz64;
      lo.tp = lo.tp64;
    }
    lo.b = take(n * L->tsize);
    lo.x = take(n * L->tsize);
    lo.x2 = l < nl - 1 ? take(n * L->tsize) : 0;
    if (cheb && l < nl - 1) {
      lo.cr = take(n * L->tsize);
      lo.ce = take(n * L->tsize);
      lo.cd = take(n * L->tsize);
    }
  }
  L->rr = o->restriction == GMG_RESTRICT_TRANSPOSE && nl > 1 ? take(N * 8) : 0;
  L->cr0 = cheb && nl > 1 ? take(N * 8) : 0;
  L->cd0 = cheb && nl > 1 ? take(L->ldv * L->tsize) : 0;
  L->chs = cheb && nl > 1 ? take((size_t)(nl - 1) * CHEB_STRIDE * 8) : 0;
  L->partials = take((size_t)MAXV * MAX_RED_BLOCKS * 8);
  L->scal = take((size_t)(L->m * (L->m + 2) + (L->m + 2) + 32) * 8);
  const size_t nc = last.n();
  L->cinv = take(nc * nc * L->tsize);
  L->cgjm = nc > GJ_MIN_CELLS && mixed ? take(nc * nc * 8) : 0;
  L->cgjb = nc > GJ_MIN_CELLS ? take(2 * nc * 8) : 0;
  L->bargs = take(sizeof(BottomArgs<double>));
  L->total = off;
  return GMG_OK;
}

// The levels small enough for the one-workgroup bottom kernel: the first
// level l >= 1 from which every level has at most BOTTOM_MAX_CELLS cells, the
// coarsest at most BOTTOM_MAX_COARSEST, and at most BOTTOM_MAX_LEVELS levels
// remain; -1 when that leaves only the coarsest (a plain direct solve).
constexpr size_t BOTTOM_MAX_CELLS = 4096;
constexpr size_t BOTTOM_MAX_COARSEST = 512;

int bottom_level(const Layout& L) {
  const int nl = (int)L.shapes.size();
  if (nl < 3 || L.shapes.back().n() > BOTTOM_MAX_COARSEST) return -1;
  int l = nl - 1;
  size_t cells = L.shapes[l].n();
  while (l > 1 && L.shapes[l - 1].n() <= BOTTOM_MAX_CELLS && nl - (l - 1) <= BOTTOM_MAX_LEVELS &&
         cells + L.shapes[l - 1].n() <= (size_t)BOTTOM_LDS_CELLS) {
    --l;
    cells += L.shapes[l].n();
  }
  return l < nl - 1 ? l : -1;
}

struct Launch {
  dim3 grid, block;
  int kc;
  int nblocks() const { return (int)(grid.x * grid.y * grid.z); }
};

// Column-marching launch over an nx x ny x nz grid with at most max_blocks
// blocks (the reduction kernels keep one partial per block).
Launch col_launch(int nx, int ny, int nz, int max_blocks = MAX_RED_BLOCKS) {
  const int gx = (nx + BX - 1) / BX;
  int gy = (ny + BY - 1) / BY;
  if ((long long)gx * gy > max_blocks) gy = std::max(1, max_blocks / gx);
  gy = std::min(gy, 65535);
  int gz = std::max(1, std::min(nz, max_blocks / (gx * gy)));
  const int kc = (nz + gz - 1) / gz;
  gz = (nz + kc - 1) / kc;
  return Launch{dim3(gx, gy, gz), dim3(BX, BY, 1), kc};
}

// One lane per cell of a row, rows of BY threads, z-chunks of at least
// min_kc planes, about `target` blocks.
Launch cell_launch(int nx, int ny, int nz, long long target, int min_kc) {
  const int gx = (nx + BX - 1) / BX, gy = (ny + BY - 1) / BY;
  int kc = (int)std::max<long long>(min_kc, ((long long)nz * gx * gy + target - 1) / target);
  kc = std::min(kc, nz);
  return Launch{dim3(gx, gy, (nz + kc - 1) / kc), dim3(BX, BY, 1), kc};
}

Launch flat_launch(size_t n) {
  const size_t b = std::min<size_t>((n + NTHREADS - 1) / NTHREADS, 8192);
  return Launch{dim3((unsigned)std::max<size_t>(b, 1)), dim3(BX, BY, 1), 0};
}

// Per-kernel event timing.
struct Profiler {
  bool on = false;
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, long long>> totals;
  std::map<std::string, const char*> names;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

}  // namespace

struct gmg_ctx {
  int nx, ny, nz;
  double hx, hy, hz;
  gmg_options opt;
  const double* a;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  Layout L;
  size_t N;
  bool mixed;
  int nc;  // cells on the coarsest level
  int cus;  // compute units of the device
  int bottom_from;  // first level run by the one-workgroup bottom kernel (-1: none)
  bool fmg_now;     // the running solve preconditions with full multigrid cycles
  bool gmres_mode;  // GMRES: one preconditioned-vector slot, x updated by M (V y)
  int nprec;        // preconditioner applications of the running solve
  // captured preconditioner applications, by (input, scale, output, FMG)
  struct GraphKey {
    const void *u, *s, *z;
    bool fmg;
    bool operator<(const GraphKey& o) const {
      if (u != o.u) return u < o.u;
      if (s != o.s) return s < o.s;
      if (z != o.z) return z < o.z;
      return fmg < o.fmg;
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  bool graphs_broken = false;
  hipStream_t cap_stream = nullptr;  // capture only (the caller's may be the null stream)
  double* pinned;
  hipError_t err;
  Profiler prof;
  // host Givens state
  std::vector<double> R, cs, sn, g, y;
  // Chebyshev smoother: Arnoldi estimate and recurrence coefficients
  // (c1, c2 of each of the CHEB_DEGREE steps) per smoothed level
  std::vector<double> cheb_lam;
  std::vector<std::array<double, 2 * CHEB_DEGREE>> cheb_coef;
};

namespace {

template <typename P>
P* wsp(gmg_ctx* c, size_t off) {
  return reinterpret_cast<P*>(c->ws + off);
}

double* scal_hcol(gmg_ctx* c, int j) { return wsp<double>(c, c->L.scal) + (size_t)j * (c->L.m + 2); }
double* scal_vscale(gmg_ctx* c) { return wsp<double>(c, c->L.scal) + (size_t)c->L.m * (c->L.m + 2); }
double* scal_misc(gmg_ctx* c) { return scal_vscale(c) + (c->L.m + 2); }

struct ProfScope {
  gmg_ctx* c;
  const char* name;
  hipEvent_t b = nullptr;
  ProfScope(gmg_ctx* c_, const char* n) : c(c_), name(n) {
    if (c->prof.on) {
      hipEvent_t a = c->prof.get();
      b = c->prof.get();
      if (a && b) {
        (void)hipEventRecord(a, c->stream);
        c->prof.pending.push_back({name, a, b});
      } else {
        b = nullptr;
      }
    }
  }
  ~ProfScope() {
    if (b) (void)hipEventRecord(b, c->stream);
  }
};

#define GMG_LAUNCH(ctx, name, kern, L, ...)                                              \
  do {                                                                                   \
    ProfScope _ps((ctx), (name));                                                        \
    hipLaunchKernelGGL(kern, (L).grid, (L).block, 0, (ctx)->stream, __VA_ARGS__);         \
    hipError_t _e = hipGetLastError();                                                   \
    if (_e != hipSuccess && (ctx)->err == hipSuccess) (ctx)->err = _e;                   \
  } while (0)

void note(gmg_ctx* c, hipError_t e) {
  if (e != hipSuccess && c->err == hipSuccess) c->err = e;
}

// ---------------------------------------------------------------------------
// Hierarchy set-up (per coefficient).
// ---------------------------------------------------------------------------

// Cholesky factor and inverse of the symmetric positive definite n x n
// matrix M (row-major), in place; returns false if not positive definite.
// The inverse is formed column by column from L L^T x = e_c (the forward
// solve starts at row c, where e_c's solution becomes nonzero), the columns
// split over host threads; L^T is kept row-major for the backward solves.
// sum_{k in [k0, k1)} x[k] y[k] in four interleaved partial sums (lets the
// host compiler vectorise the loop without reassociating it itself)
double dot4(const double* x, const double* y, int k0, int k1) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = k0;
  for (; k + 3 < k1; k += 4) {
    s0 += x[k] * y[k];
    s1 += x[k + 1] * y[k + 1];
    s2 += x[k + 2] * y[k + 2];
    s3 += x[k + 3] * y[k + 3];
  }
  for (; k < k1; ++k) s0 += x[k] * y[k];
  return (s0 + s1) + (s2 + s3);
}

bool spd_inverse(std::vector<double>& M, int n) {
  std::vector<double> Lf(M);
  for (int j = 0; j < n; ++j) {
    const double* lj = &Lf[(size_t)j * n];
    double d = Lf[(size_t)j * n + j] - dot4(lj, lj, 0, j);
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    Lf[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      const double* li = &Lf[(size_t)i * n];
      Lf[(size_t)i * n + j] = (li[j] - dot4(li, lj, 0, j)) / d;
    }
  }
  std::vector<double> Lt((size_t)n * n, 0.0);  // Lt[i][k] = L[k][i]
  for (int i = 0; i < n; ++i)
    for (int k = 0; k <= i; ++k) Lt[(size_t)k * n + i] = Lf[(size_t)i * n + k];
  auto columns = [&](int c0, int c1) {
    std::vector<double> col(n);
    for (int c = c0; c < c1; ++c) {
      std::fill(col.begin(), col.begin() + c, 0.0);
      for (int i = c; i < n; ++i) {
        const double* li = &Lf[(size_t)i * n];
        col[i] = ((i == c ? 1.0 : 0.0) - dot4(li, col.data(), c, i)) / li[i];
      }
      for (int i = n - 1; i >= 0; --i) {
        const double* ti = &Lt[(size_t)i * n];
        col[i] = (col[i] - dot4(ti, col.data(), i + 1, n)) / ti[i];
      }
      for (int i = 0; i < n; ++i) M[(size_t)i * n + c] = col[i];
    }
  };
  const int nt = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
  if (n < 256 || nt == 1) {
    columns(0, n);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) pool.emplace_back(columns, (int)((long long)n * t / nt), (int)((long long)n * (t + 1) / nt));
    for (auto& th : pool) th.join();
  }
  // symmetrise the rounding
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double v = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
      M[(size_t)i * n + j] = M[(size_t)j * n + i] = v;
    }
  return true;
}

// Dense matrix of the coarsest level from its face coefficients (host).
void assemble_coarsest(const LevelShape& s, const std::vector<double>& wx, const std::vector<double>& wy,
                       const std::vector<double>& wz, const std::vector<double>& tp, const double* a_fine,
                       bool fine_cells, std::vector<double>& M) {
  const int nx = s.nx, ny = s.ny, nz = s.nz;
  const int n = nx * ny * nz;
  const double ix = 1.0 / (s.hx * s.hx), iy = 1.0 / (s.hy * s.hy), iz = 1.0 / (s.hz * s.hz);
  M.assign((size_t)n * n, 0.0);
  auto id = [&](int i, int j, int k) { return (k * ny + j) * nx + i; };
  auto couple = [&](int p, int q, double w) {
    M[(size_t)p * n + p] += w;
    M[(size_t)q * n + q] += w;
    M[(size_t)p * n + q] -= w;
    M[(size_t)q * n + p] -= w;
  };
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = id(i, j, k);
        if (fine_cells) {  // single-level grid: faces from the cell coefficient
          const double ac = a_fine[c];
          if (i + 1 < nx) couple(c, id(i + 1, j, k), 0.5 * (ac + a_fine[id(i + 1, j, k)]) * ix);
          if (j + 1 < ny) couple(c, id(i, j + 1, k), 0.5 * (ac + a_fine[id(i, j + 1, k)]) * iy);
          if (k + 1 < nz) couple(c, id(i, j, k + 1), 0.5 * (ac + a_fine[id(i, j, k + 1)]) * iz);
          if (k == 0) M[(size_t)c * n + c] += 2.0 * ac * iz;
          if (k == nz - 1) M[(size_t)c * n + c] += 2.0 * ac * iz;
        } else {
          if (i + 1 < nx) couple(c, id(i + 1, j, k), wx[id(i + 1, j, k)] * ix);
          if (j + 1 < ny) couple(c, id(i, j + 1, k), wy[id(i, j + 1, k)] * iy);
          if (k + 1 < nz) couple(c, id(i, j, k + 1), wz[id(i, j, k + 1)] * iz);
          if (k == 0) M[(size_t)c * n + c] += 2.0 * wz[c] * iz;
          if (k == nz - 1) M[(size_t)c * n + c] += 2.0 * tp[j * nx + i] * iz;
        }
      }
}

// Inverse of the coarsest matrix M (n x n, SPD, row-major host copy) on the
// GPU by in-place Gauss-Jordan elimination without pivoting (every pivot of
// an SPD matrix is positive): n steps, each saving row and column k, then
// updating every element.  O(n^3) work spread over the GPU instead of the
// host's O(n^3) Cholesky inverse (about 20 s at n = 4096 on 8 host cores);
// the result lands in cinv in the V-cycle precision.
int gpu_inverse(gmg_ctx* c, const std::vector<double>& M, int n) {
  const Layout& L = c->L;
  double* A = c->mixed ? wsp<double>(c, L.cgjm) : wsp<double>(c, L.cinv);
  double* rk = wsp<double>(c, L.cgjb);
  double* ck = rk + n;
  note(c, hipMemcpyAsync(A, M.data(), (size_t)n * n * 8, hipMemcpyHostToDevice, c->stream));
  const Launch vl{dim3((unsigned)((n + 255) / 256)), dim3(256, 1, 1), 0};
  const Launch ml{dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256, 1, 1), 0};
  for (int k = 0; k < n; ++k) {
    GMG_LAUNCH(c, "gj_save", k_gj_save, vl, (const double*)A, n, k, rk, ck);
    GMG_LAUNCH(c, "gj_step", k_gj_step, ml, A, n, k, (const double*)rk, (const double*)ck);
  }
  // the diagonal of an SPD inverse is positive
  GMG_LAUNCH(c, "gj_diag", k_gj_diag, vl, (const double*)A, n, rk);
  std::vector<double> d(n);
  note(c, hipMemcpyAsync(d.data(), rk, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  note(c, hipStreamSynchronize(c->stream));
  if (c->err != hipSuccess) return GMG_ERR_HIP;
  for (double v : d)
    if (!(v > 0.0) || !std::isfinite(v)) return GMG_ERR_NONFINITE;
  if (c->mixed) {
    const size_t nn = (size_t)n * n;
    GMG_LAUNCH(c, "convert_f64_f32", (k_convert<float, double>), flat_launch(nn), (const double*)A,
               wsp<float>(c, L.cinv), nn);
    note(c, hipStreamSynchronize(c->stream));
  }
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

int build_hierarchy(gmg_ctx* c) {
  Layout& L = c->L;
  const int nl = (int)L.shapes.size();
  // check the coefficient: finite and positive
  {
    const Launch fl = flat_launch(c->N);
    const int nb = std::min<int>(fl.grid.x, MAX_RED_BLOCKS);
    Launch l2 = fl;
    l2.grid.x = nb;
    double* part = wsp<double>(c, L.partials);
    GMG_LAUNCH(c, "check_coef", k_check_coef, l2, c->a, c->N, part);
    std::vector<double> h(2 * (size_t)nb);
    note(c, hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    note(c, hipStreamSynchronize(c->stream));
    if (c->err != hipSuccess) return GMG_ERR_HIP;
    double mn = 1e308, bad = 0;
    for (int b = 0; b < nb; ++b) {
      mn = std::min(mn, h[2 * b]);
      bad += h[2 * b + 1];
    }
    if (bad > 0) return GMG_ERR_NONFINITE;
    if (!(mn > 0.0)) return GMG_ERR_ARG;
  }
  if (c->mixed) {
    const Launch fl = flat_launch(c->N);
    GMG_LAUNCH(c, "convert_f64_f32", (k_convert<float, double>), fl, c->a, wsp<float>(c, L.a32), c->N);
  }
  for (int l = 1; l < nl; ++l) {
    const LevelShape& f = L.shapes[l - 1];
    const LevelShape& s = L.shapes[l];
    const LevelOffsets& o = L.lv[l];
    const Launch lc = col_launch(s.nx, s.ny, s.nz, 1 << 16);
    if (l == 1) {
      GMG_LAUNCH(c, "faces_from_cells", k_faces_from_cells, lc, c->a, f.geom(), wsp<double>(c, o.wx64),
                 wsp<double>(c, o.wy64), wsp<double>(c, o.wz64), wsp<double>(c, o.tp64), lc.kc);
    } else {
      const LevelOffsets& p = L.lv[l - 1];
      GMG_LAUNCH(c, "coarsen_faces", k_coarsen_faces, lc, wsp<double>(c, p.wx64), wsp<double>(c, p.wy64),
                 wsp<double>(c, p.wz64), wsp<double>(c, p.tp64), f.geom(), wsp<double>(c, o.wx64),
                 wsp<double>(c, o.wy64), wsp<double>(c, o.wz64), wsp<double>(c, o.tp64), lc.kc);
    }
    if (c->mixed) {
      const size_t n = s.n(), nxy = (size_t)s.nx * s.ny;
      const Launch fl = flat_launch(n);
      GMG_LAUNCH(c, "convert_f64_f32", (k_convert<float, double>), fl, wsp<double>(c, o.wx64),
                 wsp<float>(c, o.wx), n);
      GMG_LAUNCH(c, "convert_f64_f32", (k_convert<float, double>), fl, wsp<double>(c, o.wy64),
                 wsp<float>(c, o.wy), n);
      GMG_LAUNCH(c, "convert_f64_f32", (k_convert<float, double>), fl, wsp<double>(c, o.wz64),
                 wsp<float>(c, o.wz), n);
      GMG_LAUNCH(c, "convert_f64_f32", (k_convert<float, double>), flat_launch(nxy), wsp<double>(c, o.tp64),
                 wsp<float>(c, o.tp), nxy);
    }
  }
  // coarsest level: dense matrix on the host, Cholesky inverse, upload
  const LevelShape& s = L.shapes.back();
  const int n = (int)s.n();
  std::vector<double> wx, wy, wz, tp, afine, M;
  if (nl == 1) {
    afine.resize(n);
    note(c, hipMemcpyAsync(afine.data(), c->a, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  } else {
    const LevelOffsets& o = L.lv[nl - 1];
    const size_t nxy = (size_t)s.nx * s.ny;
    wx.resize(n);
    wy.resize(n);
    wz.resize(n);
    tp.resize(nxy);
    note(c, hipMemcpyAsync(wx.data(), wsp<double>(c, o.wx64), (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    note(c, hipMemcpyAsync(wy.data(), wsp<double>(c, o.wy64), (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    note(c, hipMemcpyAsync(wz.data(), wsp<double>(c, o.wz64), (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    note(c, hipMemcpyAsync(tp.data(), wsp<double>(c, o.tp64), nxy * 8, hipMemcpyDeviceToHost, c->stream));
  }
  note(c, hipStreamSynchronize(c->stream));
  if (c->err != hipSuccess) return GMG_ERR_HIP;
  assemble_coarsest(s, wx, wy, wz, tp, afine.data(), nl == 1, M);
  if (n > GJ_MIN_CELLS) return gpu_inverse(c, M, n);
  if (!spd_inverse(M, n)) return GMG_ERR_NONFINITE;
  if (c->mixed) {
    std::vector<float> Mf(M.begin(), M.end());
    note(c, hipMemcpyAsync(wsp<float>(c, L.cinv), Mf.data(), Mf.size() * 4, hipMemcpyHostToDevice, c->stream));
    note(c, hipStreamSynchronize(c->stream));
  } else {
    note(c, hipMemcpyAsync(wsp<double>(c, L.cinv), M.data(), M.size() * 8, hipMemcpyHostToDevice, c->stream));
    note(c, hipStreamSynchronize(c->stream));
  }
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

// ---------------------------------------------------------------------------
// V-cycle (Sec. 3.2): zero initial guess, red-black symmetric Gauss-Seidel.
// ---------------------------------------------------------------------------

template <typename T>
FaceCoef<T> face_coef(gmg_ctx* c, int l) {
  const LevelOffsets& o = c->L.lv[l];
  return FaceCoef<T>{wsp<T>(c, o.wx), wsp<T>(c, o.wy), wsp<T>(c, o.wz), wsp<T>(c, o.tp)};
}

// Profile name of a kernel: base + level ("fine" for level 0, "L<l>" for a
// coarser one, "coarsest") + precision (the returned string lives as long as
// the process).
const char* kname(const char* base, int level, size_t tsize) {
  static std::map<std::string, std::string> names;
  const std::string lv = level == 0 ? "_fine" : (level < 0 ? "_coarsest" : "_L" + std::to_string(level));
  std::string key = std::string(base) + lv + (tsize == 4 ? "_f32" : "_f64");
  auto it = names.find(key);
  if (it == names.end()) it = names.emplace(key, key).first;
  return it->second.c_str();
}

// A z-marching launch with fewer blocks than this is latency-bound (a small
// level): each loop trip of a block waits for its own loads, so there every
// block marches a single trip of planes instead of min_kc planes.
constexpr long long SMALL_GRID_BLOCKS = 1024;

// z-chunk of a marching launch over nz planes with `cols` blocks per chunk
// column: kc, or the kernel's planes per loop trip on a small grid.
inline int small_grid_kc(int nz, long long cols, int kc, int trip) {
  if (trip > 0 && cols * ((nz + kc - 1) / kc) < SMALL_GRID_BLOCKS) kc = trip;
  return std::min(kc, nz);
}

// Launch of the lane-pair z-marching kernels over an nx x ny x nz grid (nx
// even): one lane per x-pair, rows of BY threads, z-chunks of kc planes with
// kc >= min_kc, about `target` blocks; on a small grid, `trip` planes (the
// kernel's planes per loop trip; 0: keep min_kc).
Launch pair_launch(int nx, int ny, int nz, long long target, int min_kc, int trip = 0) {
  const int gx = (nx / 2 + BX - 1) / BX, gy = (ny + BY - 1) / BY;
  const long long cols = (long long)gx * gy;
  int kc = (int)std::max<long long>(min_kc, (nz * cols + target - 1) / target);
  kc = small_grid_kc(nz, cols, std::min(kc, nz), trip);
  return Launch{dim3(gx, gy, (nz + kc - 1) / kc), dim3(BX, BY, 1), kc};
}

// z-chunk of a column-marching launch with `cols` blocks per chunk column
// and `resident` blocks running at once: the chunk (at least min_kc planes)
// that minimises the rounds of blocks times the planes a block marches (its
// chunk plus `extra`), the smallest chunk for each chunk count, among
// chunks that give at least min_rounds rounds when any does.  (A round
// with few blocks leaves most CUs idle: at level 1 of the 512^3 grid,
// 11-plane chunks made 1032 blocks of one per CU, 4.03 rounds on 256 CUs;
// 24-plane chunks, 473 blocks in 2 rounds, took 110.5 us per sweep against
// 137.8.  The finest level's fused sweep was slower in 3 long rounds than
// in 8 short ones, 563 against 507 us, at the same modelled cost: it keeps
// at least 4.)
inline int rounds_kc(int nz, long long cols, long long resident, int min_kc, int extra, int min_rounds = 1) {
  int best = std::min(nz, min_kc), best_any = best;
  double best_cost = 1e300, best_cost_any = 1e300;
  for (int kc = std::min(nz, min_kc); kc <= nz; ++kc) {
    const long long gz = (nz + kc - 1) / kc;
    if (kc > 1 && kc > min_kc && (nz + kc - 2) / (kc - 1) == gz) continue;  // a smaller chunk gives the same count
    const long long rounds = (cols * gz + resident - 1) / resident;
    const double cost = (double)rounds * (kc + extra);
    if (cost < best_cost_any) {
      best_cost_any = cost;
      best_any = kc;
    }
    if (rounds >= min_rounds && cost < best_cost) {
      best_cost = cost;
      best = kc;
    }
  }
  return best_cost < 1e300 ? best : best_any;
}

// Waves per row of the coarse levels' fused sweep (a block spans the row),
// and the most a precision allows: a block has 16 (float32) or 8 (float64)
// waves, two of its rows are a halo, and at least one row must own cells.
inline int face_waves(const LevelShape& s) { return (s.nx / 2 + 63) / 64; }
template <typename T>
constexpr int FACE_MAX_WAVES = sizeof(T) == 4 ? 4 : 2;

// Fused symmetric sweeps on coarse level l (k_sym_face): red-black Gauss-
// Seidel with both smoothing phases, rows of at most 256 pairs in float32
// and 128 in float64 (a block spans the row: with two waves 8 rows in
// float32 and 4 in float64, of which 6 and 2 own cells; float64 at 256^3:
// 258 us per sweep against 2 x 163 us for the half-sweeps); on request, or
// by default on levels of at least 128^3 cells.  They read the face coefficients once per
// sweep instead of twice; on smaller levels, where a sweep is latency-bound,
// the fused kernel takes as long as the two half-sweep kernels it replaces
// (kernel trace of 256^3 solves: 12.2 us against 2 x 5.7 us at 64^3 and
// below), and fewer launches did not shorten the solves (with z-chunks of
// one or two planes there, 10.3 us per fused sweep, the 64^3 mixed step
// took 3.71 ms against 3.49 and the 512^3 one 87.8 against 87.0).
template <typename T>
bool fused_face(gmg_ctx* c, int l) {
  const LevelShape& s = c->L.shapes[l];
  const int fs = c->opt.fine_sweep;
  return c->opt.smoother == GMG_SMOOTH_RBGS && c->opt.nu_pre >= 1 && c->opt.nu_post >= 1 && l >= 1 &&
         l < (int)c->L.shapes.size() - 1 && face_waves(s) <= FACE_MAX_WAVES<T> &&
         (fs == GMG_SWEEP_FUSED || (fs == GMG_SWEEP_AUTO && s.n() >= ((size_t)1 << 21)));
}

// One fused symmetric sweep on coarse level l: colour c1 from Xin into Xout,
// then the other colour from the new values (FIRST: from x = 0, Xin unused).
// A block spans the row (one to four waves) and FaceSymShape's rows; z-chunks
// of at least 8 planes from the rounds model (rounds_kc).
template <typename T, bool FIRST>
void sym_face(gmg_ctx* c, int l, const T* Xin, T* Xout, const T* b, const FaceCoef<T>& co, int c1) {
  const LevelShape& s = c->L.shapes[l];
  const char* nm = kname(FIRST ? "sym_first" : "sym", l, sizeof(T));
  auto go = [&](auto wc) {
    constexpr int WX = decltype(wc)::value, R = FaceSymShape<T, WX>::R, iy = FaceSymShape<T, WX>::IY;
    const int gy = (s.ny + iy - 1) / iy;
    // blocks of the kernel resident on one CU (one, for these 16- and 8-wave
    // blocks and their registers), asked once
    static const int per_cu = [] {
      int nb = 0;
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sym_face<T, FIRST, WX>, 64 * WX * R, 0) ==
                         hipSuccess &&
                     nb > 0
                 ? nb
                 : 1;
    }();
    const int kc = rounds_kc(s.nz, gy, (long long)per_cu * c->cus, 8, 2);
    const Launch fl{dim3(1, gy, (s.nz + kc - 1) / kc), dim3(64 * WX, R, 1), kc};
    GMG_LAUNCH(c, nm, (k_sym_face<T, FIRST, WX>), fl, Xin, Xout, b, co, s.geom(), kc, c1);
  };
  switch (face_waves(s)) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    default:
      if constexpr (FACE_MAX_WAVES<T> >= 4) {
        if (face_waves(s) == 3)
          go(std::integral_constant<int, 3>{});
        else
          go(std::integral_constant<int, 4>{});
      }
  }
}

// Coarse level l (not the coarsest, so every dimension is even): red-black
// smoothing, residual and restriction with the lane-pair kernels on the
// stored face coefficients.
// From x = 0, or from the guess in x when from_x.
template <typename T>
void smooth_pre_face(gmg_ctx* c, int l, T* x, const T* b, const FaceCoef<T>& co, bool from_x) {
  const LevelShape& s = c->L.shapes[l];
  const Geom g = s.geom();
  const int nu = c->opt.nu_pre;
  if (nu == 0) {
    if (!from_x) {
      const Launch fl = flat_launch(s.n());
      GMG_LAUNCH(c, kname("fill", l, sizeof(T)), k_fill<T>, fl, x, T(0), s.n());
    }
    return;
  }
  const Launch pl = pair_launch(s.nx, s.ny, s.nz, 4096, 4, 2);
  if (from_x)
    GMG_LAUNCH(c, kname("gs", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, x, b, co, g, pl.kc, 0);
  else
    GMG_LAUNCH(c, kname("gs_first", l, sizeof(T)), (k_gs_pair_face<T, true>), pl, x, b, co, g, pl.kc, 0);
  GMG_LAUNCH(c, kname("gs", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, x, b, co, g, pl.kc, 1);
  for (int it = 1; it < nu; ++it) {
    GMG_LAUNCH(c, kname("gs", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, x, b, co, g, pl.kc, 0);
    GMG_LAUNCH(c, kname("gs", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, x, b, co, g, pl.kc, 1);
  }
}

template <typename T>
void smooth_post_face(gmg_ctx* c, int l, T* x, const T* b, const FaceCoef<T>& co) {
  const LevelShape& s = c->L.shapes[l];
  const Launch pl = pair_launch(s.nx, s.ny, s.nz, 4096, 4, 2);
  for (int it = 0; it < c->opt.nu_post; ++it) {
    GMG_LAUNCH(c, kname("gs", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, x, b, co, s.geom(), pl.kc, 1);
    GMG_LAUNCH(c, kname("gs", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, x, b, co, s.geom(), pl.kc, 0);
  }
}

// Launch of k_restrict_fw: one thread per coarse cell of fine level s.
Launch fw_launch(const LevelShape& s) {
  return Launch{dim3((s.nx / 2 + BX - 1) / BX, (s.ny / 2 + BY - 1) / BY, s.nz / 2), dim3(BX, BY, 1), 0};
}

template <typename T>
void resid_restrict_face(gmg_ctx* c, int l, const T* x, const T* b, const FaceCoef<T>& co, T* bc) {
  const LevelShape& s = c->L.shapes[l];
  if (c->opt.restriction == GMG_RESTRICT_TRANSPOSE) {
    // r = b - A x into the residual scratch, then bc = P^T r / 8
    T* r = wsp<T>(c, c->L.rr);
    const Launch cl = cell_launch(s.nx, s.ny, s.nz, 4096, 4);
    GMG_LAUNCH(c, kname("resid", l, sizeof(T)), k_resid_face<T>, cl, x, b, co, s.geom(), r, cl.kc);
    GMG_LAUNCH(c, kname("restrict_fw", l, sizeof(T)), (k_restrict_fw<T, T>), fw_launch(s), (const T*)r, bc,
               s.geom());
    return;
  }
  const Launch pl = pair_launch(s.nx, s.ny, s.nz / 2, 4096, 2, 1);
  GMG_LAUNCH(c, kname("resid_restrict", l, sizeof(T)), k_resid_restrict_face<T>, pl, x, b, co, s.geom(), bc,
             pl.kc);
}

// Finest level (colour-split X and B, right side s u): residual and
// restriction into the level-1 right side.  Transpose restriction: r = s u -
// A x in float64 (natural layout), then P^T r / 8.
template <typename T>
void resid_restrict_fine(gmg_ctx* c, const T* X, const T* B, const double* u, const double* bscale, const T* a) {
  const LevelShape& s = c->L.shapes[0];
  T* bc = wsp<T>(c, c->L.lv[1].b);
  if (c->opt.restriction == GMG_RESTRICT_TRANSPOSE) {
    double* r = wsp<double>(c, c->L.rr);
    const Launch rl = pair_launch(s.nx, s.ny, s.nz, 8192, 8);
    GMG_LAUNCH(c, kname("resid", 0, sizeof(T)), k_resid_split<T>, rl, X, u, bscale, a, s.geom(), c->L.hn, r,
               rl.kc);
    GMG_LAUNCH(c, kname("restrict_fw", 0, sizeof(T)), (k_restrict_fw<double, T>), fw_launch(s), (const double*)r,
               bc, s.geom());
    return;
  }
  const Launch l = pair_launch(s.nx, s.ny, s.nz / 2, 8192, 4, 1);
  GMG_LAUNCH(c, kname("resid_restrict", 0, sizeof(T)), k_resid_restrict_split<T>, l, X, B, a, s.geom(), c->L.hn,
             bc, l.kc);
}

// Levels >= 1 that are not the coarsest (every dimension even): x += P xc,
// or x = xin + P xc when xin is given (another buffer).
template <typename T>
void prolong_add(gmg_ctx* c, int l, T* x, const T* xc, const T* xin = nullptr) {
  const LevelShape& s = c->L.shapes[l];
  const Launch pl = pair_launch(s.nx, s.ny, s.nz / 2, 4096, 2, 1);
  GMG_LAUNCH(c, kname("prolong_add", l, sizeof(T)), (k_prolong_pair<T, false>), pl, x, xc, s.geom(), (size_t)0, 0,
             pl.kc, xin);
}

// Levels >= 1: x = P xc, the interpolated guess of a full multigrid cycle.
template <typename T>
void prolong_set(gmg_ctx* c, int l, T* x, const T* xc) {
  const LevelShape& s = c->L.shapes[l];
  const Launch pl = pair_launch(s.nx, s.ny, s.nz / 2, 4096, 2, 1);
  GMG_LAUNCH(c, kname("prolong_set", l, sizeof(T)), (k_prolong_pair<T, false, true>), pl, x, xc, s.geom(),
             (size_t)0, 0, pl.kc, (const T*)nullptr);
}

// Levels >= 1: right side of level l+1 = mean of the 8 children of level l's.
template <typename T>
void restrict_mean(gmg_ctx* c, int l) {
  const LevelShape& s = c->L.shapes[l];
  const Launch rl{dim3((s.nx / 2 + BX - 1) / BX, (s.ny / 2 + BY - 1) / BY, s.nz / 2), dim3(BX, BY, 1), 0};
  GMG_LAUNCH(c, kname("restrict", l, sizeof(T)), k_restrict_mean<T>, rl, wsp<const T>(c, c->L.lv[l].b),
             wsp<T>(c, c->L.lv[l + 1].b), s.geom());
}

template <typename T>
void coarse_solve(gmg_ctx* c, const T* b, T* x) {
  const int n = c->nc;
  const Launch lc{dim3((n + NTHREADS - 1) / NTHREADS), dim3(BX, BY, 1), 0};
  GMG_LAUNCH(c, kname("coarse_solve", -1, sizeof(T)), k_coarse_solve<T>, lc,
             wsp<const T>(c, c->L.cinv), b, x, n);
}

// The levels from l0 down to the coarsest in one workgroup (k_vcycle_bottom):
// a V-cycle, or the full multigrid cycle over those levels when fmg; its
// arguments were written to the workspace at set-up.
template <typename T>
void vcycle_bottom(gmg_ctx* c, int fmg) {
  const Launch one{dim3(1), dim3(BottomThreads<T>::value, 1, 1), 0};
  if (fmg)
    GMG_LAUNCH(c, kname("fmg_bottom", c->bottom_from, sizeof(T)), (k_vcycle_bottom<T, true>), one,
               wsp<const BottomArgs<T>>(c, c->L.bargs));
  else
    GMG_LAUNCH(c, kname("vcycle_bottom", c->bottom_from, sizeof(T)), (k_vcycle_bottom<T, false>), one,
               wsp<const BottomArgs<T>>(c, c->L.bargs));
}

// Arguments of the bottom kernel (fixed for the life of the context).
template <typename T>
int write_bottom_args(gmg_ctx* c) {
  const int nl = (int)c->L.shapes.size(), l0 = c->bottom_from;
  if (l0 < 0) return GMG_OK;
  BottomArgs<T> A{};
  A.nlev = nl - l0;
  int coff = 0, tpoff = 0;
  for (int q = 0; q < A.nlev; ++q) {
    const int l = l0 + q;
    const LevelShape& s = c->L.shapes[l];
    A.co[q] = face_coef<T>(c, l);
    A.g[q] = s.geom();
    A.coff[q] = coff;
    A.tpoff[q] = tpoff;
    coff += (int)s.n();
    tpoff += s.nx * s.ny;
  }
  if (coff > BOTTOM_LDS_CELLS || tpoff > BOTTOM_LDS_CELLS) return GMG_ERR_SHAPE;
  A.x0 = wsp<T>(c, c->L.lv[l0].x);
  A.b0 = wsp<T>(c, c->L.lv[l0].b);
  A.Ainv = wsp<const T>(c, c->L.cinv);
  A.nu_pre = c->opt.nu_pre;
  A.nu_post = c->opt.nu_post;
  note(c, hipMemcpyAsync(wsp<BottomArgs<T>>(c, c->L.bargs), &A, sizeof(A), hipMemcpyHostToDevice, c->stream));
  note(c, hipStreamSynchronize(c->stream));
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

// Chebyshev smoothing (Sec. 3.2, eq. qntn) on a coarse level l: nu
// applications of the degree-CHEB_DEGREE recurrence, each step one SSOR
// solve (red from zero, black, red) of the residual and the update of the
// direction d and the iterate x.  From x = 0 unless from_x (the first
// residual is then b itself).
template <typename T>
void cheb_smooth_face(gmg_ctx* c, int l, T* x, const T* b, const FaceCoef<T>& co, bool from_x, int nu) {
  const LevelShape& s = c->L.shapes[l];
  const LevelOffsets& o = c->L.lv[l];
  T* R = wsp<T>(c, o.cr);
  T* E = wsp<T>(c, o.ce);
  T* D = wsp<T>(c, o.cd);
  const Geom g = s.geom();
  const size_t n = s.n();
  const Launch pl = pair_launch(s.nx, s.ny, s.nz, 4096, 4);
  const Launch cl = cell_launch(s.nx, s.ny, s.nz, 4096, 4);
  const Launch ul = flat_launch(n);
  const auto& cf = c->cheb_coef[l];
  if (nu == 0 && !from_x) GMG_LAUNCH(c, kname("fill", l, sizeof(T)), k_fill<T>, ul, x, T(0), n);
  bool zero = !from_x;
  for (int it = 0; it < nu; ++it) {
    for (int st = 0; st < CHEB_DEGREE; ++st) {
      const bool first = zero && st == 0;
      const T* rhs = b;
      if (!first) {
        GMG_LAUNCH(c, kname("cheb_resid", l, sizeof(T)), k_resid_face<T>, cl, (const T*)x, b, co, g, R, cl.kc);
        rhs = R;
      }
      GMG_LAUNCH(c, kname("ssor_first", l, sizeof(T)), (k_gs_pair_face<T, true>), pl, E, rhs, co, g, pl.kc, 0);
      GMG_LAUNCH(c, kname("ssor", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, E, rhs, co, g, pl.kc, 1);
      GMG_LAUNCH(c, kname("ssor", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, E, rhs, co, g, pl.kc, 0);
      const int mode = (st == 0 ? 1 : 0) | (first ? 2 : 0);
      GMG_LAUNCH(c, kname("cheb_update", l, sizeof(T)), k_cheb_update<T>, ul, x, D, (const T*)E, cf[2 * st],
                 cf[2 * st + 1], n, (size_t)0, mode);
    }
    zero = false;
  }
}

// Levels >= 1 (face coefficients), right side in lv[l].b, result in lv[l].x:
// a V-cycle from x = 0, or from the guess in lv[l].x when from_x (the
// coarsest level is solved directly either way; a guess is never passed to
// the bottom kernel's first level).
template <typename T>
void vcycle_coarse(gmg_ctx* c, int l, bool from_x = false) {
  const int nl = (int)c->L.shapes.size();
  const LevelOffsets& o = c->L.lv[l];
  T* x = wsp<T>(c, o.x);
  const T* b = wsp<T>(c, o.b);
  if (l == nl - 1) {
    coarse_solve<T>(c, b, x);
    return;
  }
  if (l == c->bottom_from) {
    vcycle_bottom<T>(c, 0);
    return;
  }
  const FaceCoef<T> co = face_coef<T>(c, l);
  if (fused_face<T>(c, l)) {
    // the sweeps ping-pong between x and x2; the first buffer (from zero)
    // or an out-of-place prolongation (from the guess in x) makes the last
    // one land in x
    T* X[2] = {x, wsp<T>(c, o.x2)};
    const int npre = c->opt.nu_pre, npost = c->opt.nu_post, L = npre + npost;
    int cur = 0;
    if (from_x) {
      for (int it = 0; it < npre; ++it, cur ^= 1) sym_face<T, false>(c, l, X[cur], X[cur ^ 1], b, co, 0);
    } else {
      cur = (L - 1) & 1;
      sym_face<T, true>(c, l, nullptr, X[cur], b, co, 0);
      for (int it = 1; it < npre; ++it, cur ^= 1) sym_face<T, false>(c, l, X[cur], X[cur ^ 1], b, co, 0);
    }
    resid_restrict_face<T>(c, l, X[cur], b, co, wsp<T>(c, c->L.lv[l + 1].b));
    vcycle_coarse<T>(c, l + 1);
    const T* xc = wsp<T>(c, c->L.lv[l + 1].x);
    if (from_x && (L & 1)) {
      prolong_add<T>(c, l, X[cur ^ 1], xc, X[cur]);
      cur ^= 1;
    } else {
      prolong_add<T>(c, l, X[cur], xc);
    }
    for (int it = 0; it < npost; ++it, cur ^= 1) sym_face<T, false>(c, l, X[cur], X[cur ^ 1], b, co, 1);
    return;
  }
  const bool cheb = c->opt.smoother == GMG_SMOOTH_CHEBYSHEV;
  if (cheb)
    cheb_smooth_face<T>(c, l, x, b, co, from_x, c->opt.nu_pre);
  else
    smooth_pre_face<T>(c, l, x, b, co, from_x);
  resid_restrict_face<T>(c, l, x, b, co, wsp<T>(c, c->L.lv[l + 1].b));
  vcycle_coarse<T>(c, l + 1);
  prolong_add<T>(c, l, x, wsp<T>(c, c->L.lv[l + 1].x));
  if (cheb)
    cheb_smooth_face<T>(c, l, x, b, co, true, c->opt.nu_post);
  else
    smooth_post_face<T>(c, l, x, b, co);
}

// Full multigrid cycle on the levels >= l0 for the right side in lv[l0].b,
// result in lv[l0].x: right sides restricted down to the bottom kernel's
// first level (or the coarsest), the bottom kernel's full multigrid cycle
// over its levels (or the direct solve), then level by level upwards the
// interpolated coarser result as the guess of one V-cycle.
template <typename T>
void fmg_coarse(gmg_ctx* c, int l0) {
  const int nl = (int)c->L.shapes.size();
  const int lb = c->bottom_from >= 0 ? c->bottom_from : nl - 1;
  for (int l = l0; l < lb; ++l) restrict_mean<T>(c, l);
  if (c->bottom_from >= 0)
    vcycle_bottom<T>(c, 1);
  else
    coarse_solve<T>(c, wsp<const T>(c, c->L.lv[nl - 1].b), wsp<T>(c, c->L.lv[nl - 1].x));
  for (int l = lb - 1; l >= l0; --l) {
    prolong_set<T>(c, l, wsp<T>(c, c->L.lv[l].x), wsp<const T>(c, c->L.lv[l + 1].x));
    vcycle_coarse<T>(c, l, true);
  }
}

// Finest level on colour-split storage (at least two levels, so every
// dimension is even).  X and B are colour-split (colour c at offset c * hn).
template <typename T, bool FIRST>
void gs_split(gmg_ctx* c, T* X, T* B, const double* u, const double* bscale, const T* a, int colour) {
  const LevelShape& s = c->L.shapes[0];
  // about 8192 * 256 threads, z-chunks of at least 8 planes
  const int gx = (s.nx / 2 + BX - 1) / BX, gy = (s.ny + GS_ROWS - 1) / GS_ROWS;
  const long long target = 8192LL * BY / GS_ROWS;
  int kc = (int)std::max<long long>(8, (s.nz * (long long)gx * gy + target - 1) / target);
  kc = small_grid_kc(s.nz, (long long)gx * gy, std::min(kc, s.nz), SPLIT_BATCH);
  const Launch l{dim3(gx, gy, (s.nz + kc - 1) / kc), dim3(BX, GS_ROWS, 1), kc};
  const char* nm = kname(FIRST ? "gs_first" : "gs", 0, sizeof(T));
  if (FIRST && bscale)
    GMG_LAUNCH(c, nm, (k_gs_split<T, FIRST, true>), l, X, B, u, bscale, a, s.geom(), c->L.hn, l.kc, colour);
  else
    GMG_LAUNCH(c, nm, (k_gs_split<T, FIRST, false>), l, X, B, u, bscale, a, s.geom(), c->L.hn, l.kc, colour);
}

// z = M (s * u), z colour-split: pre-smoothing red, black (nu_pre times)
// from x = 0, the first red half-sweep writing the right side B; residual
// and restriction; coarse correction (added to the red cells only when a
// black half-sweep follows, which overwrites the black cells without reading
// them); post-smoothing black, red (nu_post times).
// from_x: B already holds the right side and X the guess (both colours).
template <typename T>
void vcycle_fine_split(gmg_ctx* c, const double* u, const double* bscale, T* X, bool from_x) {
  const LevelShape& s = c->L.shapes[0];
  const T* a = c->mixed ? (const T*)wsp<float>(c, c->L.a32) : (const T*)c->a;
  T* B = wsp<T>(c, c->L.b0);
  const size_t hn = c->L.hn;
  const int npre = c->opt.nu_pre, npost = c->opt.nu_post;
  if (!from_x) {
    gs_split<T, true>(c, X, B, u, bscale, a, 0);
    if (npre == 0) {  // no pre-smoothing: x = 0 (B is kept)
      const Launch fl = flat_launch(2 * hn);
      GMG_LAUNCH(c, kname("fill", 0, sizeof(T)), k_fill<T>, fl, X, T(0), 2 * hn);
    }
  }
  for (int it = 0; it < npre; ++it) {
    if (it > 0 || from_x) gs_split<T, false>(c, X, B, nullptr, nullptr, a, 0);
    gs_split<T, false>(c, X, B, nullptr, nullptr, a, 1);
  }
  resid_restrict_fine<T>(c, X, B, u, bscale, a);
  vcycle_coarse<T>(c, 1);
  {
    const Launch l = pair_launch(s.nx, s.ny, s.nz / 2, 8192, 4, 1);
    GMG_LAUNCH(c, kname("prolong_add", 0, sizeof(T)), (k_prolong_pair<T, true>), l, X,
               (const T*)wsp<T>(c, c->L.lv[1].x), s.geom(), hn, npost > 0 ? 1 : 3, l.kc,
               (const T*)nullptr);
  }
  for (int it = 0; it < npost; ++it) {
    gs_split<T, false>(c, X, B, nullptr, nullptr, a, 1);
    gs_split<T, false>(c, X, B, nullptr, nullptr, a, 0);
  }
}

// z = M (s * u) with the Chebyshev smoother on the finest level (at least
// two levels).  X (colour-split) is the iterate; the SSOR solves write their
// colour-split right side into the b0 scratch and their result into the xs
// scratch; residuals are float64 in the natural layout, where the first
// SSOR half-sweep reads them.  The first residual of the pre-smoothing is
// s u itself.
template <typename T>
void vcycle_fine_cheb(gmg_ctx* c, const double* u, const double* bscale, T* X) {
  const LevelShape& s = c->L.shapes[0];
  const T* a = c->mixed ? (const T*)wsp<float>(c, c->L.a32) : (const T*)c->a;
  T* Bs = wsp<T>(c, c->L.b0);
  T* E = wsp<T>(c, c->L.xs);
  T* D = wsp<T>(c, c->L.cd0);
  double* R = wsp<double>(c, c->L.cr0);
  const size_t hn = c->L.hn, half = c->N / 2;
  const Geom g = s.geom();
  const Launch rl = pair_launch(s.nx, s.ny, s.nz, 8192, 8);
  Launch ul = flat_launch(half);
  ul.grid.y = 2;  // the two colour arrays
  const auto& cf = c->cheb_coef[0];
  auto resid = [&]() {
    GMG_LAUNCH(c, kname("cheb_resid", 0, sizeof(T)), k_resid_split<T>, rl, (const T*)X, u, bscale, a, g, hn, R,
               rl.kc);
  };
  auto smooth = [&](bool zero, int nu) {
    if (nu == 0 && zero) {
      const Launch fl = flat_launch(2 * hn);
      GMG_LAUNCH(c, kname("fill", 0, sizeof(T)), k_fill<T>, fl, X, T(0), 2 * hn);
    }
    for (int it = 0; it < nu; ++it) {
      for (int st = 0; st < CHEB_DEGREE; ++st) {
        const bool first = zero && st == 0;
        if (first) {
          gs_split<T, true>(c, E, Bs, u, bscale, a, 0);
        } else {
          resid();
          gs_split<T, true>(c, E, Bs, R, nullptr, a, 0);
        }
        gs_split<T, false>(c, E, Bs, nullptr, nullptr, a, 1);
        gs_split<T, false>(c, E, Bs, nullptr, nullptr, a, 0);
        const int mode = (st == 0 ? 1 : 0) | (first ? 2 : 0);
        GMG_LAUNCH(c, kname("cheb_update", 0, sizeof(T)), k_cheb_update<T>, ul, X, D, (const T*)E, cf[2 * st],
                   cf[2 * st + 1], half, hn, mode);
      }
      zero = false;
    }
  };
  smooth(true, c->opt.nu_pre);
  resid();
  {
    const Launch l{dim3((s.nx / 2 + BX - 1) / BX, (s.ny / 2 + BY - 1) / BY, s.nz / 2), dim3(BX, BY, 1), 0};
    GMG_LAUNCH(c, kname("restrict_rhs", 0, sizeof(T)), k_restrict_split_rhs<T>, l, (const double*)R, nullptr, Bs,
               wsp<T>(c, c->L.lv[1].b), g, hn);
  }
  vcycle_coarse<T>(c, 1);
  {
    const Launch l = pair_launch(s.nx, s.ny, s.nz / 2, 8192, 4, 1);
    GMG_LAUNCH(c, kname("prolong_add", 0, sizeof(T)), (k_prolong_pair<T, true>), l, X,
               (const T*)wsp<T>(c, c->L.lv[1].x), g, hn, 3, l.kc, (const T*)nullptr);
  }
  smooth(false, c->opt.nu_post);
}

// Planes of the largest array a block of the fused sweep may address (the
// natural-layout float64 u and a: 16 bytes per pair and plane) within the
// 2^31 bytes of its 32-bit buffer offsets.
inline long long sym_max_planes(const LevelShape& s) {
  return (1LL << 31) / (16LL * (s.nx / 2) * s.ny);
}

// Launch of the fused symmetric sweep on the finest level: blocks of 64 x R
// threads, about 2048 * 1024 threads in all, z-chunks of at least 8 planes
// (even with the fused residual restriction: a chunk holds whole coarse
// planes) and at most sym_max_planes - 8 (a block reads up to three planes
// below its chunk and four above).
template <typename T, bool RESID = false>
int sym_default_kc(const LevelShape& s) {
  using S = SymShape<T, RESID>;
  const int gx = (s.nx / 2 + S::IX - 1) / S::IX, gy = (s.ny + S::IY - 1) / S::IY;
  const long long target = 2048LL * 1024 / (S::SX * S::R);
  return (int)std::min<long long>(s.nz, std::max<long long>(8, (s.nz * (long long)gx * gy + target - 1) / target));
}
// The launch takes the chunk from the rounds model (rounds_kc) over the
// blocks resident at once; `resident` = 0 keeps sym_default_kc.
template <typename T, bool RESID = false>
Launch sym_launch(const LevelShape& s, long long resident = 0) {
  using S = SymShape<T, RESID>;
  const int gx = (s.nx / 2 + S::IX - 1) / S::IX, gy = (s.ny + S::IY - 1) / S::IY;
  long long kc = resident > 0 ? rounds_kc(s.nz, (long long)gx * gy, resident, 8, RESID ? 3 : 2, 4)
                              : sym_default_kc<T, RESID>(s);
  kc = std::min<long long>({kc, s.nz, std::max<long long>(1, sym_max_planes(s) - 8)});
  if (RESID) kc = std::max<long long>(2, kc & ~1LL);
  return Launch{dim3(gx, gy, (unsigned)((s.nz + kc - 1) / kc)), dim3(S::SX, S::R, 1), (int)kc};
}

// Blocks of k_sym_split resident on one CU (asked once per instantiation).
template <typename T, bool FIRST, bool SCALED, bool RESID>
int sym_blocks_per_cu() {
  static const int nb = [] {
    int n = 0;
    using S = SymShape<T, RESID>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sym_split<T, FIRST, SCALED, RESID>, S::SX * S::R, 0) ==
                       hipSuccess &&
                   n > 0
               ? n
               : 1;
  }();
  return nb;
}

// One fused symmetric sweep (k_sym_split) on the finest level: colour c1
// from Xin into Xout, then the other colour from the new values.  RESID
// (not FIRST): also the residual of the result, restricted to level 1's
// right side bc (what resid_restrict_fine computes).
template <typename T, bool FIRST, bool RESID = false>
void sym_split(gmg_ctx* c, const T* Xin, T* Xout, T* B, const double* u, const double* bscale, const T* a,
               int c1, T* bc = nullptr) {
  const LevelShape& s = c->L.shapes[0];
  const char* nm = kname(RESID ? "sym_resid" : (FIRST ? "sym_first" : "sym"), 0, sizeof(T));
  if constexpr (RESID) {
    static_assert(!FIRST, "the residual is fused into a sweep from a guess only");
    const Launch l = sym_launch<T, true>(s, (long long)sym_blocks_per_cu<T, false, false, true>() * c->cus);
    GMG_LAUNCH(c, nm, (k_sym_split<T, false, false, true>), l, Xin, Xout, B, u, bscale, a, s.geom(), c->L.hn,
               l.kc, c1, bc);
  } else if (FIRST && bscale) {
    const Launch l = sym_launch<T, false>(s, (long long)sym_blocks_per_cu<T, FIRST, true, false>() * c->cus);
    GMG_LAUNCH(c, nm, (k_sym_split<T, FIRST, true, false>), l, Xin, Xout, B, u, bscale, a, s.geom(), c->L.hn,
               l.kc, c1, bc);
  } else {
    const Launch l = sym_launch<T, false>(s, (long long)sym_blocks_per_cu<T, FIRST, false, false>() * c->cus);
    GMG_LAUNCH(c, nm, (k_sym_split<T, FIRST, false, false>), l, Xin, Xout, B, u, bscale, a, s.geom(), c->L.hn,
               l.kc, c1, bc);
  }
}

// Buffer of sweep p (1-based; p = 0 the guess) of vcycle_fine_sym: the
// sweeps ping-pong between the scratch iterate and z so that the last one
// lands in z.
template <typename T>
T* sym_buffer(gmg_ctx* c, T* Z, int p) {
  const int L = c->opt.nu_pre + c->opt.nu_post;
  return ((L - p) % 2 == 0) ? Z : wsp<T>(c, c->L.xs);
}

// z = M (s * u) with fused symmetric sweeps (nu_pre, nu_post >= 1).  Same
// arithmetic as vcycle_fine_split.  from_x: B already holds the right side
// and sym_buffer(c, Z, 0) the guess.
template <typename T>
void vcycle_fine_sym(gmg_ctx* c, const double* u, const double* bscale, T* Z, bool from_x) {
  const LevelShape& s = c->L.shapes[0];
  const T* a = c->mixed ? (const T*)wsp<float>(c, c->L.a32) : (const T*)c->a;
  T* B = wsp<T>(c, c->L.b0);
  const size_t hn = c->L.hn;
  const int npre = c->opt.nu_pre, npost = c->opt.nu_post, L = npre + npost;
  auto buf = [&](int p) { return sym_buffer<T>(c, Z, p); };
  // float32: the last pre-smoothing sweep from a guess also restricts the
  // residual (mean restriction).  Measured at 512^3: 0.73 ms against 0.51 +
  // 0.45 ms for the sweep and k_resid_restrict_split.  In float64 the fused
  // kernel's histories need 200 registers, which leaves 8-row blocks owning
  // 4 rows: 1.95 ms against 0.96 + 0.85 ms, so float64 keeps the two kernels.
  const bool fuse_resid =
      sizeof(T) == 4 && c->opt.restriction == GMG_RESTRICT_MEAN && (from_x || npre >= 2);
  T* bc = wsp<T>(c, c->L.lv[1].b);
  auto sweep = [&](int p) {
    if constexpr (sizeof(T) == 4) {
      if (fuse_resid && p == npre) {
        sym_split<T, false, true>(c, buf(p - 1), buf(p), B, nullptr, nullptr, a, 0, bc);
        return;
      }
    }
    sym_split<T, false>(c, buf(p - 1), buf(p), B, nullptr, nullptr, a, 0);
  };
  if (from_x)
    sweep(1);
  else
    sym_split<T, true>(c, nullptr, buf(1), B, u, bscale, a, 0);
  for (int p = 2; p <= npre; ++p) sweep(p);
  T* X = buf(npre);
  if (!fuse_resid) resid_restrict_fine<T>(c, X, B, u, bscale, a);
  vcycle_coarse<T>(c, 1);
  {
    const Launch l = pair_launch(s.nx, s.ny, s.nz / 2, 8192, 4, 1);
    GMG_LAUNCH(c, kname("prolong_add", 0, sizeof(T)), (k_prolong_pair<T, true>), l, X,
               (const T*)wsp<T>(c, c->L.lv[1].x), s.geom(), hn, 1, l.kc,
               (const T*)nullptr);
  }
  for (int p = npre + 1; p <= L; ++p) sym_split<T, false>(c, buf(p - 1), buf(p), B, nullptr, nullptr, a, 1);
}

// Fused symmetric sweeps on the finest level (both smoothing phases
// present): on request, or by default when their z-chunks are long.  Each
// chunk of the fused sweep adds two planes of first-colour work and a
// pipeline fill, so it only wins with chunks of 16 planes or more (measured,
// solve with full multigrid cycles, V(2,3), mixed / float64: 2% / 6% faster
// at 384^3 with 21-22-plane chunks, 10% / 12% at 512^3, 9% / 13% at 768^3;
// 13% / 4% slower at 256^3 with 8-plane chunks).
template <typename T>
bool sym_chosen(gmg_ctx* c) {
  const int fs = c->opt.fine_sweep;
  return c->L.shapes.size() > 1 && sym_max_planes(c->L.shapes[0]) >= 10 &&
         (fs == GMG_SWEEP_FUSED || (fs == GMG_SWEEP_AUTO && sym_default_kc<T>(c->L.shapes[0]) >= 16));
}
template <typename T>
bool fused_sweeps(gmg_ctx* c) {
  return c->opt.nu_pre >= 1 && c->opt.nu_post >= 1 && sym_chosen<T>(c);
}

// z = M (s * u) on the finest level with right side u scaled by *bscale
// (null = 1); z in the V-cycle precision, colour-split when there are at
// least two levels, in the natural layout otherwise.
template <typename T>
void vcycle_fine(gmg_ctx* c, const double* u, const double* bscale, T* z) {
  const int nl = (int)c->L.shapes.size();
  const LevelShape& s = c->L.shapes[0];
  if (nl == 1) {
    T* b0 = wsp<T>(c, c->L.b0);
    // scaled copy of the right side, then the direct solve
    const Launch lc = col_launch(s.nx, s.ny, s.nz, 1 << 16);
    if (c->mixed) {
      GMG_LAUNCH(c, kname("gs_first", 0, 4), (k_gs_first<float, double, CellCoef<float>>), lc, (float*)z, u, bscale,
                 (float*)b0, CellCoef<float>{wsp<float>(c, c->L.a32)}, s.geom(), lc.kc, 0);
    } else {
      GMG_LAUNCH(c, kname("gs_first", 0, 8), (k_gs_first<double, double, CellCoef<double>>), lc, (double*)z, u, bscale,
                 (double*)b0, CellCoef<double>{c->a}, s.geom(), lc.kc, 0);
    }
    coarse_solve<T>(c, b0, z);
    return;
  }
  if (c->opt.smoother == GMG_SMOOTH_CHEBYSHEV)
    vcycle_fine_cheb<T>(c, u, bscale, z);
  else if (fused_sweeps<T>(c))
    vcycle_fine_sym<T>(c, u, bscale, z, false);
  else
    vcycle_fine_split<T>(c, u, bscale, z, false);
}

// Full multigrid cycle z = F (s * u) on the whole hierarchy: the right side
// B (colour-split) and its restriction in one pass, the full multigrid cycle
// on levels >= 1, then the interpolated level-1 result as the guess of one
// finest-level V-cycle.
template <typename T>
void fmg_fine(gmg_ctx* c, const double* u, const double* bscale, T* z) {
  if (c->L.shapes.size() == 1) {  // one level: the direct solve
    vcycle_fine<T>(c, u, bscale, z);
    return;
  }
  const LevelShape& s = c->L.shapes[0];
  const size_t hn = c->L.hn;
  T* B = wsp<T>(c, c->L.b0);
  {
    const Launch rl{dim3((s.nx / 2 + BX - 1) / BX, (s.ny / 2 + BY - 1) / BY, s.nz / 2), dim3(BX, BY, 1), 0};
    GMG_LAUNCH(c, kname("restrict_rhs", 0, sizeof(T)), k_restrict_split_rhs<T>, rl, u, bscale, B,
               wsp<T>(c, c->L.lv[1].b), s.geom(), hn);
  }
  fmg_coarse<T>(c, 1);
  const bool fused = fused_sweeps<T>(c);
  T* X0 = fused ? sym_buffer<T>(c, z, 0) : z;
  {
    const Launch l = pair_launch(s.nx, s.ny, s.nz / 2, 8192, 4, 1);
    // the first pre-smoothing half-sweep (red) reads only the black guess;
    // without pre-smoothing the residual reads both colours
    GMG_LAUNCH(c, kname("prolong_set", 0, sizeof(T)), (k_prolong_pair<T, true, true>), l, X0,
               (const T*)wsp<T>(c, c->L.lv[1].x), s.geom(), hn, c->opt.nu_pre > 0 ? 2 : 3, l.kc,
               (const T*)nullptr);
  }
  if (fused)
    vcycle_fine_sym<T>(c, u, bscale, z, true);
  else
    vcycle_fine_split<T>(c, u, bscale, z, true);
}

// One preconditioner application: V-cycle, or full multigrid when fmg.
void cycle_eager(gmg_ctx* c, const double* u, const double* bscale, void* z, bool fmg) {
  if (c->mixed) {
    if (fmg)
      fmg_fine<float>(c, u, bscale, (float*)z);
    else
      vcycle_fine<float>(c, u, bscale, (float*)z);
  } else {
    if (fmg)
      fmg_fine<double>(c, u, bscale, (double*)z);
    else
      vcycle_fine<double>(c, u, bscale, (double*)z);
  }
}

constexpr size_t MAX_GRAPHS = 256;

void drop_graphs(gmg_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// One preconditioner application.  With the graphs option its launches
// (about 40-150, most of them small on the coarse levels) are captured once
// per (input, scale, output, cycle) into a HIP graph and replayed
// afterwards, which takes the host's launch work out of the loop; every
// argument is a workspace address fixed for the context (the caller's
// coefficient pointer too, the graphs being dropped when it changes).
// Measured on MI355X the replays were about 1% slower than eager launches at
// 64^3-256^3: the small coarse-level kernels are bound by the GPU's latency
// between dependent dispatches, not by the host, so graphs are off by
// default.  Eager launches also while profiling (per-kernel events) or if a
// capture ever fails.
void cycle_any(gmg_ctx* c, const double* u, const double* bscale, void* z, bool fmg) {
  if (!c->opt.graphs || c->prof.on || c->graphs_broken || c->err != hipSuccess) {
    cycle_eager(c, u, bscale, z, fmg);
    return;
  }
  const gmg_ctx::GraphKey key{u, bscale, z, fmg};
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (c->graphs.size() >= MAX_GRAPHS) drop_graphs(c);
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      c->cap_stream = nullptr;
      c->graphs_broken = true;
    }
    if (c->graphs_broken || hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      c->graphs_broken = true;
      cycle_eager(c, u, bscale, z, fmg);
      return;
    }
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;  // the launches below are recorded, not run
    cycle_eager(c, u, bscale, z, fmg);
    c->stream = user;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    const bool ok = ec == hipSuccess && c->err == hipSuccess && g &&
                    hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
      (void)hipGetLastError();
      c->err = hipSuccess;  // nothing ran: the captured launches were only recorded
      c->graphs_broken = true;
      cycle_eager(c, u, bscale, z, fmg);
      return;
    }
    it = c->graphs.emplace(key, ge).first;
  }
  note(c, hipGraphLaunch(it->second, c->stream));
}

// ---------------------------------------------------------------------------
// FGMRES pieces.
// ---------------------------------------------------------------------------

Launch red_launch(gmg_ctx* c) { return col_launch(c->nx, c->ny, c->nz, MAX_RED_BLOCKS); }
// the same with one lane per x-pair of the finest level (nx even)
Launch pair_red_launch(gmg_ctx* c) { return col_launch(c->nx / 2, c->ny, c->nz, MAX_RED_BLOCKS); }

void finalize(gmg_ctx* c, int nblocks, int nv, int mode, double* out, const double* scale, double* out2) {
  const Launch one{dim3(1), dim3(FIN_THREADS, 1, 1), 0};
  GMG_LAUNCH(c, "finalize", k_finalize, one, wsp<const double>(c, c->L.partials), nblocks, nv, mode, out, scale,
             out2);
}

// r0 = b - A x (x may be null), ||b||^2 and ||r0||^2 into misc[0..1],
// v_1 scale 1/||r0|| into vscale[0]; r0 stored into V[0] when store.
void init_residual(gmg_ctx* c, const double* f, const double* x, double pb, double pt, bool store) {
  // the pair kernel loads f and x (caller's buffers) as 16-byte vectors
  auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const bool pairs = c->nx % 2 == 0 && a16(f) && a16(x) && a16(c->a);
  const Launch rl = pairs ? pair_red_launch(c) : red_launch(c);
  double* misc = scal_misc(c);
  double* r = store ? wsp<double>(c, c->L.V) : (double*)nullptr;
  const Geom g = c->L.shapes[0].geom();
  if (!pairs)
    GMG_LAUNCH(c, "init_residual", k_init_residual, rl, f, c->a, x, g, pb, pt, r, wsp<double>(c, c->L.partials),
               rl.kc);
  else if (x)
    GMG_LAUNCH(c, "init_residual", k_init_residual_pair<true>, rl, f, c->a, x, g, pb, pt, r,
               wsp<double>(c, c->L.partials), rl.kc);
  else
    GMG_LAUNCH(c, "init_residual", k_init_residual_pair<false>, rl, f, c->a, x, g, pb, pt, r,
               wsp<double>(c, c->L.partials), rl.kc);
  finalize(c, rl.nblocks(), 2, 0, misc, nullptr, nullptr);
  // misc[2] = ||r0||, vscale[0] = 1/||r0||
  const Launch one{dim3(1), dim3(FIN_THREADS, 1, 1), 0};
  GMG_LAUNCH(c, "finalize", k_finalize, one, wsp<const double>(c, c->L.partials) + rl.nblocks(), rl.nblocks(), 1,
             2, misc + 2, nullptr, scal_vscale(c));
}

// Launches of the vector-count templates (NV = 1..MAXV) through tables.
Launch red_flat(gmg_ctx* c) {
  const size_t b = std::min<size_t>((c->N + NTHREADS - 1) / NTHREADS, MAX_RED_BLOCKS);
  return Launch{dim3((unsigned)std::max<size_t>(b, 1)), dim3(BX, BY, 1), 0};
}

// Launch of the operator + multi-dot pass: lane pairs on colour-split z
// (at least two levels), one cell per thread otherwise; at most
// MAX_RED_BLOCKS blocks (one partial per block and vector).
Launch opdot_launch(gmg_ctx* c) {
  const LevelShape& s = c->L.shapes[0];
  if (c->L.shapes.size() == 1) return red_launch(c);
  const int gx = (s.nx / 2 + BX - 1) / BX;
  int gy = (s.ny + BY - 1) / BY;
  if ((long long)gx * gy > MAX_RED_BLOCKS) gy = std::max(1, MAX_RED_BLOCKS / gx);  // rows strided
  const int gz = std::max(1, std::min(s.nz, MAX_RED_BLOCKS / (gx * gy)));
  const int kc = (s.nz + gz - 1) / gz;
  return Launch{dim3(gx, gy, (s.nz + kc - 1) / kc), dim3(BX, BY, 1), kc};
}

template <typename TZ, int NV>
void launch_opdot(gmg_ctx* c, const Launch& rl, const TZ* z, double* w, const double* V) {
  const char* nm = sizeof(TZ) == 4 ? "op_multidot_zf32" : "op_multidot_zf64";
  if (c->L.shapes.size() > 1)
    GMG_LAUNCH(c, nm, (k_op_multidot_split<TZ, NV>), rl, z, c->L.hn, c->a, c->L.shapes[0].geom(), w, V, c->L.ldv,
               wsp<double>(c, c->L.partials), rl.kc);
  else
    GMG_LAUNCH(c, nm, (k_op_multidot<TZ, NV>), rl, z, c->a, c->L.shapes[0].geom(), w, V, c->L.ldv,
               wsp<double>(c, c->L.partials), rl.kc);
}
template <int NV>
void launch_dot(gmg_ctx* c, const Launch& rl, const double* w, const double* V) {
  GMG_LAUNCH(c, "multidot", k_multidot<NV>, rl, w, c->N, V, c->L.ldv, wsp<double>(c, c->L.partials));
}
template <int NV>
void launch_axpy(gmg_ctx* c, const Launch& rl, double* w, const double* V, const double* hc, const double* vs,
                 int last) {
  GMG_LAUNCH(c, "axpy_norm", k_axpy_norm<NV>, rl, w, c->N, V, c->L.ldv, hc, vs, last, wsp<double>(c, c->L.partials));
}
template <typename TZ, int NV>
void launch_update(gmg_ctx* c, const Launch& rl, double* phi, const TZ* Z, const Coeffs16& y, int set) {
  const char* nm = sizeof(TZ) == 4 ? "update_zf32" : "update_zf64";
  if (c->L.shapes.size() > 1) {
    const LevelShape& s = c->L.shapes[0];
    const Launch l = pair_launch(s.nx, s.ny, s.nz, 8192, 8);
    GMG_LAUNCH(c, nm, (k_update_split<TZ, NV>), l, phi, Z, c->L.hn, c->L.ldv, y, s.geom(), l.kc, set);
  } else {
    GMG_LAUNCH(c, nm, (k_update<TZ, NV>), rl, phi, c->N, Z, c->L.ldv, y, set);
  }
}

template <typename TZ, size_t... I>
void opdot_nv(int nv, gmg_ctx* c, const Launch& rl, const TZ* z, double* w, const double* V,
              std::index_sequence<I...>) {
  using F = void (*)(gmg_ctx*, const Launch&, const TZ*, double*, const double*);
  static constexpr F table[] = {&launch_opdot<TZ, (int)I + 1>...};
  table[nv - 1](c, rl, z, w, V);
}
template <size_t... I>
void dot_nv(int nv, gmg_ctx* c, const Launch& rl, const double* w, const double* V, std::index_sequence<I...>) {
  using F = void (*)(gmg_ctx*, const Launch&, const double*, const double*);
  static constexpr F table[] = {&launch_dot<(int)I + 1>...};
  table[nv - 1](c, rl, w, V);
}
template <size_t... I>
void axpy_nv(int nv, gmg_ctx* c, const Launch& rl, double* w, const double* V, const double* hc, const double* vs,
             int last, std::index_sequence<I...>) {
  using F = void (*)(gmg_ctx*, const Launch&, double*, const double*, const double*, const double*, int);
  static constexpr F table[] = {&launch_axpy<(int)I + 1>...};
  table[nv - 1](c, rl, w, V, hc, vs, last);
}
template <typename TZ, size_t... I>
void update_nv(int nv, gmg_ctx* c, const Launch& rl, double* phi, const TZ* Z, const Coeffs16& y, int set,
               std::index_sequence<I...>) {
  using F = void (*)(gmg_ctx*, const Launch&, double*, const TZ*, const Coeffs16&, int);
  static constexpr F table[] = {&launch_update<TZ, (int)I + 1>...};
  table[nv - 1](c, rl, phi, Z, y, set);
}

// One Arnoldi step j: z_j = M v_j, w = A z_j, classical Gram-Schmidt against
// v_0..v_j (dots fused into the operator pass), ||w||; results in hcol(j).
void arnoldi_step(gmg_ctx* c, int j) {
  const size_t N = c->L.ldv;
  double* V = wsp<double>(c, c->L.V);
  char* Zb = c->ws + c->L.Z + (size_t)(c->gmres_mode ? 0 : j) * N * c->L.tsize;
  double* vs = scal_vscale(c);
  double* hc = scal_hcol(c, j);
  cycle_any(c, V + (size_t)j * N, vs + j, Zb, c->fmg_now);
  ++c->nprec;
  const Launch rl = opdot_launch(c);
  const Launch fl = red_flat(c);
  double* w = V + (size_t)(j + 1) * N;
  const int nv = j + 1;
  const auto seq = std::make_index_sequence<MAXV>{};
  for (int q0 = 0; q0 < nv; q0 += MAXV) {
    const int nq = std::min(MAXV, nv - q0);
    if (q0 == 0) {
      if (c->mixed)
        opdot_nv<float>(nq, c, rl, (const float*)Zb, w, V, seq);
      else
        opdot_nv<double>(nq, c, rl, (const double*)Zb, w, V, seq);
      finalize(c, rl.nblocks(), nq, 1, hc + q0, vs + q0, nullptr);
    } else {
      dot_nv(nq, c, fl, w, V + (size_t)q0 * N, seq);
      finalize(c, fl.nblocks(), nq, 1, hc + q0, vs + q0, nullptr);
    }
  }
  for (int q0 = 0; q0 < nv; q0 += MAXV) {
    const int nq = std::min(MAXV, nv - q0);
    const int last = q0 + nq >= nv;
    axpy_nv(nq, c, fl, w, V + (size_t)q0 * N, hc + q0, vs + q0, last, seq);
  }
  finalize(c, fl.nblocks(), 1, 2, hc + (j + 1), nullptr, vs + (j + 1));
}

// phi += sum_{i<k} y_i z_i
// phi += Z_k y (set: phi = 0 + Z_k y, phi not read: the first update of a
// solve from a zero guess, which then needs no zero fill beforehand).
void update_solution(gmg_ctx* c, double* phi, int k, bool set) {
  const Launch fl = flat_launch(c->N);
  const auto seq = std::make_index_sequence<MAXV>{};
  for (int q0 = 0; q0 < k; q0 += MAXV) {
    const int nq = std::min(MAXV, k - q0);
    Coeffs16 y{};
    for (int q = 0; q < nq; ++q) y.v[q] = c->y[q0 + q];
    char* Zb = c->ws + c->L.Z + (size_t)q0 * c->L.ldv * c->L.tsize;
    const int st = set && q0 == 0 ? 1 : 0;
    if (c->mixed)
      update_nv<float>(nq, c, fl, phi, (const float*)Zb, y, st, seq);
    else
      update_nv<double>(nq, c, fl, phi, (const double*)Zb, y, st, seq);
  }
}

int read_back(gmg_ctx* c, const double* dev, int n) {
  note(c, hipMemcpyAsync(c->pinned, dev, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  note(c, hipStreamSynchronize(c->stream));
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

bool valid_ctx(gmg_ctx* c) { return c != nullptr; }

// ---------------------------------------------------------------------------
// The other Krylov methods (Sec. 5.3, Table t1) on natural float64 vectors
// held in the basis slots V[0..], scalars in misc[4..15].
// ---------------------------------------------------------------------------
double* kvec(gmg_ctx* c, int slot) { return wsp<double>(c, c->L.V) + (size_t)slot * c->L.ldv; }
double* kscal(gmg_ctx* c) { return scal_misc(c) + 4; }

// ---------------------------------------------------------------------------
// Bounds of the Chebyshev smoother (Sec. 3.2, eq. qntn): per smoothed level,
// 10 Arnoldi steps (Algorithm 1 without a preconditioner) on M_l^{-1} A_l,
// the largest real part of the Ritz values on the host.  Basis in the Krylov
// slots V[0..10] (natural float64, first n_l entries), stored unnormalised
// with the scales on the device as in the FGMRES steps; classical
// Gram-Schmidt with the dots fused into the pass that writes the new vector.
// Every level's steps are queued without a host wait, and one read-back
// brings all Hessenberg matrices.
// ---------------------------------------------------------------------------

// Largest real part of the eigenvalues of the m x m upper Hessenberg matrix
// H (row-major, row stride ldh) by the Francis double-shift QR iteration with
// deflation at negligible subdiagonals (Golub and Van Loan, Sec. 7.5).  Only
// the eigenvalues are wanted, so each similarity transform is applied to the
// active diagonal block alone.
int ritz_max_real(const double* Hin, int m, int ldh, double* out) {
  std::vector<double> A((size_t)m * m, 0.0);
  double fro = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = std::max(0, i - 1); j < m; ++j) {
      const double v = Hin[(size_t)i * ldh + j];
      if (!std::isfinite(v)) return GMG_ERR_ARG;
      A[(size_t)i * m + j] = v;
      fro += v * v;
    }
  fro = std::sqrt(fro);
  auto h = [&](int i, int j) -> double& { return A[(size_t)i * m + j]; };
  const double eps = 2.220446049250313e-16;
  double best = -INFINITY;
  int hi = m - 1, its = 0, total = 0;
  while (hi >= 0) {
    int lo = hi;
    while (lo > 0) {
      double sc = std::fabs(h(lo - 1, lo - 1)) + std::fabs(h(lo, lo));
      if (sc == 0.0) sc = fro;
      if (std::fabs(h(lo, lo - 1)) <= eps * sc) {
        h(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {  // 1 x 1 block
      best = std::max(best, h(hi, hi));
      --hi;
      its = 0;
      continue;
    }
    if (lo == hi - 1) {  // 2 x 2 block: real pair or complex pair
      const double p = 0.5 * (h(lo, lo) + h(hi, hi));
      const double q = 0.5 * (h(lo, lo) - h(hi, hi));
      const double disc = q * q + h(lo, hi) * h(hi, lo);
      best = std::max(best, disc >= 0.0 ? p + std::sqrt(disc) : p);
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > 100 * m) return GMG_NOT_CONVERGED;
    ++its;
    // shifts: eigenvalues of the trailing 2 x 2 block (sum s, product t);
    // every 10th step of a block an exceptional pair to break cycles
    double s, t;
    if (its % 10 == 0) {
      const double w = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
      s = 1.5 * w + h(hi, hi);
      t = w * w;
    } else {
      s = h(hi - 1, hi - 1) + h(hi, hi);
      t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    }
    // first column of (H - s1)(H - s2), then chase the bulge down
    double x = h(lo, lo) * h(lo, lo) + h(lo, lo + 1) * h(lo + 1, lo) - s * h(lo, lo) + t;
    double y = h(lo + 1, lo) * (h(lo, lo) + h(lo + 1, lo + 1) - s);
    double z = h(lo + 1, lo) * h(lo + 2, lo + 1);
    for (int k = lo; k <= hi - 1; ++k) {
      const int nr = k < hi - 1 ? 3 : 2;  // reflector length
      double v[3] = {x, y, nr == 3 ? z : 0.0};
      const double nrm = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (nrm > 0.0) {
        const double alpha = v[0] >= 0.0 ? -nrm : nrm;
        v[0] -= alpha;
        const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (vv > 0.0) {
          const double beta = 2.0 / vv;
          for (int jc = std::max(lo, k - 1); jc <= hi; ++jc) {  // rows k.. from the left
            double d = 0.0;
            for (int r = 0; r < nr; ++r) d += v[r] * h(k + r, jc);
            for (int r = 0; r < nr; ++r) h(k + r, jc) -= beta * d * v[r];
          }
          for (int ir = lo; ir <= std::min(k + 3, hi); ++ir) {  // columns k.. from the right
            double d = 0.0;
            for (int r = 0; r < nr; ++r) d += h(ir, k + r) * v[r];
            for (int r = 0; r < nr; ++r) h(ir, k + r) -= beta * d * v[r];
          }
        }
      }
      if (k < hi - 1) {
        x = h(k + 1, k);
        y = h(k + 2, k);
        z = k < hi - 2 ? h(k + 3, k) : 0.0;
      }
    }
  }
  *out = best;
  return GMG_OK;
}

// Arnoldi step j = NV - 1 of level l's estimate: w = M_l^{-1} A_l v_j into
// slot j + 1, where v_j = s_j u_j (u_j the raw vector in slot j, s_j =
// vs[j]); the operator in float64 (the finest level's from the float64
// coefficient, the coarser levels' from their float64 faces), M_l the
// smoother's SSOR solve in the V-cycle precision T.  Then h_ij = (w, v_i)
// for i <= j into hcol (dots fused into the pass that writes w), w -= sum_i
// h_ij v_i, and h_{j+1,j} = ||w||, s_{j+1} = 1 / ||w|| (0 when w = 0).
template <typename T, int NV>
void cheb_step(gmg_ctx* c, int l, double* hcol, double* vs) {
  constexpr int j = NV - 1;
  const LevelShape& s = c->L.shapes[l];
  const Geom g = s.geom();
  const size_t n = s.n();
  const double* U = kvec(c, 0);
  const double* v = kvec(c, j);
  double* w = kvec(c, j + 1);
  double* part = wsp<double>(c, c->L.partials);
  double* r = wsp<double>(c, c->L.cr0);  // A_l v_j
  int nb;
  if (l == 0) {
    if (((uintptr_t)c->a & 15) == 0) {  // a loaded as 16-byte vectors
      const Launch rl = pair_red_launch(c);
      GMG_LAUNCH(c, "cheb_op_fine", k_op_pair<0>, rl, v, (const double*)(vs + j), c->a, g, r,
                 (const double*)nullptr, c->L.ldv, part, rl.kc);
    } else {
      const Launch rl = red_launch(c);
      GMG_LAUNCH(c, "cheb_op_fine", k_op_natural<0>, rl, v, (const double*)(vs + j), c->a, g, r,
                 (const double*)nullptr, c->L.ldv, part, rl.kc);
    }
    const T* a = c->mixed ? (const T*)wsp<float>(c, c->L.a32) : (const T*)c->a;
    T* E = wsp<T>(c, c->L.xs);
    T* Bs = wsp<T>(c, c->L.b0);
    // one symmetric sweep from zero: colours 0, 1, 0
    if (sym_chosen<T>(c)) {
      sym_split<T, true>(c, E, E, Bs, r, nullptr, a, 0);
    } else {
      gs_split<T, true>(c, E, Bs, r, nullptr, a, 0);
      gs_split<T, false>(c, E, Bs, nullptr, nullptr, a, 1);
    }
    gs_split<T, false>(c, E, Bs, nullptr, nullptr, a, 0);
    const Launch dl = opdot_launch(c);
    GMG_LAUNCH(c, "cheb_natural_dots", (k_split_to_natural_dots<T, NV>), dl, (const T*)E, c->L.hn, g, w, U,
               c->L.ldv, part, dl.kc);
    nb = dl.nblocks();
  } else {
    const LevelOffsets& o = c->L.lv[l];
    const FaceCoef<double> co64{wsp<double>(c, o.wx64), wsp<double>(c, o.wy64), wsp<double>(c, o.wz64),
                                wsp<double>(c, o.tp64)};
    const Launch fl = flat_launch(n);
    double* vn = r + n;  // v_j made explicit (n_l <= N / 8)
    GMG_LAUNCH(c, "cheb_scale", k_scale_by, fl, vn, v, (const double*)(vs + j), n);
    const Launch cl = cell_launch(s.nx, s.ny, s.nz, 4096, 4);
    GMG_LAUNCH(c, kname("cheb_op", l, 8), k_resid_face<double>, cl, (const double*)vn, (const double*)nullptr,
               co64, g, r, cl.kc);
    T* R = wsp<T>(c, o.cr);
    T* E = wsp<T>(c, o.ce);
    GMG_LAUNCH(c, "convert", (k_convert<T, double>), fl, (const double*)r, R, n);
    const FaceCoef<T> co = face_coef<T>(c, l);
    const Launch pl = pair_launch(s.nx, s.ny, s.nz, 4096, 4);
    GMG_LAUNCH(c, kname("ssor_first", l, sizeof(T)), (k_gs_pair_face<T, true>), pl, E, (const T*)R, co, g, pl.kc,
               0);
    GMG_LAUNCH(c, kname("ssor", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, E, (const T*)R, co, g, pl.kc, 1);
    GMG_LAUNCH(c, kname("ssor", l, sizeof(T)), (k_gs_pair_face<T, false>), pl, E, (const T*)R, co, g, pl.kc, 0);
    Launch rf = fl;
    rf.grid.x = std::min<unsigned>(fl.grid.x, MAX_RED_BLOCKS);
    GMG_LAUNCH(c, "cheb_convert_dots", (k_convert_dots<T, NV>), rf, (const T*)E, w, n, U, c->L.ldv, part);
    nb = rf.nblocks();
  }
  finalize(c, nb, NV, 1, hcol, vs, nullptr);
  Launch rf = flat_launch(n);
  rf.grid.x = std::min<unsigned>(rf.grid.x, MAX_RED_BLOCKS);
  GMG_LAUNCH(c, "axpy_norm", k_axpy_norm<NV>, rf, w, n, U, c->L.ldv, (const double*)hcol, (const double*)vs, 1,
             part);
  finalize(c, rf.nblocks(), 1, 2, hcol + NV, nullptr, vs + NV);
}

template <typename T, size_t... I>
void cheb_step_nv(int nv, gmg_ctx* c, int l, double* hcol, double* vs, std::index_sequence<I...>) {
  using F = void (*)(gmg_ctx*, int, double*, double*);
  static constexpr F table[] = {&cheb_step<T, (int)I + 1>...};
  table[nv - 1](c, l, hcol, vs);
}

// Arnoldi estimates and recurrence coefficients of every smoothed level.
template <typename T>
int cheb_estimate(gmg_ctx* c) {
  const int nl = (int)c->L.shapes.size();
  const int ns = std::max(nl - 1, 0);
  c->cheb_lam.assign(ns, 0.0);
  c->cheb_coef.assign(ns, {});
  if (ns == 0) return GMG_OK;
  double* S = wsp<double>(c, c->L.chs);
  const auto seq = std::make_index_sequence<CHEB_ARNOLDI>{};
  for (int l = 0; l < ns; ++l) {
    double* Sl = S + (size_t)l * CHEB_STRIDE;
    double* vs = Sl + CHEB_SCALES;
    const size_t n = c->L.shapes[l].n();
    const Launch fl = flat_launch(n);
    Launch rf = fl;
    rf.grid.x = std::min<unsigned>(fl.grid.x, MAX_RED_BLOCKS);
    double* V0 = kvec(c, 0);
    GMG_LAUNCH(c, "uniform_start", k_uniform_start, fl, V0, n, (unsigned long long)l);
    GMG_LAUNCH(c, "multidot", k_multidot<1>, rf, (const double*)V0, n, (const double*)V0, c->L.ldv,
               wsp<double>(c, c->L.partials));
    finalize(c, rf.nblocks(), 1, 2, Sl + CHEB_NORM0, nullptr, vs);
    for (int j = 0; j < CHEB_ARNOLDI; ++j)
      cheb_step_nv<T>(j + 1, c, l, Sl + (size_t)j * (CHEB_ARNOLDI + 1), vs, seq);
  }
  std::vector<double> h((size_t)ns * CHEB_STRIDE);
  note(c, hipMemcpyAsync(h.data(), S, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
  note(c, hipStreamSynchronize(c->stream));
  if (c->err != hipSuccess) return GMG_ERR_HIP;
  for (int l = 0; l < ns; ++l) {
    const double* Sl = h.data() + (size_t)l * CHEB_STRIDE;
    const double n0 = Sl[CHEB_NORM0];
    if (!(n0 > 0.0) || !std::isfinite(n0)) return GMG_ERR_NONFINITE;
    double H[(CHEB_ARNOLDI + 1) * CHEB_ARNOLDI] = {};
    int m = CHEB_ARNOLDI;
    for (int j = 0; j < CHEB_ARNOLDI; ++j) {
      const double* col = Sl + (size_t)j * (CHEB_ARNOLDI + 1);
      for (int i = 0; i <= j; ++i) H[i * CHEB_ARNOLDI + j] = col[i];
      const double hn = col[j + 1];
      if (!std::isfinite(hn)) return GMG_ERR_NONFINITE;
      if (hn == 0.0) {  // invariant subspace: the later steps ran on zero vectors
        m = j + 1;
        break;
      }
      H[(j + 1) * CHEB_ARNOLDI + j] = hn;
    }
    double lam = 0.0;
    const int st = ritz_max_real(H, m, CHEB_ARNOLDI, &lam);
    if (st != GMG_OK) return st == GMG_NOT_CONVERGED ? GMG_ERR_NONFINITE : st;
    if (!(lam > 0.0)) return GMG_ERR_NONFINITE;
    c->cheb_lam[l] = lam;
    // eq. qntn on [0.1 lam, 1.1 lam]: theta, delta the centre and half-width
    const double lmin = 0.1 * lam, lmax = 1.1 * lam;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    auto& cf = c->cheb_coef[l];
    cf[0] = 0.0;
    cf[1] = 1.0 / theta;  // d = e / theta
    double rho_prev = 1.0 / sigma;
    for (int st2 = 1; st2 < CHEB_DEGREE; ++st2) {
      const double rho = 1.0 / (2.0 * sigma - rho_prev);
      cf[2 * st2] = rho * rho_prev;
      cf[2 * st2 + 1] = 2.0 * rho / delta;
      rho_prev = rho;
    }
  }
  return GMG_OK;
}

// out = M u (one V-cycle from zero) in the natural layout, float64.
void precond_natural(gmg_ctx* c, const double* u, double* out) {
  char* Zb = c->ws + c->L.Z;
  cycle_any(c, u, nullptr, Zb, false);
  ++c->nprec;
  if (c->L.shapes.size() > 1) {
    const LevelShape& s = c->L.shapes[0];
    const Launch l = pair_launch(s.nx, s.ny, s.nz, 8192, 8);
    if (c->mixed)
      GMG_LAUNCH(c, "split_to_natural", k_split_to_natural<float>, l, (const float*)Zb, c->L.hn, s.geom(), out, l.kc);
    else
      GMG_LAUNCH(c, "split_to_natural", k_split_to_natural<double>, l, (const double*)Zb, c->L.hn, s.geom(), out,
                 l.kc);
  } else {
    const Launch fl = flat_launch(c->N);
    if (c->mixed)
      GMG_LAUNCH(c, "convert_f32_f64", (k_convert<double, float>), fl, (const float*)Zb, out, c->N);
    else
      GMG_LAUNCH(c, "convert_f64_f64", (k_convert<double, double>), fl, (const double*)Zb, out, c->N);
  }
}

// y = c0 x0 + c1 x1 + c2 x2; ||y||^2 into *norm2 (device) when given.
void lincomb(gmg_ctx* c, double* y, const double* x0, double c0, const double* x1, double c1, const double* x2,
             double c2, double* norm2) {
  const Launch fl = red_flat(c);
  GMG_LAUNCH(c, "lincomb", k_lincomb3, fl, y, x0, x1, x2, c0, c1, c2, c->N, norm2 ? 1 : 0,
             wsp<double>(c, c->L.partials));
  if (norm2) finalize(c, fl.nblocks(), 1, 0, norm2, nullptr, nullptr);
}

// (w, u_q) for nv (1 or 2) vectors u_q at stride ldv from U, into out (device).
void kdots(gmg_ctx* c, const double* w, const double* U, int nv, double* out) {
  const Launch fl = red_flat(c);
  if (nv == 1)
    launch_dot<1>(c, fl, w, U);
  else
    launch_dot<2>(c, fl, w, U);
  finalize(c, fl.nblocks(), nv, 0, out, nullptr, nullptr);
}

// w = A x (homogeneous plates) with the dots (w, u_q), q < nv (1 or 2), into out.
void kapply(gmg_ctx* c, const double* x, double* w, const double* U, int nv, double* out) {
  const bool pairs = c->nx % 2 == 0 && ((uintptr_t)c->a & 15) == 0;  // a loaded as 16-byte vectors
  const Launch rl = pairs ? pair_red_launch(c) : red_launch(c);
  const Geom g = c->L.shapes[0].geom();
  double* part = wsp<double>(c, c->L.partials);
  const double* one = nullptr;
  if (pairs && nv == 1)
    GMG_LAUNCH(c, "op_natural", k_op_pair<1>, rl, x, one, c->a, g, w, U, c->L.ldv, part, rl.kc);
  else if (pairs)
    GMG_LAUNCH(c, "op_natural", k_op_pair<2>, rl, x, one, c->a, g, w, U, c->L.ldv, part, rl.kc);
  else if (nv == 1)
    GMG_LAUNCH(c, "op_natural", k_op_natural<1>, rl, x, one, c->a, g, w, U, c->L.ldv, part, rl.kc);
  else
    GMG_LAUNCH(c, "op_natural", k_op_natural<2>, rl, x, one, c->a, g, w, U, c->L.ldv, part, rl.kc);
  finalize(c, rl.nblocks(), nv, 0, out, nullptr, nullptr);
}

// GMRES solution update: u = sum_i y_i v_i (v_i = vscale_i V_i) into the
// basis slot V[k], then phi += M u.
template <int NV>
void launch_update_natural(gmg_ctx* c, const Launch& fl, double* u, const double* V, const Coeffs16& y) {
  GMG_LAUNCH(c, "update_natural", (k_update<double, NV>), fl, u, c->N, V, c->L.ldv, y, 0);
}
template <size_t... I>
void natural_update_nv(int nv, gmg_ctx* c, const Launch& fl, double* u, const double* V, const Coeffs16& y,
                       std::index_sequence<I...>) {
  using F = void (*)(gmg_ctx*, const Launch&, double*, const double*, const Coeffs16&);
  static constexpr F table[] = {&launch_update_natural<(int)I + 1>...};
  table[nv - 1](c, fl, u, V, y);
}

void gmres_update(gmg_ctx* c, double* phi, int k) {
  if (read_back(c, scal_vscale(c), k) != GMG_OK) return;
  std::vector<double> vs(c->pinned, c->pinned + k);
  double* u = kvec(c, k);
  const Launch fl = flat_launch(c->N);
  GMG_LAUNCH(c, "fill", k_fill<double>, fl, u, 0.0, c->N);
  const auto seq = std::make_index_sequence<MAXV>{};
  for (int q0 = 0; q0 < k; q0 += MAXV) {
    const int nq = std::min(MAXV, k - q0);
    Coeffs16 y{};
    for (int q = 0; q < nq; ++q) y.v[q] = c->y[q0 + q] * vs[q0 + q];
    natural_update_nv(nq, c, fl, u, kvec(c, q0), y, seq);
  }
  char* Zb = c->ws + c->L.Z;
  cycle_any(c, u, nullptr, Zb, false);
  ++c->nprec;
  Coeffs16 one{};
  one.v[0] = 1.0;
  if (c->mixed)
    launch_update<float, 1>(c, fl, phi, (const float*)Zb, one, 0);
  else
    launch_update<double, 1>(c, fl, phi, (const double*)Zb, one, 0);
}

struct KrylovOut {
  int it = 0;
  double relres = NAN;
};

// r = b - A x into V[0] (x null: x = 0), ||b|| and ||r|| on the host.
int true_residual(gmg_ctx* c, const double* f, const double* x, double pb, double pt, double& bnorm, double& rnorm) {
  init_residual(c, f, x, pb, pt, true);
  if (read_back(c, scal_misc(c), 3) != GMG_OK) return GMG_ERR_HIP;
  bnorm = std::sqrt(c->pinned[0]);
  rnorm = c->pinned[2];
  if (!std::isfinite(bnorm) || !std::isfinite(rnorm)) return GMG_ERR_NONFINITE;
  return GMG_OK;
}

// b = 0: phi = 0 (whatever the initial guess), relative residual 0, as in
// fgmres_solve.
int zero_solution(gmg_ctx* c, double* x, KrylovOut& out) {
  GMG_LAUNCH(c, "fill", k_fill<double>, flat_launch(c->N), x, 0.0, c->N);
  note(c, hipStreamSynchronize(c->stream));
  out.relres = 0.0;
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

// Preconditioned CG, or FCG (new direction A-orthogonalised against the last
// one) when flexible.  Slots: r 0, q 1, z 2, p 3.
int krylov_cg(gmg_ctx* c, const double* f, double pb, double pt, double tol, double* x, int max_iter, bool flexible,
              KrylovOut& out) {
  double* r = kvec(c, 0);
  double* q = kvec(c, 1);
  double* z = kvec(c, 2);
  double* p = kvec(c, 3);
  double* s = kscal(c);
  while (true) {
    double bnorm, rn;
    int st = true_residual(c, f, x, pb, pt, bnorm, rn);
    if (st != GMG_OK) return st;
    if (bnorm == 0.0) return zero_solution(c, x, out);
    out.relres = rn / bnorm;
    if (rn < tol * bnorm) return GMG_OK;
    if (out.it >= max_iter) return GMG_NOT_CONVERGED;
    precond_natural(c, r, z);
    lincomb(c, p, z, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr);
    kdots(c, z, r, 1, s);  // rho = (r, z)
    if (read_back(c, s, 1) != GMG_OK) return GMG_ERR_HIP;
    double rho = c->pinned[0];
    while (out.it < max_iter) {
      kapply(c, p, q, p, 1, s);  // q = A p, (q, p)
      if (read_back(c, s, 1) != GMG_OK) return GMG_ERR_HIP;
      const double pq = c->pinned[0];
      if (!std::isfinite(pq) || pq == 0.0) return GMG_ERR_BREAKDOWN;
      const double alpha = rho / pq;
      lincomb(c, x, x, 1.0, p, alpha, nullptr, 0.0, nullptr);
      lincomb(c, r, r, 1.0, q, -alpha, nullptr, 0.0, s);
      ++out.it;
      if (read_back(c, s, 1) != GMG_OK) return GMG_ERR_HIP;
      const double rr = std::sqrt(c->pinned[0]);
      if (!std::isfinite(rr)) return GMG_ERR_NONFINITE;
      if (rr < tol * bnorm) break;
      precond_natural(c, r, z);
      kdots(c, z, r, 2, s);  // (z, r), (z, q): r and q are adjacent slots
      if (read_back(c, s, 2) != GMG_OK) return GMG_ERR_HIP;
      const double rho_new = c->pinned[0];
      const double beta = flexible ? -c->pinned[1] / pq : rho_new / rho;
      lincomb(c, p, z, 1.0, p, beta, nullptr, 0.0, nullptr);
      rho = rho_new;
    }
  }
}

// Right-preconditioned CGS.  Slots: r 0, r~ 1, p 2, u 3, q 4, v 5, M-vector 6,
// scratch 7.
int krylov_cgs(gmg_ctx* c, const double* f, double pb, double pt, double tol, double* x, int max_iter,
               KrylovOut& out) {
  double *r = kvec(c, 0), *rs = kvec(c, 1), *p = kvec(c, 2), *u = kvec(c, 3), *q = kvec(c, 4), *v = kvec(c, 5);
  double *mh = kvec(c, 6), *w = kvec(c, 7);
  double* s = kscal(c);
  while (true) {
    double bnorm, rn;
    int st = true_residual(c, f, x, pb, pt, bnorm, rn);
    if (st != GMG_OK) return st;
    if (bnorm == 0.0) return zero_solution(c, x, out);
    out.relres = rn / bnorm;
    if (rn < tol * bnorm) return GMG_OK;
    if (out.it >= max_iter) return GMG_NOT_CONVERGED;
    lincomb(c, rs, r, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr);
    lincomb(c, p, r, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr);
    lincomb(c, u, r, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr);
    double rho = rn * rn;  // (r, r~) with r~ = r
    while (out.it < max_iter) {
      precond_natural(c, p, mh);
      kapply(c, mh, v, rs, 1, s);  // v = A M p, (v, r~)
      if (read_back(c, s, 1) != GMG_OK) return GMG_ERR_HIP;
      const double sigma = c->pinned[0];
      if (!std::isfinite(sigma) || sigma == 0.0) return GMG_ERR_BREAKDOWN;
      const double alpha = rho / sigma;
      lincomb(c, q, u, 1.0, v, -alpha, nullptr, 0.0, nullptr);
      lincomb(c, w, u, 1.0, q, 1.0, nullptr, 0.0, nullptr);
      precond_natural(c, w, mh);  // u^ = M (u + q)
      lincomb(c, x, x, 1.0, mh, alpha, nullptr, 0.0, nullptr);
      kapply(c, mh, w, rs, 1, s);  // w = A u^
      lincomb(c, r, r, 1.0, w, -alpha, nullptr, 0.0, s + 1);
      kdots(c, r, rs, 1, s + 2);  // rho' = (r, r~)
      ++out.it;
      if (read_back(c, s, 3) != GMG_OK) return GMG_ERR_HIP;
      const double rr = std::sqrt(c->pinned[1]), rho_new = c->pinned[2];
      if (!std::isfinite(rr)) return GMG_ERR_NONFINITE;
      if (rr < tol * bnorm) break;
      const double beta = rho_new / rho;
      lincomb(c, u, r, 1.0, q, beta, nullptr, 0.0, nullptr);
      lincomb(c, p, u, 1.0, q, beta, p, beta * beta, nullptr);
      rho = rho_new;
    }
  }
}

// Right-preconditioned BiCGSTAB.  Slots: r 0, r~ 1, p 2, v 3, s 4, t 5,
// M p 6, M s 7.
int krylov_bicgstab(gmg_ctx* c, const double* f, double pb, double pt, double tol, double* x, int max_iter,
                    KrylovOut& out) {
  double *r = kvec(c, 0), *rs = kvec(c, 1), *p = kvec(c, 2), *v = kvec(c, 3), *sv = kvec(c, 4), *t = kvec(c, 5);
  double *ph = kvec(c, 6), *sh = kvec(c, 7);
  double* s = kscal(c);
  while (true) {
    double bnorm, rn;
    int st = true_residual(c, f, x, pb, pt, bnorm, rn);
    if (st != GMG_OK) return st;
    if (bnorm == 0.0) return zero_solution(c, x, out);
    out.relres = rn / bnorm;
    if (rn < tol * bnorm) return GMG_OK;
    if (out.it >= max_iter) return GMG_NOT_CONVERGED;
    lincomb(c, rs, r, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr);
    const Launch fl = flat_launch(c->N);
    GMG_LAUNCH(c, "fill", k_fill<double>, fl, p, 0.0, c->N);
    GMG_LAUNCH(c, "fill", k_fill<double>, fl, v, 0.0, c->N);
    double rho = 1.0, alpha = 1.0, omega = 1.0, rho_new = rn * rn;  // (r~, r) with r~ = r
    while (out.it < max_iter) {
      const double beta = (rho_new / rho) * (alpha / omega);
      lincomb(c, p, r, 1.0, p, beta, v, -beta * omega, nullptr);
      precond_natural(c, p, ph);
      kapply(c, ph, v, rs, 1, s);  // v = A M p, (v, r~)
      if (read_back(c, s, 1) != GMG_OK) return GMG_ERR_HIP;
      const double rv = c->pinned[0];
      if (!std::isfinite(rv) || rv == 0.0) return GMG_ERR_BREAKDOWN;
      alpha = rho_new / rv;
      lincomb(c, sv, r, 1.0, v, -alpha, nullptr, 0.0, s);
      if (read_back(c, s, 1) != GMG_OK) return GMG_ERR_HIP;
      if (std::sqrt(c->pinned[0]) < tol * bnorm) {  // converged half-way
        lincomb(c, x, x, 1.0, ph, alpha, nullptr, 0.0, nullptr);
        lincomb(c, r, sv, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr);
        ++out.it;
        break;
      }
      precond_natural(c, sv, sh);
      kapply(c, sh, t, sv, 1, s);  // t = A M s, (t, s)
      kdots(c, t, t, 1, s + 1);   // (t, t)
      if (read_back(c, s, 2) != GMG_OK) return GMG_ERR_HIP;
      const double ts = c->pinned[0], tt = c->pinned[1];
      if (!std::isfinite(tt) || tt == 0.0) return GMG_ERR_BREAKDOWN;
      omega = ts / tt;
      lincomb(c, x, x, 1.0, ph, alpha, sh, omega, nullptr);
      lincomb(c, r, sv, 1.0, t, -omega, nullptr, 0.0, s);
      kdots(c, r, rs, 1, s + 1);
      ++out.it;
      if (read_back(c, s, 2) != GMG_OK) return GMG_ERR_HIP;
      const double rr = std::sqrt(c->pinned[0]);
      if (!std::isfinite(rr)) return GMG_ERR_NONFINITE;
      rho = rho_new;
      rho_new = c->pinned[1];
      if (rr < tol * bnorm) break;
      if (omega == 0.0) return GMG_ERR_BREAKDOWN;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void gmg_default_options(gmg_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->restart = 10;
  opt->max_iter = 200;
  opt->nu_pre = 2;
  opt->nu_post = 2;
  opt->precision = GMG_MIXED;
  opt->coarse_max_cells = 4096;
  opt->fine_sweep = GMG_SWEEP_AUTO;
  opt->cold_cycle = GMG_CYCLE_FMG;
  opt->graphs = 0;
  opt->smoother = GMG_SMOOTH_RBGS;
  opt->warm_cycle = GMG_CYCLE_V;
  opt->restriction = GMG_RESTRICT_MEAN;
}

size_t gmg_workspace_bytes(int nx, int ny, int nz, const gmg_options* opt) {
  Layout L;
  if (make_layout(nx, ny, nz, 1.0, 1.0, 1.0, opt, &L) != GMG_OK) return 0;
  return L.total;
}

namespace {

// Context c (constructed by the caller) for the grid, coefficient and
// layout L, on the workspace ws (checked by the caller) and the host buffer
// host_buf of MAX_RESTART + 8 doubles for read-backs; builds the hierarchy.
int init_ctx(gmg_ctx* c, int nx, int ny, int nz, double hx, double hy, double hz, const double* a_dev,
             const gmg_options* opt, void* ws, size_t ws_bytes, void* hip_stream, const Layout& L,
             double* host_buf) {
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->hx = hx;
  c->hy = hy;
  c->hz = hz;
  c->opt = *opt;
  c->a = a_dev;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)ws;
  c->ws_bytes = ws_bytes;
  c->L = L;
  c->N = L.shapes[0].n();
  c->mixed = opt->precision == GMG_MIXED;
  c->nc = (int)L.shapes.back().n();
  // the Chebyshev smoother and the transpose restriction run every level
  // through the per-level kernels
  c->bottom_from =
      (opt->smoother == GMG_SMOOTH_CHEBYSHEV || opt->restriction == GMG_RESTRICT_TRANSPOSE) ? -1 : bottom_level(L);
  c->err = hipSuccess;
  c->pinned = host_buf;
  {
    int dev = 0, n = 0;
    c->cus = hipGetDevice(&dev) == hipSuccess &&
                     hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0
                 ? n
                 : 256;
  }
  const int m = opt->restart;
  c->R.assign((size_t)m * m, 0.0);
  c->cs.assign(m, 0.0);
  c->sn.assign(m, 0.0);
  c->g.assign(m + 1, 0.0);
  c->y.assign(m, 0.0);
  int r = c->mixed ? write_bottom_args<float>(c) : write_bottom_args<double>(c);
  if (r == GMG_OK) r = build_hierarchy(c);
  if (r == GMG_OK && opt->smoother == GMG_SMOOTH_CHEBYSHEV)
    r = c->mixed ? cheb_estimate<float>(c) : cheb_estimate<double>(c);
  return r;
}

int check_setup_args(double hx, double hy, double hz, const double* a_dev, const gmg_options* opt) {
  if (!a_dev || !opt) return GMG_ERR_ARG;
  if (!(hx > 0) || !(hy > 0) || !(hz > 0) || !std::isfinite(hx) || !std::isfinite(hy) || !std::isfinite(hz))
    return GMG_ERR_ARG;
  return GMG_OK;
}

}  // namespace

int gmg_setup(int nx, int ny, int nz, double hx, double hy, double hz, const double* a_dev,
              const gmg_options* opt, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
              gmg_ctx** out) {
  if (!out) return GMG_ERR_ARG;
  *out = nullptr;
  int st = check_setup_args(hx, hy, hz, a_dev, opt);
  if (st != GMG_OK) return st;
  Layout L;
  st = make_layout(nx, ny, nz, hx, hy, hz, opt, &L);
  if (st != GMG_OK) return st;
  if (!workspace_dev || workspace_bytes < L.total || ((uintptr_t)workspace_dev % ALIGN) != 0)
    return GMG_ERR_WORKSPACE;
  gmg_ctx* c = new (std::nothrow) gmg_ctx();
  if (!c) return GMG_ERR_ARG;
  double* pinned = nullptr;
  if (hipHostMalloc((void**)&pinned, (size_t)(MAX_RESTART + 8) * 8, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return GMG_ERR_HIP;
  }
  const int r = init_ctx(c, nx, ny, nz, hx, hy, hz, a_dev, opt, workspace_dev, workspace_bytes, hip_stream, L,
                         pinned);
  if (r != GMG_OK) {
    gmg_destroy(c);
    return r;
  }
  *out = c;
  return GMG_OK;
}

int gmg_update_coefficient(gmg_ctx* c, const double* a_dev) {
  if (!valid_ctx(c) || !a_dev) return GMG_ERR_ARG;
  const bool cheb = c->opt.smoother == GMG_SMOOTH_CHEBYSHEV;
  // the float64 cycle reads the coefficient itself; the Chebyshev
  // coefficients are launch arguments
  if (a_dev != c->a || cheb) drop_graphs(c);
  c->a = a_dev;
  int r = build_hierarchy(c);
  if (r == GMG_OK && cheb) r = c->mixed ? cheb_estimate<float>(c) : cheb_estimate<double>(c);
  return r;
}

int gmg_chebyshev_estimates(gmg_ctx* c, double* lam, int cap, int* nlevels) {
  if (!valid_ctx(c) || !lam || !nlevels || cap < 0 || c->opt.smoother != GMG_SMOOTH_CHEBYSHEV) return GMG_ERR_ARG;
  *nlevels = (int)c->cheb_lam.size();
  for (int l = 0; l < std::min(cap, *nlevels); ++l) lam[l] = c->cheb_lam[l];
  return GMG_OK;
}

int gmg_ritz_max_real(const double* H, int m, int ldh, double* out) {
  if (!H || !out || m < 1 || m > 64 || ldh < m) return GMG_ERR_ARG;
  return ritz_max_real(H, m, ldh, out);
}

int gmg_set_stream(gmg_ctx* c, void* hip_stream) {
  if (!valid_ctx(c)) return GMG_ERR_ARG;
  c->stream = (hipStream_t)hip_stream;
  return GMG_OK;
}

}  // extern "C"

namespace {

void gmres_update(gmg_ctx* c, double* phi, int k);

// FGMRES (Algorithm 1) or, with gmres, right-preconditioned GMRES (one slot
// for the preconditioned vector; the solution update applies M to V y).
int fgmres_core(gmg_ctx* c, const double* f_dev, double phi_bot, double phi_top, double tol, double* phi_dev,
                int use_x0, int* iterations, double* res_hist, int res_hist_cap, int* res_hist_len,
                double* final_true_relres, bool allow_fmg, bool gmres) {
  if (!valid_ctx(c) || !f_dev || !phi_dev) return GMG_ERR_ARG;
  if (!(tol >= 0.0) || !std::isfinite(phi_bot) || !std::isfinite(phi_top)) return GMG_ERR_ARG;
  if (res_hist_cap < 0 || (res_hist_cap > 0 && !res_hist)) return GMG_ERR_ARG;
  const int m = c->opt.restart;
  int it = 0, nhist = 0;
  auto push_hist = [&](double v) {
    if (nhist < res_hist_cap) res_hist[nhist] = v;
    ++nhist;
  };
  // without an initial guess phi starts at zero: the first update writes
  // phi = Z y without reading it, and phi is filled with zeros only if the
  // solve ends, or reads phi, before any update
  bool phi_zero = !use_x0;
  auto zero_phi = [&]() {
    if (!phi_zero) return;
    const Launch fl = flat_launch(c->N);
    GMG_LAUNCH(c, "fill", k_fill<double>, fl, phi_dev, 0.0, c->N);
    phi_zero = false;
  };
  auto finish = [&](int status, double relres) {
    zero_phi();
    if (iterations) *iterations = it;
    if (res_hist_len) *res_hist_len = std::min(nhist, res_hist_cap);
    if (final_true_relres) *final_true_relres = relres;
    return status;
  };
  c->fmg_now = allow_fmg && (use_x0 ? c->opt.warm_cycle : c->opt.cold_cycle) == GMG_CYCLE_FMG;
  c->gmres_mode = gmres;
  c->nprec = 0;
  double* misc = scal_misc(c);
  bool first = true;
  double bnorm = 0.0;
  // the last cycle ended on a converged estimate (or at max_iter): the true
  // residual is likely final, so its pass computes the norm without storing
  // r into V[0] (a quarter of the pass's bytes); if it is not final after
  // all, the pass runs again with the store for the restart
  bool likely_last = false;
  while (true) {
    // r_0 = b - A x_0 into V[0] (the true residual at every restart)
    init_residual(c, f_dev, (first && !use_x0) ? nullptr : phi_dev, phi_bot, phi_top, !likely_last);
    if (read_back(c, misc, 3) != GMG_OK) return finish(GMG_ERR_HIP, NAN);
    const double bn2 = c->pinned[0];
    double beta = c->pinned[2];
    if (!std::isfinite(bn2) || !std::isfinite(beta)) return finish(GMG_ERR_NONFINITE, NAN);
    if (first) {
      bnorm = std::sqrt(bn2);
      if (bnorm == 0.0) {
        phi_zero = true;
        zero_phi();
        note(c, hipStreamSynchronize(c->stream));
        push_hist(0.0);
        return finish(c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP, 0.0);
      }
      push_hist(beta / bnorm);
      first = false;
    }
    if (beta < tol * bnorm) return finish(GMG_OK, beta / bnorm);
    if (it >= c->opt.max_iter) return finish(GMG_NOT_CONVERGED, beta / bnorm);
    if (likely_last) {
      // (the same kernel and reduction: the same norms)
      init_residual(c, f_dev, phi_dev, phi_bot, phi_top, true);
      if (read_back(c, misc, 3) != GMG_OK) return finish(GMG_ERR_HIP, NAN);
      beta = c->pinned[2];
    }
    likely_last = false;
    // Arnoldi cycle
    std::fill(c->g.begin(), c->g.end(), 0.0);
    c->g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      if (it >= c->opt.max_iter) break;
      arnoldi_step(c, j);
      if (read_back(c, scal_hcol(c, j), j + 2) != GMG_OK) return finish(GMG_ERR_HIP, NAN);
      std::vector<double> h(c->pinned, c->pinned + j + 2);
      double colnorm = 0.0;
      for (double v : h) {
        if (!std::isfinite(v)) return finish(GMG_ERR_NONFINITE, NAN);
        colnorm += v * v;
      }
      colnorm = std::sqrt(colnorm);
      const bool breakdown = h[j + 1] <= BREAKDOWN_TOL * colnorm;
      // apply the previous Givens rotations to the new column, then a new
      // rotation that zeroes h_{j+1,j}
      for (int i = 0; i < j; ++i) {
        const double t = c->cs[i] * h[i] + c->sn[i] * h[i + 1];
        h[i + 1] = -c->sn[i] * h[i] + c->cs[i] * h[i + 1];
        h[i] = t;
      }
      const double d = std::hypot(h[j], h[j + 1]);
      c->cs[j] = d > 0 ? h[j] / d : 1.0;
      c->sn[j] = d > 0 ? h[j + 1] / d : 0.0;
      h[j] = d;
      for (int i = 0; i <= j; ++i) c->R[(size_t)i * m + j] = h[i];
      c->g[j + 1] = -c->sn[j] * c->g[j];
      c->g[j] = c->cs[j] * c->g[j];
      ++it;
      k = j + 1;
      const double est = std::fabs(c->g[j + 1]);
      push_hist(est / bnorm);
      if (est < tol * bnorm || breakdown) {
        likely_last = true;
        break;
      }
    }
    if (it >= c->opt.max_iter) likely_last = true;
    // y = R_k^{-1} g_k, phi += Z_k y
    for (int i = k - 1; i >= 0; --i) {
      double s = c->g[i];
      for (int q = i + 1; q < k; ++q) s -= c->R[(size_t)i * m + q] * c->y[q];
      const double rii = c->R[(size_t)i * m + i];
      c->y[i] = rii != 0.0 ? s / rii : 0.0;
    }
    if (k > 0 && !gmres) {
      update_solution(c, phi_dev, k, phi_zero);
      phi_zero = false;
    } else {
      zero_phi();
      if (k > 0) gmres_update(c, phi_dev, k);
    }
  }
}

}  // namespace

extern "C" {

int fgmres_solve(gmg_ctx* c, const double* f_dev, double phi_bot, double phi_top, double tol, double* phi_dev,
                 int use_x0, int* iterations, double* res_hist, int res_hist_cap, int* res_hist_len,
                 double* final_true_relres) {
  return fgmres_core(c, f_dev, phi_bot, phi_top, tol, phi_dev, use_x0, iterations, res_hist, res_hist_cap,
                     res_hist_len, final_true_relres, true, false);
}

// ---------------------------------------------------------------------------
// Solve without allocation: the workspace is a device array the library
// holds on every GPU it runs on.
// ---------------------------------------------------------------------------

// The array itself.  In host code its name is a host-side stand-in, not a
// device address: only scratch_device() below yields the address kernels may
// use.
static __device__ __align__(256) unsigned char scratch[GMG_STATIC_SCRATCH_BYTES];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
void* g_scratch_ptr[STATIC_MAX_DEVICES];  // device address of scratch, per device
std::mutex g_scratch_mu[STATIC_MAX_DEVICES];

// Device address of scratch on the current device (taken once per device,
// with that device current), or null with *dev < 0 on failure.
void* scratch_device(int* dev) {
  if (hipGetDevice(dev) != hipSuccess || *dev < 0 || *dev >= STATIC_MAX_DEVICES) {
    (void)hipGetLastError();
    *dev = -1;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu[*dev]);
  if (!g_scratch_ptr[*dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[*dev] = p;
  }
  return g_scratch_ptr[*dev];
}

}  // namespace

int fgmres_solve_static(int nx, int ny, int nz, double hx, double hy, double hz, const double* a_dev,
                        const gmg_options* opt, void* hip_stream, const double* f_dev, double phi_bot,
                        double phi_top, double tol, double* phi_dev, int use_x0, int* iterations, double* res_hist,
                        int res_hist_cap, int* res_hist_len, double* final_true_relres) {
  int st = check_setup_args(hx, hy, hz, a_dev, opt);
  if (st != GMG_OK) return st;
  if (opt->graphs != 0) return GMG_ERR_ARG;  // capturing a graph allocates
  Layout L;
  st = make_layout(nx, ny, nz, hx, hy, hz, opt, &L);
  if (st != GMG_OK) return st;
  if (L.total > GMG_STATIC_SCRATCH_BYTES) return GMG_ERR_WORKSPACE;
  int dev = -1;
  void* ws = scratch_device(&dev);
  if (!ws) return GMG_ERR_HIP;
  // one call at a time per GPU: every call on it uses the same array
  std::lock_guard<std::mutex> g(g_scratch_mu[dev]);
  double host_buf[MAX_RESTART + 8];
  gmg_ctx c;
  st = init_ctx(&c, nx, ny, nz, hx, hy, hz, a_dev, opt, ws, GMG_STATIC_SCRATCH_BYTES, hip_stream, L, host_buf);
  if (st == GMG_OK)
    st = fgmres_solve(&c, f_dev, phi_bot, phi_top, tol, phi_dev, use_x0, iterations, res_hist, res_hist_cap,
                      res_hist_len, final_true_relres);
  // nothing of this call may still run on the array when the next one starts
  if (hipStreamSynchronize(c.stream) != hipSuccess && st >= 0) st = GMG_ERR_HIP;
  if (c.prof.on || !c.prof.pending.empty() || !c.prof.pool.empty()) {
    for (auto& r : c.prof.pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : c.prof.pool) (void)hipEventDestroy(e);
  }
  return st;
}

int gmg_krylov_solve(gmg_ctx* c, int method, const double* f_dev, double phi_bot, double phi_top, double tol,
                     double* phi_dev, int use_x0, int* iterations, int* precond_apps, double* final_true_relres) {
  if (!valid_ctx(c) || !f_dev || !phi_dev) return GMG_ERR_ARG;
  if (method < GMG_KRYLOV_FGMRES || method > GMG_KRYLOV_BICGSTAB) return GMG_ERR_ARG;
  if (!(tol >= 0.0) || !std::isfinite(phi_bot) || !std::isfinite(phi_top)) return GMG_ERR_ARG;
  const int slots = c->opt.restart + 1;
  if ((method == GMG_KRYLOV_CG || method == GMG_KRYLOV_FCG) && slots < 4) return GMG_ERR_ARG;
  if ((method == GMG_KRYLOV_CGS || method == GMG_KRYLOV_BICGSTAB) && slots < 8) return GMG_ERR_ARG;
  int st;
  int its = 0;
  double rel = NAN;
  if (method == GMG_KRYLOV_FGMRES || method == GMG_KRYLOV_GMRES) {
    st = fgmres_core(c, f_dev, phi_bot, phi_top, tol, phi_dev, use_x0, &its, nullptr, 0, nullptr, &rel, false,
                     method == GMG_KRYLOV_GMRES);
  } else {
    c->fmg_now = false;
    c->gmres_mode = false;
    c->nprec = 0;
    if (!use_x0) {
      const Launch fl = flat_launch(c->N);
      GMG_LAUNCH(c, "fill", k_fill<double>, fl, phi_dev, 0.0, c->N);
    }
    KrylovOut out;
    const int mi = c->opt.max_iter;
    if (method == GMG_KRYLOV_CG || method == GMG_KRYLOV_FCG)
      st = krylov_cg(c, f_dev, phi_bot, phi_top, tol, phi_dev, mi, method == GMG_KRYLOV_FCG, out);
    else if (method == GMG_KRYLOV_CGS)
      st = krylov_cgs(c, f_dev, phi_bot, phi_top, tol, phi_dev, mi, out);
    else
      st = krylov_bicgstab(c, f_dev, phi_bot, phi_top, tol, phi_dev, mi, out);
    its = out.it;
    rel = out.relres;
    note(c, hipStreamSynchronize(c->stream));
    if (c->err != hipSuccess) st = GMG_ERR_HIP;
  }
  if (iterations) *iterations = its;
  if (precond_apps) *precond_apps = c->nprec;
  if (final_true_relres) *final_true_relres = rel;
  return st;
}

int gmg_apply_operator(gmg_ctx* c, const double* x_dev, double* y_dev, double phi_bot, double phi_top) {
  if (!valid_ctx(c) || !x_dev || !y_dev) return GMG_ERR_ARG;
  const Launch lc = col_launch(c->nx, c->ny, c->nz, 1 << 16);
  GMG_LAUNCH(c, "apply_bc", k_apply_bc, lc, x_dev, c->a, c->L.shapes[0].geom(), phi_bot, phi_top, y_dev, lc.kc);
  note(c, hipStreamSynchronize(c->stream));
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

namespace {
// (launched eagerly: the caller's input pointer changes from call to call,
// so a captured graph would rarely be replayed)
int cycle_api(gmg_ctx* c, const double* v_dev, double* z_dev, bool fmg) {
  if (!valid_ctx(c) || !v_dev || !z_dev) return GMG_ERR_ARG;
  const bool split = c->L.shapes.size() > 1;
  if (c->mixed) {
    float* z32 = wsp<float>(c, c->L.Z);
    cycle_eager(c, v_dev, nullptr, z32, fmg);
    const Launch fl = flat_launch(c->N);
    if (split) {  // z = 0 + 1 * z32, exact, into the natural layout
      Coeffs16 one{};
      one.v[0] = 1.0;
      launch_update<float, 1>(c, fl, z_dev, z32, one, 1);
    } else {
      GMG_LAUNCH(c, "convert_f32_f64", (k_convert<double, float>), fl, (const float*)z32, z_dev, c->N);
    }
  } else if (split) {
    double* z64 = wsp<double>(c, c->L.Z);
    cycle_eager(c, v_dev, nullptr, z64, fmg);
    const Launch fl = flat_launch(c->N);
    Coeffs16 one{};
    one.v[0] = 1.0;
    launch_update<double, 1>(c, fl, z_dev, z64, one, 1);
  } else {
    cycle_eager(c, v_dev, nullptr, z_dev, fmg);
  }
  note(c, hipStreamSynchronize(c->stream));
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}
}  // namespace

int gmg_vcycle(gmg_ctx* c, const double* v_dev, double* z_dev) { return cycle_api(c, v_dev, z_dev, false); }

int gmg_fmg(gmg_ctx* c, const double* v_dev, double* z_dev) {
  if (valid_ctx(c) && c->opt.smoother == GMG_SMOOTH_CHEBYSHEV) return GMG_ERR_ARG;  // V-cycles only
  return cycle_api(c, v_dev, z_dev, true);
}

int gmg_face_flux_grad(gmg_ctx* c, const double* phi_dev, const double* lam_dev, double phi_bot, double phi_top,
                       double* dLda_dev) {
  if (!valid_ctx(c) || !phi_dev || !lam_dev || !dLda_dev) return GMG_ERR_ARG;
  auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (c->nx % 2 == 0 && a16(phi_dev) && a16(lam_dev) && a16(dLda_dev)) {
    const Launch lc = col_launch(c->nx / 2, c->ny, c->nz, 1 << 16);
    GMG_LAUNCH(c, "face_grad", k_face_grad_pair, lc, phi_dev, lam_dev, c->L.shapes[0].geom(), phi_bot, phi_top,
               dLda_dev, lc.kc);
  } else {
    const Launch lc = col_launch(c->nx, c->ny, c->nz, 1 << 16);
    GMG_LAUNCH(c, "face_grad", k_face_grad, lc, phi_dev, lam_dev, c->L.shapes[0].geom(), phi_bot, phi_top,
               dLda_dev, lc.kc);
  }
  note(c, hipStreamSynchronize(c->stream));
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

namespace {

// The assembly and field kernels of a time step, enqueued without waiting.
int launch_assemble(gmg_ctx* c, const double* ne_dev, const double* np_dev, const gmg_step_params* prm,
                    double* a_dev, double* f_dev) {
  if (!ne_dev || !np_dev || !prm || !a_dev || !f_dev) return GMG_ERR_ARG;
  const double vals[] = {prm->eps0_over_e, prm->tau_eff, prm->mu_e, prm->mu_p, prm->De[0], prm->De[1], prm->De[2]};
  for (double v : vals)
    if (!std::isfinite(v)) return GMG_ERR_ARG;
  if (c->ny > 65535 * BY) return GMG_ERR_SHAPE;
  const StepCoef p{prm->eps0_over_e, prm->tau_eff, prm->mu_e, prm->mu_p,
                   prm->De[0] / (c->hx * c->hx), prm->De[1] / (c->hy * c->hy), prm->De[2] / (c->hz * c->hz)};
  auto a16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  if (c->nx % 2 == 0 && a16(ne_dev) && a16(np_dev) && a16(a_dev) && a16(f_dev)) {
    const Launch l = cell_launch(c->nx / 2, c->ny, c->nz, 8192, 8);
    GMG_LAUNCH(c, "assemble_step", k_assemble_step_pair, l, ne_dev, np_dev, c->L.shapes[0].geom(), p, a_dev, f_dev,
               l.kc);
  } else {
    const Launch l = cell_launch(c->nx, c->ny, c->nz, 8192, 8);
    GMG_LAUNCH(c, "assemble_step", k_assemble_step, l, ne_dev, np_dev, c->L.shapes[0].geom(), p, a_dev, f_dev,
               l.kc);
  }
  return GMG_OK;
}

int launch_field(gmg_ctx* c, const double* phi_dev, double phi_bot, double phi_top, double* ex_dev, double* ey_dev,
                 double* ez_dev, double* emag_dev) {
  if (!phi_dev || !ex_dev || !ey_dev || !ez_dev || !emag_dev) return GMG_ERR_ARG;
  if (!std::isfinite(phi_bot) || !std::isfinite(phi_top)) return GMG_ERR_ARG;
  if (c->ny > 65535 * BY) return GMG_ERR_SHAPE;
  auto a16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  if (c->nx % 2 == 0 && a16(phi_dev) && a16(ex_dev) && a16(ey_dev) && a16(ez_dev) && a16(emag_dev)) {
    const Launch l = cell_launch(c->nx / 2, c->ny, c->nz, 8192, 8);
    GMG_LAUNCH(c, "electric_field", k_electric_field_pair, l, phi_dev, c->L.shapes[0].geom(), c->hx, c->hy, c->hz,
               phi_bot, phi_top, ex_dev, ey_dev, ez_dev, emag_dev, l.kc);
  } else {
    const Launch l = cell_launch(c->nx, c->ny, c->nz, 8192, 8);
    GMG_LAUNCH(c, "electric_field", k_electric_field, l, phi_dev, c->L.shapes[0].geom(), c->hx, c->hy, c->hz,
               phi_bot, phi_top, ex_dev, ey_dev, ez_dev, emag_dev, l.kc);
  }
  return GMG_OK;
}

int wait_stream(gmg_ctx* c) {
  note(c, hipStreamSynchronize(c->stream));
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

}  // namespace

int gmg_assemble_elliptic(gmg_ctx* c, const double* ne_dev, const double* np_dev, const gmg_step_params* prm,
                          double* a_dev, double* f_dev) {
  if (!valid_ctx(c)) return GMG_ERR_ARG;
  const int st = launch_assemble(c, ne_dev, np_dev, prm, a_dev, f_dev);
  return st != GMG_OK ? st : wait_stream(c);
}

int gmg_electric_field(gmg_ctx* c, const double* phi_dev, double phi_bot, double phi_top, double* ex_dev,
                       double* ey_dev, double* ez_dev, double* emag_dev) {
  if (!valid_ctx(c)) return GMG_ERR_ARG;
  const int st = launch_field(c, phi_dev, phi_bot, phi_top, ex_dev, ey_dev, ez_dev, emag_dev);
  return st != GMG_OK ? st : wait_stream(c);
}

int gmg_elliptic_step(gmg_ctx* c, const double* ne_dev, const double* np_dev, const gmg_step_params* prm,
                      double phi_bot, double phi_top, double tol, double* a_dev, double* f_dev, double* phi_dev,
                      int use_x0, double* ex_dev, double* ey_dev, double* ez_dev, double* emag_dev, int* iterations,
                      double* final_true_relres) {
  if (!valid_ctx(c) || !phi_dev || !ex_dev || !ey_dev || !ez_dev || !emag_dev) return GMG_ERR_ARG;
  if (!std::isfinite(phi_bot) || !std::isfinite(phi_top) || !(tol >= 0.0)) return GMG_ERR_ARG;
  int st = launch_assemble(c, ne_dev, np_dev, prm, a_dev, f_dev);
  if (st != GMG_OK) return st;
  st = gmg_update_coefficient(c, a_dev);
  if (st != GMG_OK) return st;
  const int solved = fgmres_solve(c, f_dev, phi_bot, phi_top, tol, phi_dev, use_x0, iterations, nullptr, 0, nullptr,
                                  final_true_relres);
  if (solved < 0) return solved;
  st = launch_field(c, phi_dev, phi_bot, phi_top, ex_dev, ey_dev, ez_dev, emag_dev);
  if (st != GMG_OK) return st;
  st = wait_stream(c);
  return st != GMG_OK ? st : solved;
}

int gmg_density_update(gmg_ctx* c, const double* ne_dev, const double* np_dev, const double* le_dev,
                       const double* lp_dev, double dt, double* ne_out, double* np_out) {
  if (!valid_ctx(c) || !ne_dev || !np_dev || !le_dev || !lp_dev || !ne_out || !np_out) return GMG_ERR_ARG;
  if (!std::isfinite(dt)) return GMG_ERR_ARG;
  GMG_LAUNCH(c, "density_update", k_density_update, flat_launch(c->N), ne_dev, np_dev, le_dev, lp_dev, dt, ne_out,
             np_out, c->N);
  return wait_stream(c);
}

int gmg_get_levels(gmg_ctx* c, int* nlevels, int* shapes, int cap) {
  if (!valid_ctx(c) || !nlevels) return GMG_ERR_ARG;
  *nlevels = (int)c->L.shapes.size();
  for (int l = 0; l < std::min(cap, *nlevels); ++l) {
    shapes[3 * l] = c->L.shapes[l].nx;
    shapes[3 * l + 1] = c->L.shapes[l].ny;
    shapes[3 * l + 2] = c->L.shapes[l].nz;
  }
  return GMG_OK;
}

int gmg_profile_enable(gmg_ctx* c, int enable) {
  if (!valid_ctx(c)) return GMG_ERR_ARG;
  c->prof.on = enable != 0;
  return GMG_OK;
}

static void profile_collect(gmg_ctx* c) {
  note(c, hipStreamSynchronize(c->stream));
  for (auto& r : c->prof.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& t = c->prof.totals[r.name];
      t.first += ms;
      t.second += 1;
      c->prof.names[r.name] = r.name;
    }
    c->prof.pool.push_back(r.a);
    c->prof.pool.push_back(r.b);
  }
  c->prof.pending.clear();
}

int gmg_profile_reset(gmg_ctx* c) {
  if (!valid_ctx(c)) return GMG_ERR_ARG;
  profile_collect(c);
  c->prof.totals.clear();
  return GMG_OK;
}

int gmg_profile_read(gmg_ctx* c, const char** names, double* total_ms, long long* launches, int cap, int* count) {
  if (!valid_ctx(c) || !count) return GMG_ERR_ARG;
  profile_collect(c);
  int i = 0;
  for (auto& kv : c->prof.totals) {
    if (i < cap) {
      if (names) names[i] = c->prof.names[kv.first];
      if (total_ms) total_ms[i] = kv.second.first;
      if (launches) launches[i] = kv.second.second;
    }
    ++i;
  }
  *count = i;
  return c->err == hipSuccess ? GMG_OK : GMG_ERR_HIP;
}

void gmg_destroy(gmg_ctx* c) {
  if (!c) return;
  if (c->prof.on || !c->prof.pending.empty()) (void)hipStreamSynchronize(c->stream);
  for (auto& r : c->prof.pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

const char* gmg_status_string(int s) {
  switch (s) {
    case GMG_OK: return "ok";
    case GMG_NOT_CONVERGED: return "not converged within max_iter Arnoldi steps";
    case GMG_ERR_ARG: return "invalid argument (null pointer, bad option, non-positive coefficient or tolerance)";
    case GMG_ERR_SHAPE: return "grid does not coarsen to at most coarse_max_cells cells";
    case GMG_ERR_NONFINITE: return "non-finite value in the coefficient, right side, initial guess or iteration";
    case GMG_ERR_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case GMG_ERR_HIP: return "HIP runtime error";
    case GMG_ERR_BREAKDOWN: return "breakdown: zero denominator in the Krylov recurrences";
    default: return "unknown status";
  }
}

}  // extern "C"
