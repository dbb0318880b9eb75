"""Python binding of the C ABI (include/gmg.h): argument marshalling only.

PyTorch provides device memory (the caller's tensors and the solver's
workspace) and the stream; every step of the solve runs in the HIP library.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib

FP64, MIXED = 0, 1
_PRECISION = {"fp64": FP64, "mixed": MIXED}
_FINE_SWEEP = {"auto": 0, "half": 1, "fused": 2}
_COLD_CYCLE = {"vcycle": 0, "fmg": 1}
_SMOOTHER = {"rbgs": 0, "chebyshev": 1}
_RESTRICTION = {"mean": 0, "transpose": 1}
OK, NOT_CONVERGED = 0, 1


class GMGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.load().gmg_status_string(status).decode()
        super().__init__(f"{where}: status {status}: {msg}")


@dataclass
class SolveResult:
    phi: torch.Tensor
    status: int
    iterations: int
    res_hist: list = field(default_factory=list)
    final_relres: float = float("nan")

    @property
    def converged(self) -> bool:
        return self.status == OK


def _check_field(t: torch.Tensor, shape, name: str, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device, got {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the solver on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class GMGPoisson:
    """Hierarchy and workspace for -div(a grad phi) = f on a (nz, ny, nx) grid
    (eq. e18), solved by FGMRES(restart) with one V-cycle per step.

    a: float64 CUDA/HIP tensor (nz, ny, nx), > 0.  h: (hx, hy, hz), default
    unit cube.  precision: "mixed" (float32 V-cycle) or "fp64".  fine_sweep:
    Gauss-Seidel smoother kernels, "half" (one per half-sweep), "fused" (one
    per symmetric sweep on the finest level and the coarse levels that allow
    it) or "auto" (fused where it was measured faster).  cold_cycle: preconditioner
    of a solve without an initial guess, "fmg" (full multigrid, the default)
    or "vcycle"; warm_cycle: the same for a warm-started solve, "vcycle"
    (the paper's choice, the default) or "fmg".  graphs: replay each
    preconditioner application from a captured HIP graph (same results).
    smoother: "rbgs" (red-black symmetric Gauss-Seidel, nu_pre / nu_post
    sweeps) or "chebyshev" (the degree-2 Chebyshev polynomial in the
    SSOR-preconditioned level operator, Sec. 3.2 eq. qntn, nu_pre / nu_post
    applications, default 1 each; V-cycles only, so cold_cycle defaults to
    "vcycle").  restriction: "mean" (of the 8 children, the default) or
    "transpose" (R = P^T / 8: with nu_pre = nu_post a symmetric V-cycle, for
    the conjugate gradient method; V-cycles only, so cold_cycle defaults to
    "vcycle")."""

    def __init__(self, a: torch.Tensor, h=None, precision: str = "mixed", restart: int = 10,
                 max_iter: int = 200, nu_pre: int | None = None, nu_post: int | None = None,
                 coarse_max_cells: int = 4096, fine_sweep: str = "auto", cold_cycle: str | None = None,
                 graphs: bool = False, smoother: str = "rbgs", warm_cycle: str = "vcycle",
                 restriction: str = "mean"):
        self._lib = _lib.load()
        if a.dim() != 3:
            raise ValueError("a must be 3-D (nz, ny, nx)")
        self.shape = tuple(a.shape)
        nz, ny, nx = self.shape
        _check_field(a, self.shape, "a")
        self.device = a.device
        self.h = tuple(float(v) for v in (h if h is not None else (1.0 / nx, 1.0 / ny, 1.0 / nz)))
        if precision not in _PRECISION:
            raise ValueError(f"precision must be one of {sorted(_PRECISION)}")
        self.precision = precision
        if fine_sweep not in _FINE_SWEEP:
            raise ValueError(f"fine_sweep must be one of {sorted(_FINE_SWEEP)}")
        if smoother not in _SMOOTHER:
            raise ValueError(f"smoother must be one of {sorted(_SMOOTHER)}")
        cheb = smoother == "chebyshev"
        if restriction not in _RESTRICTION:
            raise ValueError(f"restriction must be one of {sorted(_RESTRICTION)}")
        vonly = cheb or restriction == "transpose"
        if cold_cycle is None:
            cold_cycle = "vcycle" if vonly else "fmg"
        if nu_pre is None:
            nu_pre = 1 if cheb else 2
        if nu_post is None:
            nu_post = 1 if cheb else 2
        self.smoother = smoother
        if cold_cycle not in _COLD_CYCLE:
            raise ValueError(f"cold_cycle must be one of {sorted(_COLD_CYCLE)}")
        if warm_cycle not in _COLD_CYCLE:
            raise ValueError(f"warm_cycle must be one of {sorted(_COLD_CYCLE)}")
        if cheb and (cold_cycle == "fmg" or warm_cycle == "fmg"):
            raise ValueError("the Chebyshev smoother runs V-cycles only (cold_cycle = warm_cycle = 'vcycle')")
        if restriction == "transpose" and (cheb or cold_cycle == "fmg" or warm_cycle == "fmg"):
            raise ValueError("the transpose restriction runs red-black V-cycles only "
                             "(smoother = 'rbgs', cold_cycle = warm_cycle = 'vcycle')")
        opt = _lib.Options()
        self._lib.gmg_default_options(ctypes.byref(opt))
        opt.restart, opt.max_iter = int(restart), int(max_iter)
        opt.nu_pre, opt.nu_post = int(nu_pre), int(nu_post)
        opt.precision = _PRECISION[precision]
        opt.coarse_max_cells = int(coarse_max_cells)
        opt.fine_sweep = _FINE_SWEEP[fine_sweep]
        opt.cold_cycle = _COLD_CYCLE[cold_cycle]
        opt.graphs = int(bool(graphs))
        opt.smoother = _SMOOTHER[smoother]
        opt.warm_cycle = _COLD_CYCLE[warm_cycle]
        opt.restriction = _RESTRICTION[restriction]
        self.options = opt
        nbytes = self._lib.gmg_workspace_bytes(nx, ny, nz, ctypes.byref(opt))
        if nbytes == 0:
            raise GMGError(-2, "gmg_workspace_bytes")
        self.workspace_bytes = int(nbytes)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self._ws = raw[off:off + nbytes]
        self._a = a
        self._stream = None
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            st = self._lib.gmg_setup(nx, ny, nz, *self.h, _ptr(a), ctypes.byref(opt),
                                     _ptr(self._ws), ctypes.c_size_t(nbytes),
                                     ctypes.c_void_p(stream), ctypes.byref(self._ctx))
        if st != OK:
            self._ctx = ctypes.c_void_p()
            raise GMGError(st, "gmg_setup")
        self._stream = stream

    # -- plumbing ---------------------------------------------------------
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            self._lib.gmg_set_stream(self._ctx, ctypes.c_void_p(s))
            self._stream = s

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            self._lib.gmg_destroy(ctx)
            self._ctx = ctypes.c_void_p()

    close = __del__

    def chebyshev_estimates(self):
        """Arnoldi estimate lambda of each smoothed level (Chebyshev smoother;
        the bounds of eq. qntn are 0.1 and 1.1 lambda)."""
        n = ctypes.c_int()
        out = (ctypes.c_double * 64)()
        st = self._lib.gmg_chebyshev_estimates(self._ctx, out, 64, ctypes.byref(n))
        if st != OK:
            raise GMGError(st, "gmg_chebyshev_estimates")
        return [out[i] for i in range(min(n.value, 64))]

    @property
    def levels(self):
        n = ctypes.c_int()
        shapes = (ctypes.c_int * 96)()
        self._lib.gmg_get_levels(self._ctx, ctypes.byref(n), shapes, 32)
        return [tuple(shapes[3 * i:3 * i + 3]) for i in range(min(n.value, 32))]

    # -- operations -------------------------------------------------------
    def update_coefficient(self, a: torch.Tensor):
        _check_field(a, self.shape, "a", self.device)
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.gmg_update_coefficient(self._ctx, _ptr(a))
        if st != OK:
            raise GMGError(st, "gmg_update_coefficient")
        self._a = a

    def solve(self, f: torch.Tensor, phi_bot: float = 0.0, phi_top: float = 1.0, tol: float = 1e-8,
              x0: torch.Tensor | None = None, out: torch.Tensor | None = None,
              raise_on_error: bool = True) -> SolveResult:
        _check_field(f, self.shape, "f", self.device)
        if out is None:
            out = torch.empty_like(f)
        _check_field(out, self.shape, "out", self.device)
        use_x0 = 0
        if x0 is not None:
            _check_field(x0, self.shape, "x0", self.device)
            if x0.data_ptr() != out.data_ptr():
                out.copy_(x0)
            use_x0 = 1
        cap = int(self.options.max_iter) + 2
        hist = (ctypes.c_double * cap)()
        its, nh = ctypes.c_int(0), ctypes.c_int(0)
        rel = ctypes.c_double(float("nan"))
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.fgmres_solve(self._ctx, _ptr(f), float(phi_bot), float(phi_top), float(tol),
                                        _ptr(out), use_x0, ctypes.byref(its), hist, cap,
                                        ctypes.byref(nh), ctypes.byref(rel))
        if st < 0 and raise_on_error:
            raise GMGError(st, "fgmres_solve")
        return SolveResult(phi=out, status=st, iterations=its.value,
                           res_hist=list(hist[:nh.value]), final_relres=rel.value)

    def apply(self, x: torch.Tensor, phi_bot: float = 0.0, phi_top: float = 0.0) -> torch.Tensor:
        """A x - lifting (left side of e18 with the given plate values)."""
        _check_field(x, self.shape, "x", self.device)
        y = torch.empty_like(x)
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.gmg_apply_operator(self._ctx, _ptr(x), _ptr(y), float(phi_bot), float(phi_top))
        if st != OK:
            raise GMGError(st, "gmg_apply_operator")
        return y

    def vcycle(self, v: torch.Tensor) -> torch.Tensor:
        """One V-cycle from a zero guess: z = M v."""
        return self._cycle(v, "gmg_vcycle")

    def fmg(self, v: torch.Tensor) -> torch.Tensor:
        """One full multigrid cycle: z = F v."""
        return self._cycle(v, "gmg_fmg")

    def _cycle(self, v: torch.Tensor, entry: str) -> torch.Tensor:
        _check_field(v, self.shape, "v", self.device)
        z = torch.empty_like(v)
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = getattr(self._lib, entry)(self._ctx, _ptr(v), _ptr(z))
        if st != OK:
            raise GMGError(st, entry)
        return z

    KRYLOV = {"fgmres": 0, "gmres": 1, "cg": 2, "fcg": 3, "cgs": 4, "bicgstab": 5}

    def krylov_solve(self, f: torch.Tensor, phi_bot: float, phi_top: float, method: str = "cg",
                     tol: float = 1e-8, x0: torch.Tensor | None = None, out: torch.Tensor | None = None,
                     raise_on_error: bool = True):
        """Solve with one of the Krylov methods of the comparison in Sec. 5.3
        (fgmres, gmres, cg, fcg, cgs, bicgstab), one V-cycle per
        preconditioner application.  Returns (SolveResult, preconditioner
        applications)."""
        if method not in self.KRYLOV:
            raise ValueError(f"method must be one of {sorted(self.KRYLOV)}")
        _check_field(f, self.shape, "f", self.device)
        phi = out if out is not None else torch.empty_like(f)
        _check_field(phi, self.shape, "out", self.device)
        if x0 is not None:
            _check_field(x0, self.shape, "x0", self.device)
            if x0.data_ptr() != phi.data_ptr():
                phi.copy_(x0)
        its, napp, rel = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.gmg_krylov_solve(self._ctx, self.KRYLOV[method], _ptr(f), float(phi_bot),
                                            float(phi_top), float(tol), _ptr(phi), int(x0 is not None),
                                            ctypes.byref(its), ctypes.byref(napp), ctypes.byref(rel))
        if st < 0 and raise_on_error:
            raise GMGError(st, "gmg_krylov_solve")
        return SolveResult(phi=phi, status=st, iterations=its.value, final_relres=rel.value), napp.value

    def assemble_elliptic(self, n_e: torch.Tensor, n_p: torch.Tensor, eps0_over_e: float, tau_eff: float,
                          mu_e: float, mu_p: float, De=(0.0, 0.0, 0.0), out=None):
        """Coefficient a = P and right side f of the elliptic problem of a
        semi-implicit step from the densities (Sec. 2.2, eq. e18); returns
        (a, f), written into ``out`` = (a, f) when given."""
        _check_field(n_e, self.shape, "n_e", self.device)
        _check_field(n_p, self.shape, "n_p", self.device)
        a, f = out if out is not None else (torch.empty_like(n_e), torch.empty_like(n_e))
        _check_field(a, self.shape, "a", self.device)
        _check_field(f, self.shape, "f", self.device)
        prm = _lib.StepParams(float(eps0_over_e), float(tau_eff), float(mu_e), float(mu_p),
                              (ctypes.c_double * 3)(*[float(v) for v in De]))
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.gmg_assemble_elliptic(self._ctx, _ptr(n_e), _ptr(n_p), ctypes.byref(prm), _ptr(a),
                                                 _ptr(f))
        if st != OK:
            raise GMGError(st, "gmg_assemble_elliptic")
        return a, f

    def electric_field(self, phi: torch.Tensor, phi_bot: float, phi_top: float, out=None):
        """E = -grad phi by central differences and |E|: (E_x, E_y, E_z, |E|)."""
        _check_field(phi, self.shape, "phi", self.device)
        outs = out if out is not None else tuple(torch.empty_like(phi) for _ in range(4))
        for o, nm in zip(outs, ("E_x", "E_y", "E_z", "|E|")):
            _check_field(o, self.shape, nm, self.device)
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.gmg_electric_field(self._ctx, _ptr(phi), float(phi_bot), float(phi_top),
                                              *[_ptr(o) for o in outs])
        if st != OK:
            raise GMGError(st, "gmg_electric_field")
        return outs

    def face_flux_grad(self, phi: torch.Tensor, lam: torch.Tensor, phi_bot: float, phi_top: float):
        """dL/da from the solution phi and the adjoint lam."""
        return self.face_flux_grad_into(phi, lam, phi_bot, phi_top, torch.empty_like(phi))

    def face_flux_grad_into(self, phi, lam, phi_bot: float, phi_top: float, out: torch.Tensor):
        _check_field(phi, self.shape, "phi", self.device)
        _check_field(lam, self.shape, "lam", self.device)
        _check_field(out, self.shape, "out", self.device)
        with torch.cuda.device(self.device):
            self._sync_stream()
            st = self._lib.gmg_face_flux_grad(self._ctx, _ptr(phi), _ptr(lam), float(phi_bot),
                                              float(phi_top), _ptr(out))
        if st != OK:
            raise GMGError(st, "gmg_face_flux_grad")
        return out

    # -- profiling --------------------------------------------------------
    def profile(self, enable: bool = True):
        self._lib.gmg_profile_enable(self._ctx, int(bool(enable)))

    def profile_reset(self):
        self._lib.gmg_profile_reset(self._ctx)

    def profile_read(self) -> dict:
        cap = 256
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_longlong * cap)()
        n = ctypes.c_int()
        with torch.cuda.device(self.device):
            self._lib.gmg_profile_read(self._ctx, names, ms, cnt, cap, ctypes.byref(n))
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(min(n.value, cap))}


@dataclass
class StepInfo:
    """Result of SemiImplicitStepper.step: the new densities, the potential
    and field of the step's elliptic solve (phi^{n+1/2}, E^{n+1/2} in the
    second-order scheme; phi^{n+1}, E^{n+1} in the first-order one), and the
    solve's status, iterations and final relative residual."""
    n_e: torch.Tensor
    n_p: torch.Tensor
    phi: torch.Tensor
    E: tuple
    status: int
    iterations: int
    final_relres: float


class SemiImplicitStepper:
    """Time steps of the paper's semi-implicit schemes around the GPU solve
    (Sec. 2.1).  scheme "second" (eqs. e1, e2, semi2): the elliptic problem
    with tau/2 from the densities at t_n gives phi^{n+1/2}, E^{n+1/2} (one
    solve per step, warm-started from the previous step's phi); the
    predictor n^{n+1/2} = n^n + tau/2 L(n^n) and the corrector n^{n+1} = n^n
    + tau L(n^{n+1/2}), both with E^{n+1/2}.  scheme "first" (eqs.
    semi-implicit, e15): tau in the elliptic problem, n^{n+1} = n^n + tau
    L(n^n) with E^{n+1}.

    ``transport(n_e, n_p, E) -> (L_e, L_p)`` is the caller's: the time
    derivatives of the densities (drift, diffusion, source; the paper's MUSCL
    fluxes are not part of this library) for the frozen field E = (E_x, E_y,
    E_z, |E|), as float64 tensors of the grid's shape.  The assembly, solve,
    field and density updates run in the HIP library (gmg_elliptic_step,
    gmg_density_update).

    a: a template float64 (nz, ny, nx) tensor (only its shape and device are
    used); h, precision and the other keyword arguments go to GMGPoisson."""

    def __init__(self, a: torch.Tensor, phi_bot: float, phi_top: float, eps0_over_e: float, mu_e: float,
                 mu_p: float, De=(0.0, 0.0, 0.0), scheme: str = "second", tol: float = 1e-8, h=None, **solver_kw):
        if scheme not in ("second", "first"):
            raise ValueError("scheme must be 'second' or 'first'")
        self.solver = GMGPoisson(torch.ones_like(a), h=h, **solver_kw)
        self._lib = self.solver._lib
        self.shape, self.device = self.solver.shape, self.solver.device
        self.scheme, self.tol = scheme, float(tol)
        self.bc = (float(phi_bot), float(phi_top))
        self.coef = (float(eps0_over_e), float(mu_e), float(mu_p), tuple(float(v) for v in De))
        self.a = torch.empty_like(a)
        self.f = torch.empty_like(a)
        self.phi = torch.zeros_like(a)
        self.E = tuple(torch.empty_like(a) for _ in range(4))
        self._warm = False

    def _update(self, n_e, n_p, l_e, l_p, dt, out_e, out_p):
        for t, nm in ((n_e, "n_e"), (n_p, "n_p"), (l_e, "L_e"), (l_p, "L_p"), (out_e, "out n_e"),
                      (out_p, "out n_p")):
            _check_field(t, self.shape, nm, self.device)
        with torch.cuda.device(self.device):
            self.solver._sync_stream()
            st = self._lib.gmg_density_update(self.solver._ctx, _ptr(n_e), _ptr(n_p), _ptr(l_e), _ptr(l_p),
                                              float(dt), _ptr(out_e), _ptr(out_p))
        if st != OK:
            raise GMGError(st, "gmg_density_update")

    def step(self, n_e: torch.Tensor, n_p: torch.Tensor, tau: float, transport, out=None) -> StepInfo:
        """One time step from (n_e, n_p) at t_n; the new densities go to
        ``out`` = (n_e, n_p) when given (may be the inputs), else to new
        tensors.  phi and E of the result are the stepper's buffers,
        overwritten by the next step."""
        _check_field(n_e, self.shape, "n_e", self.device)
        _check_field(n_p, self.shape, "n_p", self.device)
        eps, mu_e, mu_p, De = self.coef
        tau_eff = 0.5 * tau if self.scheme == "second" else tau
        prm = _lib.StepParams(eps, float(tau_eff), mu_e, mu_p, (ctypes.c_double * 3)(*De))
        its = ctypes.c_int(0)
        rel = ctypes.c_double(float("nan"))
        with torch.cuda.device(self.device):
            self.solver._sync_stream()
            st = self._lib.gmg_elliptic_step(self.solver._ctx, _ptr(n_e), _ptr(n_p), ctypes.byref(prm), *self.bc,
                                             self.tol, _ptr(self.a), _ptr(self.f), _ptr(self.phi),
                                             int(self._warm), *[_ptr(e) for e in self.E], ctypes.byref(its),
                                             ctypes.byref(rel))
        if st < 0:
            raise GMGError(st, "gmg_elliptic_step")
        self.solver._a = self.a  # the context keeps the coefficient's pointer
        self._warm = True
        oe, op = out if out is not None else (torch.empty_like(n_e), torch.empty_like(n_p))
        l_e, l_p = transport(n_e, n_p, self.E)
        if self.scheme == "first":
            self._update(n_e, n_p, l_e, l_p, tau, oe, op)
        else:
            he, hp = torch.empty_like(n_e), torch.empty_like(n_p)
            self._update(n_e, n_p, l_e, l_p, 0.5 * tau, he, hp)  # predictor (eq. e1)
            l_e, l_p = transport(he, hp, self.E)
            self._update(n_e, n_p, l_e, l_p, tau, oe, op)  # corrector (eq. e2)
        return StepInfo(oe, op, self.phi, self.E, st, its.value, rel.value)


STATIC_SCRATCH_BYTES = 64 << 20  # GMG_STATIC_SCRATCH_BYTES of include/gmg.h


def fgmres_solve_static(a: torch.Tensor, f: torch.Tensor, phi_bot: float, phi_top: float, tol: float,
                        out: torch.Tensor, h=None, x0: torch.Tensor | None = None, precision: str = "mixed",
                        **options) -> SolveResult:
    """fgmres_solve_static of the C ABI: hierarchy set-up and FGMRES solve in
    one call, on the device array the library holds per GPU (it allocates no
    device memory; the grid's workspace must fit STATIC_SCRATCH_BYTES, else
    GMGError with status -4).  out: the caller's phi (float64, a's shape);
    x0: initial guess (copied into out first).  options: integer fields of
    gmg_options by name (restart, max_iter, nu_pre, nu_post, fine_sweep,
    cold_cycle, smoother, warm_cycle, restriction, ...), on top of
    gmg_default_options."""
    lib = _lib.load()
    shape = tuple(a.shape)
    if len(shape) != 3:
        raise ValueError("a must be 3-D (nz, ny, nx)")
    nz, ny, nx = shape
    for t, name in ((a, "a"), (f, "f"), (out, "out")):
        _check_field(t, shape, name, a.device)
    if precision not in _PRECISION:
        raise ValueError(f"precision must be one of {sorted(_PRECISION)}")
    opt = _lib.Options()
    lib.gmg_default_options(ctypes.byref(opt))
    opt.precision = _PRECISION[precision]
    names = {fld[0] for fld in _lib.Options._fields_}
    for k, v in options.items():
        if k not in names or k == "precision":
            raise ValueError(f"unknown option {k}")
        setattr(opt, k, int(v))
    hh = tuple(float(v) for v in (h if h is not None else (1.0 / nx, 1.0 / ny, 1.0 / nz)))
    if x0 is not None:
        _check_field(x0, shape, "x0", a.device)
        if x0.data_ptr() != out.data_ptr():
            out.copy_(x0)
    cap = int(opt.max_iter) + 2
    hist = (ctypes.c_double * cap)()
    its, nh = ctypes.c_int(0), ctypes.c_int(0)
    rel = ctypes.c_double(float("nan"))
    with torch.cuda.device(a.device):
        stream = torch.cuda.current_stream(a.device).cuda_stream
        st = lib.fgmres_solve_static(nx, ny, nz, *hh, _ptr(a), ctypes.byref(opt), ctypes.c_void_p(stream), _ptr(f),
                                     float(phi_bot), float(phi_top), float(tol), _ptr(out), int(x0 is not None),
                                     ctypes.byref(its), hist, cap, ctypes.byref(nh), ctypes.byref(rel))
    if st < 0:
        raise GMGError(st, "fgmres_solve_static")
    return SolveResult(phi=out, status=st, iterations=its.value, res_hist=list(hist[:nh.value]),
                       final_relres=rel.value)


class _PoissonSolve(torch.autograd.Function):
    """phi = A(a)^{-1} (f + lifting(a)); the backward solves the adjoint with
    the same (self-adjoint) operator and hierarchy: lambda = A^{-1} dL/dphi,
    dL/df = lambda, dL/da from the face products of grad phi and grad lambda."""

    @staticmethod
    def forward(ctx, f, a, phi_bot, phi_top, tol, precision, kwargs):
        solver = GMGPoisson(a.detach(), precision=precision, **kwargs)
        res = solver.solve(f.detach().contiguous(), phi_bot, phi_top, tol)
        if res.status != OK:
            raise GMGError(res.status, "poisson_solve forward")
        ctx.solver = solver
        ctx.bc = (float(phi_bot), float(phi_top))
        ctx.tol = tol
        ctx.iterations = res.iterations
        ctx.save_for_backward(res.phi)
        return res.phi

    @staticmethod
    def backward(ctx, grad_phi):
        (phi,) = ctx.saved_tensors
        solver = ctx.solver
        adj = solver.solve(grad_phi.contiguous(), 0.0, 0.0, ctx.tol)
        if adj.status != OK:
            raise GMGError(adj.status, "poisson_solve backward (adjoint)")
        lam = adj.phi
        dLda = solver.face_flux_grad(phi, lam, *ctx.bc) if ctx.needs_input_grad[1] else None
        dLdf = lam if ctx.needs_input_grad[0] else None
        return dLdf, dLda, None, None, None, None, None


def poisson_solve(f: torch.Tensor, a: torch.Tensor, phi_bot: float = 0.0, phi_top: float = 1.0,
                  tol: float = 1e-8, precision: str = "mixed", **kwargs) -> torch.Tensor:
    """Differentiable solve of e18: returns phi; gradients flow to f and a."""
    return _PoissonSolve.apply(f, a, phi_bot, phi_top, tol, precision, kwargs)
