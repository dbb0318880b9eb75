"""The C-ABI library loads and exports every entry point of include/gmg.h;
host-only calls behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmg.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"sizeof"})


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    from paper_1812_08606_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert "fgmres_solve" in names and "gmg_setup" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(__import__("paper_1812_08606_amd._lib", fromlist=["x"]).SIGNATURES)


def test_default_options_and_workspace(lib):
    from paper_1812_08606_amd._lib import Options
    opt = Options()
    lib.gmg_default_options(ctypes.byref(opt))
    assert (opt.restart, opt.max_iter, opt.nu_pre, opt.nu_post, opt.precision, opt.coarse_max_cells,
            opt.fine_sweep, opt.cold_cycle, opt.graphs) == (10, 200, 2, 2, 1, 4096, 0, 1, 0)
    n64 = lib.gmg_workspace_bytes(64, 64, 64, ctypes.byref(opt))
    N = 64 ** 3
    # 11 float64 Krylov vectors + 10 float32 preconditioned vectors dominate
    assert 11 * N * 8 + 10 * N * 4 < n64 < 11 * N * 8 + 10 * N * 4 + 4 * N * 8
    assert lib.gmg_workspace_bytes(100, 100, 100, ctypes.byref(opt)) == 0  # 25^3 coarsest
    assert lib.gmg_workspace_bytes(0, 4, 4, ctypes.byref(opt)) == 0
    opt.restart = 0
    assert lib.gmg_workspace_bytes(64, 64, 64, ctypes.byref(opt)) == 0
    opt.restart = 10
    opt.fine_sweep = 3
    assert lib.gmg_workspace_bytes(64, 64, 64, ctypes.byref(opt)) == 0
    opt.fine_sweep = 2
    assert lib.gmg_workspace_bytes(64, 64, 64, ctypes.byref(opt)) == n64
    opt.fine_sweep = 0
    opt.precision = 0
    assert lib.gmg_workspace_bytes(64, 64, 64, ctypes.byref(opt)) > n64


def test_status_strings(lib):
    for s in (0, 1, -1, -2, -3, -4, -5, -6, 99):
        assert lib.gmg_status_string(s)


def test_null_arguments_rejected(lib):
    from paper_1812_08606_amd._lib import Options
    opt = Options()
    lib.gmg_default_options(ctypes.byref(opt))
    out = ctypes.c_void_p()
    assert lib.gmg_setup(8, 8, 8, 0.1, 0.1, 0.1, None, ctypes.byref(opt), None, 0, None,
                         ctypes.byref(out)) == -1
    assert lib.fgmres_solve(None, None, 0.0, 1.0, 1e-8, None, 0, None, None, 0, None, None) == -1
    assert lib.gmg_krylov_solve(None, 2, None, 0.0, 1.0, 1e-8, None, 0, None, None, None) == -1
    assert lib.gmg_assemble_elliptic(None, None, None, None, None, None) == -1
    assert lib.gmg_electric_field(None, None, 0.0, 1.0, None, None, None, None) == -1
    assert lib.gmg_fmg(None, None, None) == -1
