"""ctypes loader of libgmg.so (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmg.so")

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
P_int = ctypes.POINTER(c_int)
P_double = ctypes.POINTER(c_double)


class Options(ctypes.Structure):
    _fields_ = [
        ("restart", c_int),
        ("max_iter", c_int),
        ("nu_pre", c_int),
        ("nu_post", c_int),
        ("precision", c_int),
        ("coarse_max_cells", c_int),
        ("fine_sweep", c_int),
        ("cold_cycle", c_int),
        ("graphs", c_int),
        ("smoother", c_int),
        ("warm_cycle", c_int),
        ("restriction", c_int),
    ]


class StepParams(ctypes.Structure):
    _fields_ = [
        ("eps0_over_e", c_double),
        ("tau_eff", c_double),
        ("mu_e", c_double),
        ("mu_p", c_double),
        ("De", c_double * 3),
    ]


SIGNATURES = {
    "gmg_default_options": (None, [ctypes.POINTER(Options)]),
    "gmg_workspace_bytes": (c_size_t, [c_int, c_int, c_int, ctypes.POINTER(Options)]),
    "gmg_setup": (c_int, [c_int, c_int, c_int, c_double, c_double, c_double, c_void_p,
                          ctypes.POINTER(Options), c_void_p, c_size_t, c_void_p,
                          ctypes.POINTER(c_void_p)]),
    "gmg_update_coefficient": (c_int, [c_void_p, c_void_p]),
    "gmg_set_stream": (c_int, [c_void_p, c_void_p]),
    "fgmres_solve": (c_int, [c_void_p, c_void_p, c_double, c_double, c_double, c_void_p, c_int,
                             P_int, P_double, c_int, P_int, P_double]),
    "fgmres_solve_static": (c_int, [c_int, c_int, c_int, c_double, c_double, c_double, c_void_p,
                                    ctypes.POINTER(Options), c_void_p, c_void_p, c_double, c_double, c_double,
                                    c_void_p, c_int, P_int, P_double, c_int, P_int, P_double]),
    "gmg_krylov_solve": (c_int, [c_void_p, c_int, c_void_p, c_double, c_double, c_double, c_void_p, c_int,
                                 P_int, P_int, P_double]),
    "gmg_apply_operator": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double]),
    "gmg_vcycle": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmg_fmg": (c_int, [c_void_p, c_void_p, c_void_p]),
    "gmg_face_flux_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_void_p]),
    "gmg_assemble_elliptic": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(StepParams), c_void_p,
                                      c_void_p]),
    "gmg_electric_field": (c_int, [c_void_p, c_void_p, c_double, c_double, c_void_p, c_void_p, c_void_p,
                                   c_void_p]),
    "gmg_elliptic_step": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(StepParams), c_double, c_double,
                                  c_double, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                                  c_void_p, P_int, P_double]),
    "gmg_density_update": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                   c_void_p]),
    "gmg_get_levels": (c_int, [c_void_p, P_int, P_int, c_int]),
    "gmg_chebyshev_estimates": (c_int, [c_void_p, P_double, c_int, P_int]),
    "gmg_ritz_max_real": (c_int, [P_double, c_int, c_int, P_double]),
    "gmg_profile_enable": (c_int, [c_void_p, c_int]),
    "gmg_profile_reset": (c_int, [c_void_p]),
    "gmg_profile_read": (c_int, [c_void_p, ctypes.POINTER(ctypes.c_char_p), P_double,
                                 ctypes.POINTER(ctypes.c_longlong), c_int, P_int]),
    "gmg_destroy": (None, [c_void_p]),
    "gmg_status_string": (ctypes.c_char_p, [c_int]),
}

_LIB = None


def load():
    """Load the HIP library; raises ImportError if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1812_08606_amd/build.py` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(lib, name):
            raise ImportError(f"{LIB_PATH} does not export {name} (built from older sources): "
                              "rebuild it with `python paper_1812_08606_amd/build.py`")
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
