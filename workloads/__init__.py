"""Seeded synthetic inputs shaped like the paper's streamer workloads.

This module only draws coefficient and source fields; it holds none of the
solver's arithmetic.  Both the CPU oracle's tests and the GPU path's tests and
benchmark take their inputs from here, so the two sides always see the same
numbers.

Geometry follows the paper's test problems (Sec. 5.2 and Sec. 6): the unit
cube between two plates at z=0 and z=1, a charged filament along the z axis
(the Gaussian seeds of eq. eq51 and of the two-streamer application).  The
coefficient stands for the discrete P of Sec. 2.2, a = 1 + kappa * n_e, and the
source for the right side of eq. e18, f = 50 (n_p - n_e).

Fields are float64 arrays of shape (nz, ny, nx), C order, x fastest; cell i
has centre (i + 1/2) h.  Random numbers come from numpy's PCG64 seeded with
``SEED_BASE + config_number``.
"""
from .streamer import (  # noqa: F401
    SEED_BASE,
    Problem,
    cell_centres,
    smoothstep_window,
    config_gaussian_source,
    config_filament,
    config_two_filaments,
    config_streamer_mesh,
    probe_box_mask,
    make_config,
    CONFIG_SIZES,
)
