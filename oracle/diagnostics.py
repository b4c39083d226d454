"""Global diagnostics in FP64: volume integrals of tracers and momentum,
the divergence measure and the advective CFL number.

The integral of a finite-volume field is the volume-weighted sum of its cell
values (finite-volume appendix, discrete integral identity).
"""
import numpy as np

from .fv import interior, z_spacings
from .pressure import divergence


def volume_integral(field_interior, ph):
    dx, dy, _ = ph.spacing
    dzc, _ = z_spacings(ph)
    return float(np.sum(field_interior * dzc[:, None, None])) * dx * dy


def max_abs_divergence(state, ph):
    u = interior(state["u"], ph, "u")
    v = interior(state["v"], ph, "v")
    w = interior(state["w"], ph, "w")
    return float(np.max(np.abs(divergence(u, v, w, ph))))


def scaled_divergence(state, ph):
    """max|div u| * min(spacing) / max|u|: dimensionless, 0 for an exactly
    divergence-free field."""
    vmax = max(float(np.max(np.abs(interior(state[n], ph, n)))) for n in ("u", "v", "w"))
    hmin = min(ph.spacing[0], ph.spacing[1], float(np.min(z_spacings(ph)[0])))
    return max_abs_divergence(state, ph) * hmin / max(vmax, 1e-300)


def cfl(state, dt, ph):
    dx, dy, _ = ph.spacing
    dzc, _ = z_spacings(ph)
    return dt * max(float(np.max(np.abs(interior(state["u"], ph, "u")))) / dx,
                    float(np.max(np.abs(interior(state["v"], ph, "v")))) / dy,
                    float(np.max(np.abs(interior(state["w"], ph, "w")))) / float(np.min(dzc)))
