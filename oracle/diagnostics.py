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


def momentum_integrals(state, ph):
    """Volume integrals of u, v and w over their own control volumes: u and v
    faces carry the volume of the cell they sit beside in z (dx dy dzc[k]), a
    w face the volume dx dy dzf[k] between the centres either side of it
    (finite-volume appendix: the discrete integral is the sum of value times
    control volume)."""
    dx, dy, _ = ph.spacing
    dzc, dzf = z_spacings(ph)
    u = interior(state["u"], ph, "u")
    v = interior(state["v"], ph, "v")
    w = interior(state["w"], ph, "w")
    nwf = w.shape[0]
    return (float(np.sum(u * dzc[:, None, None])) * dx * dy,
            float(np.sum(v * dzc[:, None, None])) * dx * dy,
            float(np.sum(w * dzf[:nwf, None, None])) * dx * dy)


def cfl_rate(state, ph):
    """The advective CFL number per unit time step, max(max|u|/dx,
    max|v|/dy, max|w|/dz_min): cfl(state, dt, ph) = dt * cfl_rate(state, ph)."""
    return cfl(state, 1.0, ph)
