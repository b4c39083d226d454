"""Vertically implicit diffusion (vertically implicit time-discretisation
paragraph of the time-stepping appendix: the tracer-time-discretisation
equation and its momentum counterpart for the predictor velocity).

Given the explicit update x~ of a substage that spans dt_eff, the new value
solves, column by column,

    (1 - dt_eff d/dz K d/dz) x = x~,

with the second-order discretisation of the vertical diffusion operator:

* cell-centred fields (u, v, tracers; K = nu or kappa):
    (L x)_k = [K (x_{k+1} - x_k)/dzf_{k+1} - K (x_k - x_{k-1})/dzf_k] / dzc_k,
  no diffusive flux through the walls (the prescribed top flux of a tracer
  is part of the explicit tendency);
* w on the z faces (K = nu), unknowns on the interior faces 1..nz-1:
    (L w)_k = [K (w_{k+1} - w_k)/dzc_k - K (w_k - w_{k-1})/dzc_{k-1}] / dzf_k,
  with w = 0 on the wall faces.

Reading: for an RK3 substage dt_eff = (gamma_m - zeta_m) dt, the fraction
of the step the substage spans.  The systems are solved with a banded
(tridiagonal) library solver.
"""
import numpy as np
import scipy.linalg as sla

from .fv import z_spacings


def centred_bands(ph, K, dt_eff):
    """Bands (sub, diag, sup) of 1 - dt_eff L for cell-centred fields."""
    dzc, dzf = z_spacings(ph)
    nz = ph.nz
    lo = np.zeros(nz)
    up = np.zeros(nz)
    lo[1:] = K / (dzc[1:] * dzf[1:nz])
    up[:-1] = K / (dzc[:-1] * dzf[1:nz])
    return -dt_eff * lo, 1.0 + dt_eff * (lo + up), -dt_eff * up


def face_bands(ph, K, dt_eff):
    """Bands of 1 - dt_eff L for w on the interior faces 1..nz-1."""
    dzc, dzf = z_spacings(ph)
    nz = ph.nz
    k = np.arange(1, nz)
    lo = K / (dzc[k - 1] * dzf[k])      # couples to w_{k-1} (0 at face 1's wall)
    up = K / (dzc[k] * dzf[k])          # couples to w_{k+1} (0 at face nz-1's wall)
    sub = -dt_eff * lo
    sup = -dt_eff * up
    sub[0] = 0.0
    sup[-1] = 0.0
    return sub, 1.0 + dt_eff * (lo + up), sup


def _solve_columns(x, sub, diag, sup):
    """Solve the tridiagonal system along axis 0 for every column of x."""
    n = x.shape[0]
    ab = np.zeros((3, n))
    ab[0, 1:] = sup[:-1]
    ab[1, :] = diag
    ab[2, :-1] = sub[1:]
    flat = x.reshape(n, -1)
    return sla.solve_banded((1, 1), ab, flat).reshape(x.shape)


def implicit_diffusion(name, x, ph, dt_eff):
    """x^{new} from the explicit update x~ (an interior array) of field `name`."""
    assert ph.z_bounded
    if name == "w":
        K = ph.nu
        out = x.copy()
        sub, diag, sup = face_bands(ph, K, dt_eff)
        out[1:ph.nz] = _solve_columns(x[1:ph.nz], sub, diag, sup)
        out[0] = 0.0
        out[ph.nz] = 0.0
        return out
    K = ph.nu if name in ("u", "v") else ph.kappa
    sub, diag, sup = centred_bands(ph, K, dt_eff)
    return _solve_columns(x, sub, diag, sup)
