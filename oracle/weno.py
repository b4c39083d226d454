"""Reconstruction of interface values (reconstruction subsection of the
finite-volume appendix).

Conventions: the interface sits between cells i-1 and i (x_{i-1/2}).  For a
positive advecting velocity the five upwind cells are (a, b, c, d, e) =
(q_{i-3}, q_{i-2}, q_{i-1}, q_i, q_{i+1}); for a negative one the mirrored
set (q_{i+2}, q_{i+1}, q_i, q_{i-1}, q_{i-2}).

Fifth-order WENO combines three shifted third-order upwind stencils with
weights that tend to (1/10, 6/10, 3/10) for smooth data (so that the
combination becomes fifth-order upwind) and favour the smoothest stencil near
jumps.  The printed shifted stencils of the paper's fifth-order WENO equation
are garbled (two of the three have their coefficients reversed and do not
evaluate at x_{i-1/2}); the paper's own third-order upwind equation fixes the
central stencil as (-c_{i-2} + 5 c_{i-1} + 2 c_i)/6, and the three candidates
below are the standard left-biased ones of Jiang & Shu (1996).  The paper
names WENO-Z for the weights; we use the WENO-Z weights of Borges et al.
(2008) with tau = |beta_0 - beta_2|, exponent q and regulariser eps passed in.
"""
import numpy as np

IDEAL = (0.1, 0.6, 0.3)


def candidates(a, b, c, d, e):
    """Three third-order reconstructions at the interface."""
    r0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    r1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    r2 = (2.0 * c + 5.0 * d - e) / 6.0
    return r0, r1, r2


def smoothness(a, b, c, d, e):
    """Jiang-Shu smoothness indicators of the three candidate stencils."""
    b0 = 13.0 / 12.0 * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    return b0, b1, b2


def weno5z(a, b, c, d, e, eps=1e-15, q=2):
    """WENO-Z reconstruction from five upwind-ordered values."""
    r0, r1, r2 = candidates(a, b, c, d, e)
    b0, b1, b2 = smoothness(a, b, c, d, e)
    tau = np.abs(b0 - b2)
    a0 = IDEAL[0] * (1.0 + (tau / (b0 + eps)) ** q)
    a1 = IDEAL[1] * (1.0 + (tau / (b1 + eps)) ** q)
    a2 = IDEAL[2] * (1.0 + (tau / (b2 + eps)) ** q)
    s = a0 + a1 + a2
    return (a0 * r0 + a1 * r1 + a2 * r2) / s


def weno5_linear(a, b, c, d, e):
    """The ideal-weight limit: fifth-order upwind reconstruction."""
    r0, r1, r2 = candidates(a, b, c, d, e)
    return IDEAL[0] * r0 + IDEAL[1] * r1 + IDEAL[2] * r2


def upwind1(qm1, q0, vel):
    """First-order upwind interface value (upwind-biased equation)."""
    return np.where(vel > 0, qm1, q0)


def upwind3(qm2, qm1, q0, qp1, vel):
    """Third-order upwind interface value (upwind-biased equation)."""
    pos = (-qm2 + 5.0 * qm1 + 2.0 * q0) / 6.0
    neg = (2.0 * qm1 + 5.0 * q0 - qp1) / 6.0
    return np.where(vel > 0, pos, neg)


def reconstruct(scheme, qs, vel, eps=1e-15, q=2):
    """Upwind-selected reconstruction at an interface.

    qs: the six values (q_{i-3}, q_{i-2}, q_{i-1}, q_i, q_{i+1}, q_{i+2})
    around the interface x_{i-1/2}; vel: the advecting velocity there.
    scheme: "weno5z", "weno5_linear" or "none" (returns zeros).
    """
    m3, m2, m1, p0, p1, p2 = qs
    if scheme == "none":
        return np.zeros_like(np.broadcast_to(p0, np.shape(vel)), dtype=float)
    if scheme == "weno5z":
        pos = weno5z(m3, m2, m1, p0, p1, eps, q)
        neg = weno5z(p2, p1, p0, m1, m2, eps, q)
    elif scheme == "weno5_linear":
        pos = weno5_linear(m3, m2, m1, p0, p1)
        neg = weno5_linear(p2, p1, p0, m1, m2)
    else:
        raise ValueError(scheme)
    return np.where(vel > 0, pos, neg)
