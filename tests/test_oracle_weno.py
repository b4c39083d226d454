"""Pins of the oracle's reconstruction against what the mathematics fixes.

Reconstruction subsection of the finite-volume appendix (fifth-order WENO
equation, upwind-biased equation and its centred + diffusive decompositions).
"""
import numpy as np
import pytest

from oracle import weno


def cell_averages_of_monomial(p, centres, h):
    """Exact cell averages of x**p over [x - h/2, x + h/2]."""
    a = centres - h / 2
    b = centres + h / 2
    return (b ** (p + 1) - a ** (p + 1)) / ((p + 1) * h)


def _stencil_values(p, h=0.37, x_iface=0.11):
    # cells i-3..i+2 around the interface x_{i-1/2}
    centres = x_iface + h * (np.arange(-3, 3) + 0.5)
    return cell_averages_of_monomial(p, centres, h), x_iface ** p


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_linear_weights_exact_to_degree_4(p):
    q, exact = _stencil_values(p)
    for vel in (1.0, -1.0):
        r = weno.reconstruct("weno5_linear", list(q), np.array(vel))
        assert abs(float(r) - exact) <= 1e-13 * max(1.0, abs(exact))


def test_linear_weights_not_exact_at_degree_5():
    q, exact = _stencil_values(5)
    r = weno.reconstruct("weno5_linear", list(q), np.array(1.0))
    assert abs(float(r) - exact) > 1e-8


def test_linear_weights_equal_unique_fifth_order_stencil():
    """The ideal combination must equal the unique 5-cell stencil that is
    exact for cell averages of polynomials of degree <= 4 (solved here as a
    Vandermonde-type system, independent of the candidate formulas)."""
    h = 1.0
    centres = h * (np.arange(-3, 2) + 0.5)  # cells i-3..i+1 -> upwind set for u > 0
    A = np.array([cell_averages_of_monomial(p, centres, h) for p in range(5)])
    rhs = np.array([0.0 ** p for p in range(5)])  # point values at x = 0
    coef = np.linalg.solve(A, rhs)
    assert np.allclose(coef * 60.0, [2, -13, 47, 27, -3], atol=1e-12)
    basis = np.eye(5)
    got = [float(weno.weno5_linear(*basis[k])) for k in range(5)]
    assert np.allclose(got, coef, atol=1e-15)


@pytest.mark.parametrize("p", [0, 1, 2])
def test_wenoz_exact_to_degree_2(p):
    q, exact = _stencil_values(p)
    for vel in (1.0, -1.0):
        r = weno.reconstruct("weno5z", list(q), np.array(vel))
        assert abs(float(r) - exact) <= 1e-13 * max(1.0, abs(exact))


def test_wenoz_mirror_symmetry():
    rng = np.random.default_rng(3)
    q = rng.standard_normal((6, 1000))
    pos = weno.reconstruct("weno5z", list(q), np.ones(1000))
    # mirror the data about the interface: q_{i-1+s} <-> q_{i-s}
    qm = q[::-1]
    neg = weno.reconstruct("weno5z", list(qm), -np.ones(1000))
    assert np.array_equal(pos, neg)


def test_wenoz_convex_bounded_near_jump():
    """At a step the weights must pick the smooth stencil: the reconstruction
    stays within the data range (no overshoot of the jump)."""
    q = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    r = float(weno.reconstruct("weno5z", q, np.array(1.0)))
    assert -1e-12 <= r <= 1.0 + 1e-12
    assert r < 1e-6  # upwind side is flat: essentially zero
    q2 = [0.0, 0.0, 1.0, 1.0, 1.0, 1.0]
    r2 = float(weno.reconstruct("weno5z", q2, np.array(1.0)))
    assert 1.0 - 1e-6 < r2 <= 1.0 + 1e-12


def _order(errors, ns):
    e = np.array(errors)
    n = np.array(ns, dtype=float)
    return np.polyfit(np.log(n), np.log(e), 1)[0] * -1


def test_wenoz_fifth_order_on_exponential():
    """Reconstruction error of exp(x) on [0, 1] (no critical points) must
    decrease at fifth order."""
    errs, ns = [], [16, 32, 64, 128]   # 256 hits the round-off floor of the averages
    for n in ns:
        h = 1.0 / n
        centres = (np.arange(-3, n + 3) + 0.5) * h
        avg = (np.exp(centres + h / 2) - np.exp(centres - h / 2)) / h
        # interfaces i = 0..n: x = i h
        qs = [avg[3 + o: 3 + o + n + 1] for o in range(-3, 3)]
        r = weno.reconstruct("weno5z", qs, np.ones(n + 1))
        errs.append(np.max(np.abs(r - np.exp(np.arange(n + 1) * h))))
    assert _order(errs[1:], ns[1:]) >= 4.8


def test_upwind1_is_centred_plus_diffusion():
    rng = np.random.default_rng(1)
    c = rng.standard_normal((2, 500))
    u = rng.standard_normal(500)
    dx = 0.3
    lhs = u * weno.upwind1(c[0], c[1], u)
    kappa1 = np.abs(u) * dx / 2
    rhs = u * (c[0] + c[1]) / 2 - kappa1 * (c[1] - c[0]) / dx
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-14)


def test_upwind3_is_centred4_plus_hyperdiffusion():
    rng = np.random.default_rng(2)
    c = rng.standard_normal((4, 500))   # c_{i-2}, c_{i-1}, c_i, c_{i+1}
    u = rng.standard_normal(500)
    dx = 0.7
    lhs = u * weno.upwind3(c[0], c[1], c[2], c[3], u)
    centred4 = (-c[0] + 7 * c[1] + 7 * c[2] - c[3]) / 12
    third_diff = (c[3] - 3 * c[2] + 3 * c[1] - c[0]) / dx ** 3
    kappa3 = np.abs(u) * dx ** 3 / 12
    rhs = u * centred4 + kappa3 * third_diff
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-13)
