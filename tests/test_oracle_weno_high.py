"""Pins of the oracle's WENO reconstructions of orders 7 and 9 and of the
centred reconstructions that interpolate the advecting velocity
(reconstruction subsection of the finite-volume appendix: a WENO scheme of
order 2r - 1 combines r shifted upwind stencils of order r; Centered(order=N)
for even N).  Every expected value below comes from the mathematics (exact
polynomial cell averages, derivative integrals by numpy's polynomial
routines, Vandermonde solves), from the order-5 formulas written out by hand
in the oracle and pinned separately, or from published constants that are
named."""
import math
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle import weno

ORDER = {4: ("weno7z", "weno7_linear"), 5: ("weno9z", "weno9_linear")}


def cell_averages(coef, centres, h):
    """Exact cell averages over [x - h/2, x + h/2] of the polynomial with
    coefficients coef (lowest first)."""
    F = P.polyint(coef)
    return (P.polyval(centres + h / 2, F) - P.polyval(centres - h / 2, F)) / h


def _stencil(r, coef, h=0.37, x_iface=0.11):
    """Cell averages on the 2r cells i-r .. i+r-1 around x_{i-1/2}."""
    centres = x_iface + h * (np.arange(-r, r) + 0.5)
    return cell_averages(coef, centres, h), P.polyval(x_iface, coef)


def _monomial(p):
    return np.eye(p + 1)[p]


@pytest.mark.parametrize("r", [4, 5])
def test_linear_weights_exact_to_degree_2r_minus_2(r):
    scheme = ORDER[r][1]
    for p in range(2 * r - 1):
        q, exact = _stencil(r, _monomial(p))
        for vel in (1.0, -1.0):
            got = float(weno.reconstruct(scheme, list(q), np.array(vel)))
            assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), (p, vel)
    q, exact = _stencil(r, _monomial(2 * r - 1))
    assert abs(float(weno.reconstruct(scheme, list(q), np.array(1.0))) - exact) > 1e-9


@pytest.mark.parametrize("r", [4, 5])
def test_linear_weights_equal_unique_stencil(r):
    """The ideal combination equals the unique (2r - 1)-cell stencil exact
    for cell averages of polynomials of degree <= 2r - 2."""
    n = 2 * r - 1
    centres = np.arange(-r, r - 1) + 0.5
    A = np.array([cell_averages(_monomial(p), centres, 1.0) for p in range(n)])
    coef = np.linalg.solve(A, np.eye(n)[0])      # point value at x = 0
    basis = np.eye(n)
    got = [float(weno.weno_linear_general(list(basis[k]), r)) for k in range(n)]
    assert np.allclose(got, coef, rtol=0, atol=1e-13)


def test_ideal_weights_published():
    """Optimal weights of WENO7 and WENO9 as tabulated by Balsara & Shu
    (2000), ordered from the most upwind stencil."""
    assert weno.ideal_weights(4) == (Fraction(1, 35), Fraction(12, 35), Fraction(18, 35),
                                     Fraction(4, 35))
    assert weno.ideal_weights(5) == (Fraction(1, 126), Fraction(10, 63), Fraction(10, 21),
                                     Fraction(20, 63), Fraction(5, 126))
    assert tuple(weno.ideal_weights(3)) == tuple(Fraction(x).limit_denominator(10)
                                                for x in weno.IDEAL)


@pytest.mark.parametrize("r", [4, 5])
def test_candidates_exact_to_degree_r_minus_1(r):
    for p in range(r + 1):
        q, exact = _stencil(r, _monomial(p))
        c = weno.candidates_general(list(q[:2 * r - 1]), r)
        for k in range(r):
            if p <= r - 1:
                assert abs(c[k] - exact) <= 1e-12 * max(1.0, abs(exact)), (p, k)
            else:
                assert abs(c[k] - exact) > 1e-9, (p, k)


@pytest.mark.parametrize("r", [3, 4, 5])
def test_indicators_are_derivative_integrals(r):
    """For data that are cell averages of a polynomial p of degree <= r - 1
    every candidate recovers p, so each indicator must be
    sum_l h^(2l-1) int over the upwind cell of (p^(l))^2.  Random p span all
    data vectors, so this fixes every entry of each quadratic form."""
    rng = np.random.default_rng(40 + r)
    h, x_iface = 0.37, 0.11
    for _ in range(3 * r * r):
        coef = rng.standard_normal(r)
        q, _ = _stencil(r, coef, h, x_iface)
        betas = weno.smoothness_general(list(q[:2 * r - 1]), r)
        want = 0.0
        for l in range(1, r):
            d = P.polyder(coef, l)
            F = P.polyint(P.polymul(d, d))
            want += h ** (2 * l - 1) * (P.polyval(x_iface, F) - P.polyval(x_iface - h, F))
        for k in range(r):
            assert abs(betas[k] - want) <= 1e-11 * max(1.0, want), (k, betas[k], want)


def test_generic_order_5_matches_jiang_shu():
    """The general construction at r = 3 reproduces the order-5 candidates,
    indicators and WENO-Z value written out by hand (Jiang & Shu 1996)."""
    rng = np.random.default_rng(9)
    v = list(rng.standard_normal((5, 200)))
    c = weno.candidates_general(v, 3)
    for got, want in zip(c, weno.candidates(*v)):
        assert np.allclose(got, want, rtol=0, atol=1e-14)
    b = weno.smoothness_general(v, 3)
    for got, want in zip(b, weno.smoothness(*v)):
        assert np.allclose(got, want, rtol=1e-13, atol=1e-14)
    assert np.allclose(weno.wenoz_general(v, 3), weno.weno5z(*v), rtol=0, atol=1e-13)


def _order(errors, ns):
    return -np.polyfit(np.log(np.array(ns, float)), np.log(np.array(errors)), 1)[0]


def _exp_stencils(r, n):
    h = 1.0 / n
    centres = (np.arange(-r, n + r) + 0.5) * h
    avg = (np.exp(centres + h / 2) - np.exp(centres - h / 2)) / h
    qs = [avg[r + o: r + o + n + 1] for o in range(-r, r)]
    return qs, np.exp(np.arange(n + 1) * h)


@pytest.mark.parametrize("r,lowest", [(4, 6.5), (5, 7.6)])
def test_global_indicator_order(r, lowest):
    """tau of WENO-Z must vanish on smooth data faster than the indicators
    themselves: O(h^7) for order 7 and O(h^8) for order 9 (a coefficient
    off by one drops it to O(h^5)/O(h^6)), while b_k = O(h^2)."""
    ns = [16, 32, 64]
    taus, b0s = [], []
    for n in ns:
        qs, _ = _exp_stencils(r, n)
        betas = weno.smoothness_general(qs[:2 * r - 1], r)
        taus.append(np.max(weno.global_indicator(betas, r)))
        b0s.append(np.max(betas[0]))
    assert _order(taus, ns) >= lowest, taus
    assert abs(_order(b0s, ns) - 2.0) < 0.1


@pytest.mark.parametrize("r,ns,lowest", [(4, [8, 16, 32], 6.6), (5, [8, 12, 16], 8.4)])
def test_wenoz_order_on_exponential(r, ns, lowest):
    errs = []
    for n in ns:
        qs, exact = _exp_stencils(r, n)
        got = weno.reconstruct(ORDER[r][0], qs, np.ones(n + 1))
        errs.append(np.max(np.abs(got - exact)))
    assert _order(errs, ns) >= lowest, errs


@pytest.mark.parametrize("r", [4, 5])
def test_wenoz_exact_to_degree_r_minus_1(r):
    for p in range(r):
        q, exact = _stencil(r, _monomial(p))
        for vel in (1.0, -1.0):
            got = float(weno.reconstruct(ORDER[r][0], list(q), np.array(vel)))
            assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), (p, vel)


@pytest.mark.parametrize("scheme", ["weno7z", "weno9z", "weno7_linear", "weno9_linear"])
def test_mirror_symmetry(scheme):
    R = weno.RADIUS[scheme]
    rng = np.random.default_rng(3)
    q = rng.standard_normal((2 * R, 500))
    pos = weno.reconstruct(scheme, list(q), np.ones(500))
    neg = weno.reconstruct(scheme, list(q[::-1]), -np.ones(500))
    assert np.allclose(pos, neg, rtol=0, atol=1e-14)


@pytest.mark.parametrize("scheme", ["weno7z", "weno9z"])
def test_no_overshoot_at_a_step(scheme):
    """At a jump the weights pick the stencils on the smooth side."""
    R = weno.RADIUS[scheme]
    for jump in range(1, 2 * R):
        q = [0.0] * jump + [1.0] * (2 * R - jump)
        r_ = float(weno.reconstruct(scheme, q, np.array(1.0)))
        assert -1e-6 <= r_ <= 1.0 + 1e-6, (jump, r_)
    q = [0.0] * R + [1.0] * R          # jump at the interface itself
    assert float(weno.reconstruct(scheme, q, np.array(1.0))) < 1e-6
    assert float(weno.reconstruct(scheme, q, np.array(-1.0))) > 1.0 - 1e-6


def test_centred_coefficients():
    """Centered(order=2) is the two-cell average (centered-reconstruction
    equation); order 4 is the (-1, 7, 7, -1)/12 that the UpwindBiased(3)
    reordering exposes; order 6 is the mean of the two order-5 upwind
    stencils written out by hand; all are symmetric."""
    assert weno.centred_coefficients(2) == (Fraction(1, 2), Fraction(1, 2))
    assert weno.centred_coefficients(4) == tuple(Fraction(c, 12) for c in (-1, 7, 7, -1))
    basis = np.eye(6)
    mean5 = [0.5 * (float(weno.weno5_linear(*basis[k, :5])) +
                    float(weno.weno5_linear(*basis[k, :0:-1]))) for k in range(6)]
    assert np.allclose([float(c) for c in weno.centred_coefficients(6)], mean5, atol=1e-15)
    for N in (2, 4, 6, 8):
        c = weno.centred_coefficients(N)
        assert c == c[::-1] and sum(c) == 1


@pytest.mark.parametrize("N", [6, 8])
def test_centred_exact_to_degree_N_minus_1(N):
    r = N // 2
    for p in range(N + 1):
        q, exact = _stencil(r, _monomial(p))
        got = weno.centred(N, list(q))
        if p <= N - 1:
            assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), p
        else:
            assert abs(got - exact) > 1e-9, p


@pytest.mark.parametrize("r", [4, 5])
def test_upwind_is_centred_plus_odd_dissipation(r):
    """The two upwind-biased linear reconstructions average to the centred
    reconstruction of order 2r on the 2r cells, so the upwind flux is a
    centred flux plus a dissipative correction (the decomposition the
    reconstruction subsection describes)."""
    basis = np.eye(2 * r)
    scheme = ORDER[r][1]
    pos = np.array([float(weno.reconstruct(scheme, list(basis[k]), np.array(1.0)))
                    for k in range(2 * r)])
    neg = np.array([float(weno.reconstruct(scheme, list(basis[k]), np.array(-1.0)))
                    for k in range(2 * r)])
    assert np.allclose(0.5 * (pos + neg), [float(c) for c in weno.centred_coefficients(2 * r)],
                       atol=1e-14)
    # the difference is a multiple of the (2r - 1)-th difference across the cells
    diff = pos - neg
    binom = np.array([(-1) ** (2 * r - 1 - t) * math.comb(2 * r - 1, t) for t in range(2 * r)])
    ratio = diff[np.abs(binom) > 0] / binom[np.abs(binom) > 0]
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
