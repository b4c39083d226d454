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

Orders 7 and 9 (WENO(order=9) in the paper's examples and its global-ocean
configuration, which also uses order 7 for tracers) follow the construction
the reconstruction subsection describes for order 5: a WENO reconstruction of
order 2r - 1 combines r upwind stencils of r cells, shifted against each
other by one cell, with weights that reduce to the ideal ones for smooth
data.  Everything that the construction defines exactly is derived here from
its definition in rational arithmetic, in units of the cell width with the
interface at x = 0 and cell m covering [m, m + 1]:
  * a candidate value is that of the degree r - 1 polynomial whose averages
    over its r cells are the data, taken at the interface;
  * the ideal weights make the candidates' combination equal the single
    (2r - 1)-cell stencil of the same construction;
  * the Jiang-Shu indicator of a candidate is the sum over l = 1..r-1 of the
    integral over the upwind cell (-1, 0) of the squared l-th derivative of
    its polynomial (scaled by h^(2l-1), which cancels in units of h);
  * the centred reconstruction of even order N (the advecting velocity of
    momentum advection, N = 2r - 2; the paper's Centered(order=N)) is the
    same construction on the N cells centred on the interface.
Readings where the paper is silent: the WENO-Z global indicator tau of
orders 7 and 9 is the combination of Castro, Costa & Don (2011),
|b0 + 3 b1 - 3 b2 - b3| and |b0 + 2 b1 - 6 b2 + 2 b3 + b4|; the exponent q
and eps are those of order 5; the advecting velocity of momentum advection
is interpolated with the centred reconstruction one order below the WENO
order (order 4 for WENO5, 6 for WENO7, 8 for WENO9).
"""
from fractions import Fraction
from functools import lru_cache

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


# ---------------------------------------------------------------------------
# Orders 2r - 1 = 7 and 9 (and the centred reconstructions), from the
# construction itself.
# ---------------------------------------------------------------------------

# Coefficients of the WENO-Z global indicator tau (Castro, Costa & Don 2011).
TAU = {3: (1, 0, -1), 4: (1, 3, -3, -1), 5: (1, 2, -6, 2, 1)}

RADIUS = {"none": 3, "weno5z": 3, "weno5_linear": 3, "weno7z": 4, "weno7_linear": 4,
          "weno9z": 5, "weno9_linear": 5}


def _inverse(A):
    """Exact inverse of a square matrix of Fractions (Gauss-Jordan)."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [x * inv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def polynomial_map(cells):
    """Matrix C with a = C v: the coefficients a_j (of x**j) of the
    polynomial of degree len(cells) - 1 whose averages over the unit cells
    [m, m + 1], m in cells, are v."""
    n = len(cells)
    A = [[Fraction((m + 1) ** (j + 1) - m ** (j + 1), j + 1) for j in range(n)] for m in cells]
    return _inverse(A)


def interface_stencil(cells):
    """Weights on the cell averages giving that polynomial's value at x = 0."""
    return polynomial_map(cells)[0]


@lru_cache(maxsize=None)
def centred_coefficients(order):
    """Centred reconstruction of even order N at the interface from the N
    cells -N/2 .. N/2 - 1 (Fractions)."""
    if order % 2 or order < 2:
        raise ValueError(order)
    return tuple(interface_stencil(list(range(-order // 2, order // 2))))


@lru_cache(maxsize=None)
def candidate_coefficients(r):
    """The r candidate stencils for u > 0: candidate k on cells -r+k .. k-1
    (k = 0 is the most upwind), as r tuples of Fractions."""
    return tuple(tuple(interface_stencil(list(range(-r + k, k)))) for k in range(r))


@lru_cache(maxsize=None)
def ideal_weights(r):
    """d_k such that sum_k d_k (candidate k) is the (2r - 1)-cell stencil on
    cells -r .. r - 2 (solved on its first r entries, checked on the rest)."""
    big = interface_stencil(list(range(-r, r - 1)))
    cand = candidate_coefficients(r)
    # column k of E: candidate k placed at offset k of the big stencil
    E = [[cand[k][t - k] if 0 <= t - k < r else Fraction(0) for k in range(r)]
         for t in range(2 * r - 1)]
    Einv = _inverse(E[:r])
    d = [sum(Einv[k][t] * big[t] for t in range(r)) for k in range(r)]
    for t in range(2 * r - 1):
        if sum(E[t][k] * d[k] for k in range(r)) != big[t]:
            raise ArithmeticError("candidates do not combine into the big stencil")
    return tuple(d)


@lru_cache(maxsize=None)
def smoothness_matrices(r):
    """beta_k = v^T M_k v for the data v of candidate k: the sum over
    l = 1..r-1 of the integral over (-1, 0) of (p_k^(l))^2."""
    out = []
    for k in range(r):
        C = polynomial_map(list(range(-r + k, k)))
        # Q[j][j']: integral over (-1, 0) of d^l x^j * d^l x^j', summed over l
        Q = [[Fraction(0)] * r for _ in range(r)]
        for l in range(1, r):
            for j in range(l, r):
                for jj in range(l, r):
                    cj = Fraction(np.prod(range(j - l + 1, j + 1), dtype=object))
                    cjj = Fraction(np.prod(range(jj - l + 1, jj + 1), dtype=object))
                    m = j + jj - 2 * l
                    Q[j][jj] += cj * cjj * Fraction((-1) ** m, m + 1)
        M = [[sum(C[a][i] * Q[a][b] * C[b][jv] for a in range(r) for b in range(r))
              for jv in range(r)] for i in range(r)]
        out.append(tuple(tuple(row) for row in M))
    return tuple(out)


def _f(x):
    return np.array([float(v) for v in x]) if isinstance(x[0], Fraction) else np.array(x, float)


def candidates_general(vals, r):
    """The r candidate values from the 2r - 1 upwind-ordered values."""
    cand = candidate_coefficients(r)
    return [sum(float(cand[k][t]) * vals[k + t] for t in range(r)) for k in range(r)]


@lru_cache(maxsize=None)
def difference_forms(r):
    """N_k with beta_k = delta^T N_k delta, delta_t = v_{t+1} - v_t: M_k
    vanishes on constants, so with v_t = v_0 + sum_{s<t} delta_s the form
    depends on the differences alone."""
    out = []
    for M in smoothness_matrices(r):
        N = [[sum(M[a][b] for a in range(s + 1, r) for b in range(u + 1, r))
              for u in range(r - 1)] for s in range(r - 1)]
        out.append(tuple(tuple(row) for row in N))
    return tuple(out)


def smoothness_general(vals, r):
    """The r Jiang-Shu indicators beta_k = v_k^T M_k v_k, evaluated on the
    differences of neighbouring values (no cancellation against the mean
    of the data)."""
    Ns = difference_forms(r)
    out = []
    for k in range(r):
        dlt = [vals[k + t + 1] - vals[k + t] for t in range(r - 1)]
        out.append(sum(dlt[a] * sum(float(Ns[k][a][b]) * dlt[b] for b in range(r - 1))
                       for a in range(r - 1)))
    return out


def global_indicator(betas, r):
    """WENO-Z tau of order 2r - 1."""
    return np.abs(sum(c * b for c, b in zip(TAU[r], betas)))


def wenoz_general(vals, r, eps=1e-15, q=2):
    """WENO-Z reconstruction of order 2r - 1 from the 2r - 1 upwind-ordered
    values vals (cells -r .. r - 2 for u > 0)."""
    d = ideal_weights(r)
    recs = candidates_general(vals, r)
    betas = smoothness_general(vals, r)
    tau = global_indicator(betas, r)
    alphas = [float(d[k]) * (1.0 + (tau / (betas[k] + eps)) ** q) for k in range(r)]
    total = sum(alphas)
    return sum(a * rk for a, rk in zip(alphas, recs)) / total


def weno_linear_general(vals, r):
    """The ideal-weight limit of order 2r - 1."""
    d = ideal_weights(r)
    return sum(float(dk) * rk for dk, rk in zip(d, candidates_general(vals, r)))


def centred(order, vals):
    """Centred reconstruction of even order from `order` values (cells
    -order/2 .. order/2 - 1 around the interface)."""
    c = centred_coefficients(order)
    return sum(float(ci) * v for ci, v in zip(c, vals))


def reconstruct(scheme, qs, vel, eps=1e-15, q=2):
    """Upwind-selected reconstruction at an interface.

    qs: the 2R values q_{i-R} .. q_{i+R-1} around the interface x_{i-1/2}
    (R = RADIUS[scheme]: six values for order 5, eight for 7, ten for 9);
    vel: the advecting velocity there.  scheme: "weno5z", "weno5_linear",
    "weno7z", "weno7_linear", "weno9z", "weno9_linear" or "none" (zeros).
    """
    R = RADIUS[scheme]
    if len(qs) != 2 * R:
        raise ValueError(f"{scheme} needs {2 * R} values")
    if scheme == "none":
        return np.zeros_like(np.broadcast_to(qs[R], np.shape(vel)), dtype=float)
    if R > 3:
        up = list(qs[:2 * R - 1])              # cells -R .. R-2
        down = list(qs[:0:-1])                 # mirrored: cells R-1 .. -R+1
        if scheme.endswith("z"):
            pos = wenoz_general(up, R, eps, q)
            neg = wenoz_general(down, R, eps, q)
        else:
            pos = weno_linear_general(up, R)
            neg = weno_linear_general(down, R)
        return np.where(vel > 0, pos, neg)
    m3, m2, m1, p0, p1, p2 = qs
    if scheme == "weno5z":
        pos = weno5z(m3, m2, m1, p0, p1, eps, q)
        neg = weno5z(p2, p1, p0, m1, m2, eps, q)
    elif scheme == "weno5_linear":
        pos = weno5_linear(m3, m2, m1, p0, p1)
        neg = weno5_linear(p2, p1, p0, m1, m2)
    else:
        raise ValueError(scheme)
    return np.where(vel > 0, pos, neg)
