"""Analytic fields and their exact nonhydrostatic tendencies (sympy), used to
pin the oracle's discrete operators by convergence under grid refinement.

The continuous tendencies are those of the nonhydrostatic momentum and tracer
equations in flux form: -d_j(u_j u_i) + nu lap u_i - f z x u + b z_hat and
-d_j(u_j c) + kappa lap c.
"""
import numpy as np
import sympy as sp

X, Y, Z = sp.symbols("x y z", real=True)


def periodic_fields():
    u = sp.sin(X) * sp.cos(Y) * sp.cos(Z) + sp.Rational(3, 10) * sp.sin(2 * Y + Z) + sp.Rational(1, 5)
    v = -sp.cos(X) * sp.sin(Y) * sp.cos(Z) + sp.Rational(2, 5) * sp.cos(X + 2 * Z) - sp.Rational(1, 10)
    w = sp.Rational(1, 2) * sp.sin(X + Y) * sp.cos(Z) + sp.Rational(1, 5) * sp.sin(2 * X) + sp.Rational(3, 20)
    c = sp.cos(X) * sp.sin(2 * Y) + sp.Rational(1, 2) * sp.sin(Z + X)
    return {"u": u, "v": v, "w": w, "c": c}


def bounded_fields():
    """Fields on [0, 2pi)^2 x [0, pi] compatible with the wall conditions:
    u, v, T, S even about z = 0, pi (cosines), w odd (sines, 0 on walls)."""
    u = sp.sin(X) * sp.cos(Y) * sp.cos(Z) + sp.Rational(3, 10) * sp.cos(2 * Y) * sp.cos(2 * Z) + sp.Rational(1, 5)
    v = -sp.cos(X) * sp.sin(Y) * sp.cos(Z) + sp.Rational(2, 5) * sp.sin(X) * sp.cos(3 * Z) - sp.Rational(1, 10)
    w = sp.Rational(1, 2) * sp.sin(X + Y) * sp.sin(Z) + sp.Rational(1, 5) * sp.cos(2 * X) * sp.sin(2 * Z)
    T = sp.cos(X) * sp.sin(2 * Y) * sp.cos(Z) + sp.Rational(1, 2) * sp.cos(2 * Z) + 3
    S = sp.sin(X + Y) * sp.cos(2 * Z) + 1
    return {"u": u, "v": v, "w": w, "T": T, "S": S}


def exact_tendencies(fields, nu, kappa, f=0.0, g=0.0, alpha=0.0, beta=0.0, t_ref=0.0, s_ref=0.0):
    u, v, w = fields["u"], fields["v"], fields["w"]
    vel = (u, v, w)
    coords = (X, Y, Z)

    def adv(q):
        return -sum(sp.diff(vel[j] * q, coords[j]) for j in range(3))

    def lap(q):
        return sum(sp.diff(q, c, 2) for c in coords)

    out = {"u": adv(u) + nu * lap(u) + f * v,
           "v": adv(v) + nu * lap(v) - f * u,
           "w": adv(w) + nu * lap(w)}
    if "T" in fields:
        b = g * (alpha * (fields["T"] - t_ref) - beta * (fields["S"] - s_ref))
        out["w"] = out["w"] + b
    for name in fields:
        if name not in ("u", "v", "w"):
            out[name] = adv(fields[name]) + kappa * lap(fields[name])
    return out


def sample(expr, ph, loc, nzf=None):
    """Evaluate a sympy expression at the staggered points of `loc`
    ('c' centres, 'u', 'v', 'w' faces) as an interior array."""
    dx, dy, dz = ph.spacing
    fn = sp.lambdify((X, Y, Z), expr, "numpy")
    xi = ph.x0 + (np.arange(ph.nx) + (0.0 if loc == "u" else 0.5)) * dx
    yi = ph.y0 + (np.arange(ph.ny) + (0.0 if loc == "v" else 0.5)) * dy
    if loc == "w":
        nk = nzf if nzf is not None else ph.nz
        zi = ph.z0 + np.arange(nk) * dz
    else:
        zi = ph.z0 + (np.arange(ph.nz) + 0.5) * dz
    Zg, Yg, Xg = np.meshgrid(zi, yi, xi, indexing="ij")
    return np.broadcast_to(fn(Xg, Yg, Zg), Zg.shape).astype(float).copy()
