"""Nonhydrostatic tendencies (everything but the nonhydrostatic pressure).

Momentum: flux-form advection (flux-form-advection equation; momentum
advection subsection: a high-order centred advecting velocity times a WENO
reconstruction of the advected component), f-plane Coriolis, buoyancy from a
linear equation of state, constant-coefficient Laplacian closure
(ScalarDiffusivity).  Tracers: flux divergence of advective + diffusive
fluxes (flux-divergence and advection-flux-divergence equations) with a
prescribed flux through the top wall.

Readings where the paper is silent:
* the advecting-velocity interpolation for momentum is the centred
  reconstruction one order below the WENO order: fourth order,
  (-a0 + 7 a1 + 7 a2 - a3) / 12, with WENO5; sixth order with WENO7 and
  eighth order with WENO9 (stencils widened symmetrically);
* Coriolis uses four-point averages of the other horizontal component;
* buoyancy b = g (alpha (T - T0) - beta (S - S0)) enters G_w averaged to
  the w faces;
* walls are impenetrable, free-slip and no-flux except for the prescribed
  top tracer flux (upward positive);
* immersed cells (grid-fitted boundary, oracle/immersed.py) close their
  faces: zero velocity and velocity tendency there, no diffusive tracer flux
  through them, no top flux into an immersed top cell.

Vertically stretched grids (unevenly spaced z faces, staggered-grid listing
of the finite-volume appendix): flux divergences divide the z difference of
the fluxes by the thickness of the control volume (dzc[k] for cells, dzf[k]
for the w cells around face k) and vertical diffusive fluxes divide by the
distance between the two values they difference.  Readings: the WENO
reconstructions, the fourth-order advecting-velocity interpolation and the
buoyancy average to w faces keep their uniform-grid coefficients in index
space along z.  With implicit vertical diffusion (vertically implicit
time-discretisation paragraph) the z diffusive fluxes are left out of G;
the prescribed top flux stays explicit.

All tendencies are returned as interior arrays; G_w has nz + 1 faces when z
is bounded (wall faces hold 0).
"""
import numpy as np

from . import immersed
from .fv import view, z_spacings
from .weno import RADIUS, centred, reconstruct


def interp4(a0, a1, a2, a3):
    """Centred fourth-order interpolation to the midpoint of a1 and a2."""
    return (-a0 + 7.0 * a1 + 7.0 * a2 - a3) / 12.0


def _offsets(ph):
    """Offsets of the 2R values a reconstruction at x_{i-1/2} reads."""
    R = RADIUS[ph.advection]
    return tuple(range(-R, R))


def _ioffsets(ph):
    """Offsets of the values the advecting-velocity interpolation reads."""
    R = RADIUS[ph.advection]
    return tuple(range(-(R - 1), R - 1))


def _interp(ph, vals):
    """Centred interpolation of the advecting velocity (order 2R - 2)."""
    if len(vals) == 4:
        return interp4(*vals)
    return centred(len(vals), vals)


def _rec(ph, qs, vel):
    return reconstruct(ph.advection, qs, vel, ph.weno_eps, ph.weno_q)


def _div(Fx, Fy, Fz, ph, hz):
    """Flux divergence (1/V) sum over directions of delta(A F) on a grid
    uniform in x and y: A_x / V = 1/dx, A_y / V = 1/dy, A_z / V = 1/hz with
    hz the control-volume thickness per level, shape (nz, 1, 1).  Fluxes carry
    one extra entry along their own axis."""
    dx, dy, _ = ph.spacing
    return ((Fx[:, :, 1:] - Fx[:, :, :-1]) / dx
            + (Fy[:, 1:, :] - Fy[:, :-1, :]) / dy
            + (Fz[1:] - Fz[:-1]) / hz)


def _zgrid(ph):
    """(dzc, dzf) as (n, 1, 1) columns, and the centre thicknesses on the
    w-flux positions (centres -1..nz-1: the mirror or periodic image first)."""
    dzc, dzf = z_spacings(ph)
    below = dzc[0] if ph.z_bounded else dzc[-1]
    dzc_w = np.concatenate([[below], dzc])
    return dzc[:, None, None], dzf[:, None, None], dzc_w[:, None, None]


def _zdiff(ph, coef):
    """Coefficient of the explicit vertical diffusive flux: zero when the
    vertical diffusion is implicit."""
    return 0.0 if getattr(ph, "implicit_z", False) else coef


def tracer_tendency(c, s, ph, top_flux=0.0):
    """G_c for a centred tracer c given padded velocities s['u'], s['v'], s['w']."""
    u, v, w = s["u"], s["v"], s["w"]
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    dx, dy, _ = ph.spacing
    dzc, dzf, _ = _zgrid(ph)
    k = ph.kappa
    kz = _zdiff(ph, k)
    ox, oy, oz = _open(ph)
    # x faces i = 0..nx
    U = view(u, ni=nx + 1, ph=ph)
    Fx = U * _rec(ph, [view(c, di=o, ni=nx + 1, ph=ph) for o in _offsets(ph)], U)
    Fx = Fx - ox * k * (view(c, ni=nx + 1, ph=ph) - view(c, di=-1, ni=nx + 1, ph=ph)) / dx
    # y faces j = 0..ny
    V = view(v, nj=ny + 1, ph=ph)
    Fy = V * _rec(ph, [view(c, dj=o, nj=ny + 1, ph=ph) for o in _offsets(ph)], V)
    Fy = Fy - oy * k * (view(c, nj=ny + 1, ph=ph) - view(c, dj=-1, nj=ny + 1, ph=ph)) / dy
    # z faces k = 0..nz
    W = view(w, nk=nz + 1, ph=ph)
    Fz = W * _rec(ph, [view(c, dk=o, nk=nz + 1, ph=ph) for o in _offsets(ph)], W)
    Fz = Fz - oz * kz * (view(c, nk=nz + 1, ph=ph) - view(c, dk=-1, nk=nz + 1, ph=ph)) / dzf
    if ph.z_bounded:
        Fz[0] = 0.0           # bottom wall: no flux
        # top wall: prescribed upward flux (into fluid top cells only)
        Fz[nz] = top_flux * immersed.fluid(ph)[nz - 1] if immersed.has_immersed(ph) else top_flux
    return -_div(Fx, Fy, Fz, ph, dzc)


def _open(ph):
    """Open flags of the x, y, z faces with one extra entry along each
    axis (1 everywhere without immersed cells)."""
    if not immersed.has_immersed(ph):
        return 1.0, 1.0, 1.0
    ox, oy, oz = immersed.open_faces(ph)
    ox = np.concatenate([ox, ox[:, :, :1]], axis=2)
    oy = np.concatenate([oy, oy[:, :1, :]], axis=1)
    if not ph.z_bounded:
        oz = np.concatenate([oz, oz[:1]], axis=0)
    return ox, oy, oz


def u_tendency(s, ph):
    """Advection + diffusion of u at (F, C, C) and the Coriolis term."""
    u, v, w = s["u"], s["v"], s["w"]
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    dx, dy, _ = ph.spacing
    dzc, dzf, _ = _zgrid(ph)
    nu = ph.nu
    nuz = _zdiff(ph, nu)
    # x: entry i holds the flux at cell centre i-1 (between faces i-1 and i)
    Ub = _interp(ph, [view(u, di=o, ni=nx + 1, ph=ph) for o in _ioffsets(ph)])
    X = Ub * _rec(ph, [view(u, di=o, ni=nx + 1, ph=ph) for o in _offsets(ph)], Ub)
    X = X - nu * (view(u, ni=nx + 1, ph=ph) - view(u, di=-1, ni=nx + 1, ph=ph)) / dx
    # y: corners (x face i, y face j); v interpolated along x to the x face
    Vt = _interp(ph, [view(v, di=o, nj=ny + 1, ph=ph) for o in _ioffsets(ph)])
    Y = Vt * _rec(ph, [view(u, dj=o, nj=ny + 1, ph=ph) for o in _offsets(ph)], Vt)
    Y = Y - nu * (view(u, nj=ny + 1, ph=ph) - view(u, dj=-1, nj=ny + 1, ph=ph)) / dy
    # z: (x face i, centre j, z face k); w interpolated along x to the x face
    Wt = _interp(ph, [view(w, di=o, nk=nz + 1, ph=ph) for o in _ioffsets(ph)])
    Z = Wt * _rec(ph, [view(u, dk=o, nk=nz + 1, ph=ph) for o in _offsets(ph)], Wt)
    Z = Z - nuz * (view(u, nk=nz + 1, ph=ph) - view(u, dk=-1, nk=nz + 1, ph=ph)) / dzf
    if ph.z_bounded:
        Z[0] = 0.0
        Z[nz] = 0.0
    G = -_div(X, Y, Z, ph, dzc)
    # Coriolis: -f z x u  ->  +f v averaged to the u point
    vbar = 0.25 * (view(v, di=-1, ph=ph) + view(v, ph=ph)
                   + view(v, di=-1, dj=1, ph=ph) + view(v, dj=1, ph=ph))
    return G + ph.f * vbar


def v_tendency(s, ph):
    """Advection + diffusion of v at (C, F, C) and the Coriolis term."""
    u, v, w = s["u"], s["v"], s["w"]
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    dx, dy, _ = ph.spacing
    dzc, dzf, _ = _zgrid(ph)
    nu = ph.nu
    nuz = _zdiff(ph, nu)
    # x: corners (x face i, y face j); u interpolated along y to the y face
    Ut = _interp(ph, [view(u, dj=o, ni=nx + 1, ph=ph) for o in _ioffsets(ph)])
    X = Ut * _rec(ph, [view(v, di=o, ni=nx + 1, ph=ph) for o in _offsets(ph)], Ut)
    X = X - nu * (view(v, ni=nx + 1, ph=ph) - view(v, di=-1, ni=nx + 1, ph=ph)) / dx
    # y: entry j holds the flux at cell centre j-1
    Vb = _interp(ph, [view(v, dj=o, nj=ny + 1, ph=ph) for o in _ioffsets(ph)])
    Y = Vb * _rec(ph, [view(v, dj=o, nj=ny + 1, ph=ph) for o in _offsets(ph)], Vb)
    Y = Y - nu * (view(v, nj=ny + 1, ph=ph) - view(v, dj=-1, nj=ny + 1, ph=ph)) / dy
    # z: (centre i, y face j, z face k); w interpolated along y
    Wt = _interp(ph, [view(w, dj=o, nk=nz + 1, ph=ph) for o in _ioffsets(ph)])
    Z = Wt * _rec(ph, [view(v, dk=o, nk=nz + 1, ph=ph) for o in _offsets(ph)], Wt)
    Z = Z - nuz * (view(v, nk=nz + 1, ph=ph) - view(v, dk=-1, nk=nz + 1, ph=ph)) / dzf
    if ph.z_bounded:
        Z[0] = 0.0
        Z[nz] = 0.0
    G = -_div(X, Y, Z, ph, dzc)
    # Coriolis: -f z x u  ->  -f u averaged to the v point
    ubar = 0.25 * (view(u, dj=-1, ph=ph) + view(u, di=1, dj=-1, ph=ph)
                   + view(u, ph=ph) + view(u, di=1, ph=ph))
    return G - ph.f * ubar


def buoyancy(s, ph):
    """Linear equation of state, b = g (alpha (T - T0) - beta (S - S0)), at
    cell centres (padded array).  The reference values only shift b by a
    constant, whose face average is a discrete gradient removed exactly by
    the projection."""
    return ph.g * (ph.alpha * (s["T"] - ph.t_ref) - ph.beta * (s["S"] - ph.s_ref))


def w_tendency(s, ph):
    """Advection + diffusion of w at (C, C, F) plus buoyancy."""
    u, v, w = s["u"], s["v"], s["w"]
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    dx, dy, _ = ph.spacing
    _, dzf, dzc_w = _zgrid(ph)
    nu = ph.nu
    nuz = _zdiff(ph, nu)
    # faces k = 0..nz-1 are computed; walls are overwritten below
    # x: (x face i, centre j, z face k); u interpolated along z to the z face
    Ut = _interp(ph, [view(u, dk=o, ni=nx + 1, ph=ph) for o in _ioffsets(ph)])
    X = Ut * _rec(ph, [view(w, di=o, ni=nx + 1, ph=ph) for o in _offsets(ph)], Ut)
    X = X - nu * (view(w, ni=nx + 1, ph=ph) - view(w, di=-1, ni=nx + 1, ph=ph)) / dx
    # y: (centre i, y face j, z face k); v interpolated along z
    Vt = _interp(ph, [view(v, dk=o, nj=ny + 1, ph=ph) for o in _ioffsets(ph)])
    Y = Vt * _rec(ph, [view(w, dj=o, nj=ny + 1, ph=ph) for o in _offsets(ph)], Vt)
    Y = Y - nu * (view(w, nj=ny + 1, ph=ph) - view(w, dj=-1, nj=ny + 1, ph=ph)) / dy
    # z: entry k holds the flux at cell centre k-1 (between faces k-1 and k)
    Wb = _interp(ph, [view(w, dk=o, nk=nz + 1, ph=ph) for o in _ioffsets(ph)])
    Z = Wb * _rec(ph, [view(w, dk=o, nk=nz + 1, ph=ph) for o in _offsets(ph)], Wb)
    Z = Z - nuz * (view(w, nk=nz + 1, ph=ph) - view(w, dk=-1, nk=nz + 1, ph=ph)) / dzc_w
    # the w cell around face k spans the centres k-1 and k: thickness dzf[k]
    G = -_div(X, Y, Z, ph, dzf[:nz])
    if ph.buoyancy:
        b = buoyancy(s, ph)
        G = G + 0.5 * (view(b, dk=-1, ph=ph) + view(b, ph=ph))
    if ph.z_bounded:
        G = np.concatenate([G, np.zeros((1, ny, nx))], axis=0)
        G[0] = 0.0
        G[nz] = 0.0
    return G


def tendencies(s, ph, workers=1):
    """All tendencies of the prognostic fields of a padded state dict, with
    the eddy-viscosity LES closure's contribution when one is configured.

    workers > 1 evaluates the fields' tendencies (independent computations)
    on that many threads; NumPy releases the interpreter lock inside its
    array operations, so large grids run in parallel.  Every value is
    computed by the same operations either way."""
    jobs = {"u": lambda: u_tendency(s, ph), "v": lambda: v_tendency(s, ph),
            "w": lambda: w_tendency(s, ph)}
    for name in ph.tracers:
        jobs[name] = (lambda n: lambda: tracer_tendency(s[n], s, ph, ph.top_flux.get(n, 0.0)))(name)
    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            fut = {n: ex.submit(f) for n, f in jobs.items()}
            T = {n: f.result() for n, f in fut.items()}
    else:
        T = {n: f() for n, f in jobs.items()}
    G = {"u": T["u"], "v": T["v"], "w": T["w"]}
    if immersed.has_immersed(ph):
        # velocities on closed faces do not change
        G["u"], G["v"], G["w"] = immersed.mask_velocities(G["u"], G["v"], G["w"], ph)
    for name in ph.tracers:
        G[name] = T[name]
    kind = getattr(ph, "les", "none")
    if kind != "none":
        from .les import les_tendencies
        L = les_tendencies(s, ph, kind)
        for name in G:
            G[name] = G[name] + L[name]
    return G
