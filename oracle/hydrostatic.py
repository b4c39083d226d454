"""Hydrostatic baroclinic step on a latitude-longitude grid.

Test infrastructure: a plain FP64 statement of the hydrostatic model
(hydrostatic-model subsection: hydrostatic balance, diagnostic continuity,
the momentum equations in the WENO vector-invariant form, the tracer
equation) and of its time stepping (hydrostatic time-discretisation
appendix: QAB2 predictor, depth-integrated slow forcing, split-explicit
barotropic substeps, correction and restart).

Readings (the paper gives the continuous vector-invariant form and defers
its discretisation to a work it cites; these are ours):
* C-grid on the thin shell (the metrics of `free_surface.latlon_metrics`,
  continued past the walls by the same formulas), uniform dz, walls at the
  latitude edges and in z, periodic longitude.  Halos: x periodic; at the
  y walls even mirrors for u, T, S and an odd mirror about the wall face
  for v (v = 0 on the walls); at the z walls even mirrors.
* w at z faces, diagnosed upwards from the floor (w = 0) by
  w_{k+1} = w_k - dz div_h(u_h)_k.  The linear free surface leaves
  w at the top face nonzero: the advective flux through the top face
  carries the top cell's own value (so a uniform tracer, or a velocity
  uniform in depth, has no vertical advection); the floor flux is zero.
* p_hy at centres from dp/dz = b with p = 0 at the top face:
  p_{nz-1} = -dz b_{nz-1} / 2, p_k = p_{k+1} - dz (b_k + b_{k+1}) / 2.
* Vertical vorticity zeta at cell corners (x face i, y face j) from the
  metric circulation around the dual cell, divided by its area.
* At a u point: + zeta_hat Vbar, with Vbar the four-point average of v and
  zeta_hat the WENO reconstruction of zeta along y (corners j-2..j+3)
  upwinded by Vbar.  At a v point: - zeta_hat Ubar, reconstructed along x.
* Kinetic energy at centres, (u_i^2 + u_{i+1}^2 + v_j^2 + v_{j+1}^2) / 4,
  differenced to u and v points.
* Vertical advection d(W u)/dz - u dW/dz, W = w averaged to the u (v)
  column; d(W u)/dz in flux form with u reconstructed by WENO along z,
  upwinded by W.
* Coriolis f = 2 Omega sin(latitude of the point) times the four-point
  average of the other component.
* Hydrostatic pressure gradient (p_i - p_{i-1}) / dx, (p_j - p_{j-1}) / dy.
* Explicit vertical viscosity and diffusivity; the surface momentum flux is
  the kinematic wind stress (tau_x, tau_y) / rho_0; free-slip, no-flux
  floor; no horizontal closure.
* Tracers in flux form with face areas and cell volumes of the shell,
  WENO in every direction (stencils in index space).
* QAB2: X~ = X + dt [(3/2 + chi) G^n - (1/2 + chi) G^{n-1}], chi = 0.1,
  chi = -1/2 on a first step, for u, v, T, S.  Gbar = sum_k dz of the same
  combination of G_u, G_v.
"""
import numpy as np

from .weno import reconstruct
from . import free_surface as fs

H = 3
CHI = 0.1


class LatLonGrid:
    """Lat-lon C-grid: metric factors as functions of the row index (any
    integer, so they continue past the walls)."""

    def __init__(self, ph):
        self.nx, self.ny, self.nz = ph.nx, ph.ny, ph.nz
        self.R = ph.radius
        self.dlam = np.deg2rad(ph.lon_extent / ph.nx)
        self.dphi = np.deg2rad(ph.lat_extent / ph.ny)
        self.phi0 = np.deg2rad(ph.lat0)
        self.dz = ph.depth / ph.nz
        self.dy = self.R * self.dphi
        self.lat0, self.lat_extent, self.lon_extent = ph.lat0, ph.lat_extent, ph.lon_extent

    def phi_c(self, j):
        return self.phi0 + (np.asarray(j, float) + 0.5) * self.dphi

    def phi_f(self, j):
        return self.phi0 + np.asarray(j, float) * self.dphi

    def dx_c(self, j):
        """x spacing along row j (between u points, and between centres)."""
        return self.R * np.cos(self.phi_c(j)) * self.dlam

    def dx_f(self, j):
        """x length of y face j."""
        return self.R * np.cos(self.phi_f(j)) * self.dlam

    def area_c(self, j):
        return self.R ** 2 * self.dlam * (np.sin(self.phi_f(np.asarray(j) + 1)) - np.sin(self.phi_f(j)))

    def area_corner(self, j):
        """Area of the dual cell around y face j (between rows j-1 and j)."""
        return self.R ** 2 * self.dlam * (np.sin(self.phi_c(j)) - np.sin(self.phi_c(np.asarray(j) - 1)))

    def metrics(self):
        return fs.latlon_metrics(self.nx, self.ny, self.lat0, self.lat_extent, self.R,
                                 self.lon_extent)


# ---------------------------------------------------------------------------
# Padded fields: index [H + k, H + j, H + i]
# ---------------------------------------------------------------------------

def pad(a, kind):
    """Interior (nz, ny, nx) ("c") or (nz, ny + 1, nx) ("v") -> padded copy
    with the halos of the readings above."""
    nz, nyi, nx = a.shape
    ny = nyi - 1 if kind == "v" else nyi
    P = np.zeros((nz + 2 * H, ny + 2 * H, nx + 2 * H))
    P[H:H + nz, H:H + nyi, H:H + nx] = a
    P[:, :, :H] = P[:, :, nx:nx + H]
    P[:, :, H + nx:] = P[:, :, H:2 * H]
    if kind == "c":
        for s in range(H):
            P[:, H - 1 - s] = P[:, H + s]
            P[:, H + ny + s] = P[:, H + ny - 1 - s]
    elif kind == "v":
        P[:, H] = 0.0
        P[:, H + ny] = 0.0
        for s in range(1, H + 1):
            P[:, H - s] = -P[:, H + s]
        for s in range(1, H):
            P[:, H + ny + s] = -P[:, H + ny - s]
    else:
        raise ValueError(kind)
    for s in range(H):
        P[H - 1 - s] = P[H + s]
        P[H + nz + s] = P[H + nz - 1 - s]
    return P


def blk(P, k0, k1, j0, j1, i0, i1):
    """P over the index ranges [k0, k1) x [j0, j1) x [i0, i1) (interior
    indices, which may reach into the halo)."""
    return P[H + k0:H + k1, H + j0:H + j1, H + i0:H + i1]


# ---------------------------------------------------------------------------
# Diagnostic fields
# ---------------------------------------------------------------------------

def horizontal_divergence(up, vp, g, i0, i1):
    """div_h(u_h) at centres, rows 0..ny-1, columns [i0, i1)."""
    nz, ny = g.nz, g.ny
    j = np.arange(ny)
    fx = g.dy * (blk(up, 0, nz, 0, ny, i0 + 1, i1 + 1) - blk(up, 0, nz, 0, ny, i0, i1))
    fy = (g.dx_f(j + 1)[None, :, None] * blk(vp, 0, nz, 1, ny + 1, i0, i1)
          - g.dx_f(j)[None, :, None] * blk(vp, 0, nz, 0, ny, i0, i1))
    return (fx + fy) / g.area_c(j)[None, :, None]


def diagnose_w(up, vp, g, i0=0, i1=None):
    """w at the nz + 1 z faces, columns [i0, i1): w_0 = 0,
    w_{k+1} = w_k - dz div_h(u_h)_k."""
    i1 = g.nx if i1 is None else i1
    div = horizontal_divergence(up, vp, g, i0, i1)
    w = np.zeros((g.nz + 1,) + div.shape[1:])
    for k in range(g.nz):
        w[k + 1] = w[k] - g.dz * div[k]
    return w


def hydrostatic_pressure(b, dz):
    """p_hy at centres: p_{nz-1} = -dz b_{nz-1} / 2,
    p_k = p_{k+1} - dz (b_k + b_{k+1}) / 2."""
    nz = b.shape[0]
    p = np.zeros_like(b)
    p[nz - 1] = -0.5 * dz * b[nz - 1]
    for k in range(nz - 2, -1, -1):
        p[k] = p[k + 1] - 0.5 * dz * (b[k] + b[k + 1])
    return p


def vorticity(up, vp, g, j0, j1, i0, i1):
    """zeta at corners (x face i, y face j) for j in [j0, j1), i in [i0, i1):
    [dy (v_{i,j} - v_{i-1,j}) - (dx_c(j) u_{i,j} - dx_c(j-1) u_{i,j-1})]
    / area of the dual cell."""
    nz = g.nz
    j = np.arange(j0, j1)
    circ = (g.dy * (blk(vp, 0, nz, j0, j1, i0, i1) - blk(vp, 0, nz, j0, j1, i0 - 1, i1 - 1))
            - (g.dx_c(j)[None, :, None] * blk(up, 0, nz, j0, j1, i0, i1)
               - g.dx_c(j - 1)[None, :, None] * blk(up, 0, nz, j0 - 1, j1 - 1, i0, i1)))
    return circ / g.area_corner(j)[None, :, None]


def buoyancy(T, S, ph):
    return ph.g * (ph.alpha * (T - ph.t_ref) - ph.beta * (S - ph.s_ref))


# ---------------------------------------------------------------------------
# Tendencies
# ---------------------------------------------------------------------------

def _rec(ph, qs, vel):
    return reconstruct(ph.advection, qs, vel, ph.weno_eps, ph.weno_q)


def _vertical_flux(col_p, W, ph, nz):
    """W * WENO_z(q) at the nz + 1 faces of padded columns col_p (shape
    (nz + 2H, ...)); zero at the floor, W * q_{nz-1} at the top face."""
    qs = [col_p[H + o:H + o + nz + 1] for o in range(-3, 3)]
    F = W * _rec(ph, qs, W)
    F[0] = 0.0
    F[nz] = W[nz] * col_p[H + nz - 1]
    return F


def tendencies(state, ph, g, tau_x, tau_y):
    """G_u (nz, ny, nx), G_v (nz, ny + 1, nx; zero on the walls), G_T, G_S.

    state: interior u (nz, ny, nx), v (nz, ny + 1, nx), T, S (nz, ny, nx).
    tau_x (ny, nx), tau_y (ny + 1, nx): kinematic surface stress at u and v
    points.  Returns (G, diagnostics)."""
    nx, ny, nz = g.nx, g.ny, g.nz
    dz = g.dz
    up, vp = pad(state["u"], "c"), pad(state["v"], "v")
    jc = np.arange(ny)
    jf = np.arange(ny + 1)

    # diagnostic fields
    w = diagnose_w(up, vp, g, -1, nx)                # columns -1..nx-1
    wc = w[:, :, 1:]                                 # columns 0..nx-1
    b = buoyancy(state["T"], state["S"], ph)
    p = hydrostatic_pressure(b, dz)
    pp = pad(p, "c")
    zeta = vorticity(up, vp, g, -2, ny + 3, -2, nx + 3)   # corners j, i in [-2, n+2]

    def Z(j0, j1, i0, i1):
        return zeta[:, j0 + 2:j1 + 2, i0 + 2:i1 + 2]

    ke = 0.25 * (blk(up, 0, nz, -1, ny + 1, -1, nx + 1) ** 2
                 + blk(up, 0, nz, -1, ny + 1, 0, nx + 2) ** 2
                 + blk(vp, 0, nz, -1, ny + 1, -1, nx + 1) ** 2
                 + blk(vp, 0, nz, 0, ny + 2, -1, nx + 1) ** 2)   # rows, cols -1..n

    def KE(j0, j1, i0, i1):
        return ke[:, j0 + 1:j1 + 1, i0 + 1:i1 + 1]

    # ---- u points (x face i, row j)
    u = blk(up, 0, nz, 0, ny, 0, nx)
    vbar = 0.25 * (blk(vp, 0, nz, 0, ny, -1, nx - 1) + blk(vp, 0, nz, 0, ny, 0, nx)
                   + blk(vp, 0, nz, 1, ny + 1, -1, nx - 1) + blk(vp, 0, nz, 1, ny + 1, 0, nx))
    zs = [Z(o, ny + o, 0, nx) for o in range(-2, 4)]          # corners j-2..j+3
    Gu = _rec(ph, zs, vbar) * vbar
    Gu += 2 * ph.omega * np.sin(g.phi_c(jc))[None, :, None] * vbar
    dxc = g.dx_c(jc)[None, :, None]
    Gu -= (KE(0, ny, 0, nx) - KE(0, ny, -1, nx - 1)) / dxc
    Gu -= (blk(pp, 0, nz, 0, ny, 0, nx) - blk(pp, 0, nz, 0, ny, -1, nx - 1)) / dxc
    Wu = 0.5 * (w[:, :, 0:nx] + w[:, :, 1:nx + 1])
    Fz = _vertical_flux(up[:, H:H + ny, H:H + nx], Wu, ph, nz)
    Gu -= (Fz[1:] - Fz[:-1]) / dz - u * (Wu[1:] - Wu[:-1]) / dz
    Fv = np.zeros((nz + 1, ny, nx))
    Fv[1:nz] = ph.nu * (u[1:] - u[:-1]) / dz
    Fv[nz] = tau_x
    Gu += (Fv[1:] - Fv[:-1]) / dz

    # ---- v points (x centre i, y face j), faces 1..ny-1
    v = blk(vp, 0, nz, 0, ny + 1, 0, nx)
    ubar = 0.25 * (blk(up, 0, nz, -1, ny, 0, nx) + blk(up, 0, nz, -1, ny, 1, nx + 1)
                   + blk(up, 0, nz, 0, ny + 1, 0, nx) + blk(up, 0, nz, 0, ny + 1, 1, nx + 1))
    zs = [Z(0, ny + 1, o, nx + o) for o in range(-2, 4)]      # corners i-2..i+3
    Gv = -_rec(ph, zs, ubar) * ubar
    Gv -= 2 * ph.omega * np.sin(g.phi_f(jf))[None, :, None] * ubar
    Gv -= (KE(0, ny + 1, 0, nx) - KE(-1, ny, 0, nx)) / g.dy
    Gv -= (blk(pp, 0, nz, 0, ny + 1, 0, nx) - blk(pp, 0, nz, -1, ny, 0, nx)) / g.dy
    wpad = np.zeros((nz + 1, ny + 2, nx))
    wpad[:, 1:ny + 1] = wc
    Wv = 0.5 * (wpad[:, 0:ny + 1] + wpad[:, 1:ny + 2])       # used on faces 1..ny-1 only
    Fz = _vertical_flux(vp[:, H:H + ny + 1, H:H + nx], Wv, ph, nz)
    Gv -= (Fz[1:] - Fz[:-1]) / dz - v * (Wv[1:] - Wv[:-1]) / dz
    Fv = np.zeros((nz + 1, ny + 1, nx))
    Fv[1:nz] = ph.nu * (v[1:] - v[:-1]) / dz
    Fv[nz] = tau_y
    Gv += (Fv[1:] - Fv[:-1]) / dz
    Gv[:, 0] = 0.0
    Gv[:, ny] = 0.0

    # ---- tracers
    Ax = g.dy * dz
    Ay = (g.dx_f(jf) * dz)[None, :, None]
    Az = g.area_c(jc)[None, :, None]
    vol = Az * dz
    uf = blk(up, 0, nz, 0, ny, 0, nx + 1)
    G = {"u": Gu, "v": Gv}
    for name in ("T", "S"):
        if name not in state:
            continue
        cp = pad(state[name], "c")
        Fx = uf * _rec(ph, [blk(cp, 0, nz, 0, ny, o, nx + 1 + o) for o in range(-3, 3)], uf) * Ax
        Fy = v * _rec(ph, [blk(cp, 0, nz, o, ny + 1 + o, 0, nx) for o in range(-3, 3)], v) * Ay
        Fy[:, 0] = 0.0
        Fy[:, ny] = 0.0
        Fzt = _vertical_flux(cp[:, H:H + ny, H:H + nx], wc, ph, nz) * Az
        c = blk(cp, 0, nz, 0, ny, 0, nx)
        Fzt[1:nz] -= ph.kappa * (c[1:] - c[:-1]) / dz * Az
        G[name] = -((Fx[:, :, 1:] - Fx[:, :, :-1]) + (Fy[:, 1:] - Fy[:, :-1])
                    + (Fzt[1:] - Fzt[:-1])) / vol
    return G, {"w": wc, "p": p, "zeta": zeta, "b": b}


# ---------------------------------------------------------------------------
# Time stepping
# ---------------------------------------------------------------------------

PROGNOSTIC = ("u", "v", "T", "S")


def qab2(X, Gn, Gm, dt):
    """QAB2 predictor; Gm None means a first step (chi = -1/2)."""
    chi = -0.5 if Gm is None else CHI
    comb = (1.5 + chi) * Gn
    if Gm is not None:
        comb = comb - (0.5 + chi) * Gm
    return X + dt * comb, comb


def step(state, Gprev, ph, g, tau_x, tau_y, dt, N, weights):
    """One baroclinic step.  state: u, v, T, S (3D) and eta, U, V (2D).
    Gprev: the previous step's tendencies, or None for a first step.
    Returns (new state, G, Gbar = (GU, GV))."""
    Gn, _ = tendencies(state, ph, g, tau_x, tau_y)
    new = {}
    comb = {}
    for n in PROGNOSTIC:
        new[n], comb[n] = qab2(state[n], Gn[n], None if Gprev is None else Gprev[n], dt)
    GU = g.dz * comb["u"].sum(axis=0)
    GV = g.dz * comb["v"].sum(axis=0)
    m = g.metrics()
    _, _, _, eb, ub, vb = fs.substeps(state["eta"], state["U"], state["V"], GU, GV,
                                      ph.g, ph.depth, dt, N, weights, m)
    dzv = np.full(g.nz, g.dz)
    new["u"] = fs.correct_baroclinic(new["u"], dzv, ub, ph.depth)
    vc = new["v"].copy()
    vc[:, 1:g.ny] = fs.correct_baroclinic(vc[:, 1:g.ny], dzv, vb[1:g.ny], ph.depth)
    vc[:, 0] = 0.0
    vc[:, g.ny] = 0.0
    new["v"] = vc
    new["eta"], new["U"], new["V"] = eb, ub, vb
    return new, Gn, (GU, GV)


def run(state, ph, tau_x, tau_y, dt, N, weights, nsteps):
    g = LatLonGrid(ph)
    G = None
    for _ in range(nsteps):
        state, G, _ = step(state, G, ph, g, tau_x, tau_y, dt, N, weights)
    return state, G
