"""Split-explicit barotropic substeps of the hydrostatic model (hydrostatic
time-discretisation appendix): forward-backward substeps of the depth-
integrated transport U_h = (U, V) and the free surface eta,

    eta^{n+1} = eta^n - dtau div_h(U_h^n)
    U_h^{n+1} = U_h^n - dtau [ g H grad_h eta^{n+1} - Gbar ]

with dtau = dt / N, M substeps, frozen slow forcing Gbar (the depth integral
of the QAB2 combination of the slow tendencies), and the running averages
Ubar = sum_{n=1..M} a_n U_h^n, etabar = sum_{n=1..M} a_n eta^n.  Afterwards
the baroclinic velocity is corrected so that its depth integral equals Ubar,
and eta, U_h restart from the averages.

Readings: linear free surface (H in place of H + eta); the averaging
weights a_n are an input (the paper's default filter is defined in a work
it cites); no Coriolis term in the substeps (it lives in Gbar).

Discretisation (finite-volume, C-grid, metric factors of a thin spherical
shell or of a uniform rectilinear grid): eta at cell centres, U at x faces,
V at y faces; x periodic; y periodic or bounded by walls where V = 0.
  div_h(U_h)_c = [ Ly (U_{i+1} - U_i) + Lx_{j+1} V_{j+1} - Lx_j V_j ] / A_c
  (grad eta)_x at a u face = (eta_i - eta_{i-1}) / dx_u,
  (grad eta)_y at a v face = (eta_j - eta_{j-1}) / dy_v.
"""
import numpy as np


class Metrics:
    """Metric factors of a 2D C-grid (arrays along y; uniform along x).

    len_u : (ny,)    length of an x face (meters)
    dx_u  : (ny,)    distance between the centres either side of an x face
    len_v : (nyf,)   length of a y face; nyf = ny + 1 with walls, ny periodic
    dy_v  : (nyf,)   distance between the centres either side of a y face
    area  : (ny,)    cell area
    """

    def __init__(self, nx, ny, len_u, dx_u, len_v, dy_v, area, y_walls):
        self.nx, self.ny = nx, ny
        self.len_u = np.asarray(len_u, float)
        self.dx_u = np.asarray(dx_u, float)
        self.len_v = np.asarray(len_v, float)
        self.dy_v = np.asarray(dy_v, float)
        self.area = np.asarray(area, float)
        self.y_walls = y_walls


def latlon_metrics(nx, ny, lat0_deg, lat_extent_deg, radius, lon_extent_deg=360.0):
    """Thin-shell spherical metrics of a latitude-longitude grid periodic in
    longitude with walls at the southern and northern edges."""
    dlam = np.deg2rad(lon_extent_deg / nx)
    dphi = np.deg2rad(lat_extent_deg / ny)
    phi_f = np.deg2rad(lat0_deg) + np.arange(ny + 1) * dphi   # y faces
    phi_c = phi_f[:-1] + 0.5 * dphi                            # centres
    len_u = np.full(ny, radius * dphi)
    dx_u = radius * np.cos(phi_c) * dlam
    len_v = radius * np.cos(phi_f) * dlam
    dy_v = np.full(ny + 1, radius * dphi)
    area = radius ** 2 * dlam * (np.sin(phi_f[1:]) - np.sin(phi_f[:-1]))
    return Metrics(nx, ny, len_u, dx_u, len_v, dy_v, area, True)


def rectilinear_metrics(nx, ny, dx, dy, y_walls=False):
    nyf = ny + 1 if y_walls else ny
    return Metrics(nx, ny, np.full(ny, dy), np.full(ny, dx), np.full(nyf, dx),
                   np.full(nyf, dy), np.full(ny, dx * dy), y_walls)


def divergence(U, V, m):
    """Transport divergence at cell centres.  U: (ny, nx); V: (nyf, nx)."""
    fx = m.len_u[:, None] * U
    d = np.roll(fx, -1, axis=1) - fx
    fy = m.len_v[:, None] * V
    if m.y_walls:
        d = d + (fy[1:] - fy[:-1])
    else:
        d = d + (np.roll(fy, -1, axis=0) - fy)
    return d / m.area[:, None]


def substep(eta, U, V, GU, GV, g, H, dtau, m):
    """One forward-backward substep; returns (eta^{n+1}, U^{n+1}, V^{n+1})."""
    eta1 = eta - dtau * divergence(U, V, m)
    gx = (eta1 - np.roll(eta1, 1, axis=1)) / m.dx_u[:, None]
    U1 = U - dtau * (g * H * gx - GU)
    if m.y_walls:
        V1 = V.copy()
        gy = (eta1[1:] - eta1[:-1]) / m.dy_v[1:-1, None]
        V1[1:-1] = V[1:-1] - dtau * (g * H * gy - GV[1:-1])
        V1[0] = 0.0
        V1[-1] = 0.0
    else:
        gy = (eta1 - np.roll(eta1, 1, axis=0)) / m.dy_v[:, None]
        V1 = V - dtau * (g * H * gy - GV)
    return eta1, U1, V1


def substeps(eta, U, V, GU, GV, g, H, dt, N, weights, m):
    """M = len(weights) substeps of length dt / N with running averages.
    Returns (eta^M, U^M, V^M, etabar, Ubar, Vbar)."""
    dtau = dt / N
    eb = np.zeros_like(eta)
    ub = np.zeros_like(U)
    vb = np.zeros_like(V)
    for a in weights:
        eta, U, V = substep(eta, U, V, GU, GV, g, H, dtau, m)
        eb += a * eta
        ub += a * U
        vb += a * V
    return eta, U, V, eb, ub, vb


def correct_baroclinic(u, dz, Ubar, H):
    """u_h^{m+1} = u~_h + (Ubar - sum_k dz_k u~_h) / H for a velocity u of
    shape (nz, ny, nx) at the points where Ubar lives."""
    return u + (Ubar - np.tensordot(dz, u, axes=(0, 0)))[None] / H
