"""Eddy-viscosity LES closures (closure paragraph of the nonhydrostatic model
section: the closure flux divergence d_m tau_nm for SmagorinskyLilly, and the
AnisotropicMinimumDissipation closure it lists), on the C-grid of the
finite-volume appendix.  Test infrastructure: the oracle of the GPU path.

Eddy viscosity at cell centres:

* Smagorinsky-Lilly (Smagorinsky 1963; Lilly's stratification factor):
    nu_e = (C_s Delta)^2 |S| sqrt(max(0, 1 - C_b N^2 / |S|^2)),
  S_ij = (d_j u_i + d_i u_j) / 2, |S| = sqrt(2 S_ij S_ij), N^2 = db/dz,
  Delta = (dx dy dzc)^(1/3);
* anisotropic minimum dissipation (Rozema et al. 2015; Abkar et al. 2016;
  Vreugdenhil & Taylor 2018):
    nu_e = max(0, -C sum_k Delta_k^2 (d_k u_i)(d_k u_j) S_ij / (d_l u_m d_l u_m)),
    kappa_e(c) = max(0, -C sum_k Delta_k^2 (d_k u_i)(d_k c)(d_i c) / (d_l c d_l c)).
  Smagorinsky-Lilly uses kappa_e = nu_e / Pr.

The closure then adds d_j(2 nu_e S_ij) to G_ui and d_i(kappa_e d_i c) to
G_c, as flux divergences with the fluxes at their natural C-grid locations.

Readings (the paper names the models and prints the Smagorinsky-Lilly flux
in a notation whose constants are ambiguous):
* the standard forms above, C_s = 0.16, C_b = 1, Pr = 1, C = 1/12;
* the diagonal strain components live at cell centres; the off-diagonal
  ones at the cell edges (xy at (F,F,C), xz at (F,C,F), yz at (C,F,F)).
  Smagorinsky-Lilly's |S|^2 averages the squared edge values to the centre
  (four edges each); AMD averages the edge gradients themselves (it needs
  their signs);
* N^2 at a centre is the mean of the buoyancy gradients on its two z faces
  (zero on a wall face); tracer gradients likewise for AMD (two faces);
* the viscosity on an edge is the mean of the four surrounding centres,
  the diffusivity on a face the mean of its two centres;
* walls: the mirror halos make the wall values of S_xz, S_yz and dc/dz zero,
  and the diffusive fluxes through the wall faces are zero; the prescribed
  top flux stays with the explicit tendency.
"""
import numpy as np

from .fv import H, z_spacings

CS, CB, PR = 0.16, 1.0, 1.0
CAMD = 1.0 / 12.0


def _grid(ph):
    dx, dy, _ = ph.spacing
    dzc, dzf = z_spacings(ph)
    return dx, dy, dzc, dzf


class _P:
    """Padded-array accessor with interior offsets: a[k + dk, j + dj, i + di]
    over the interior (and one extra layer where asked)."""

    def __init__(self, ph):
        self.ph = ph

    def v(self, a, di=0, dj=0, dk=0, ni=0, nj=0, nk=0):
        ph = self.ph
        return a[H + dk:H + dk + ph.nz + nk, H + dj:H + dj + ph.ny + nj, H + di:H + di + ph.nx + ni]


def velocity_gradients(s, ph):
    """Gradient components at their natural locations, each an array over the
    interior with one extra entry along the axes needed to average to
    centres:  diagonal (C,C,C); d u/dy, d v/dx at (F,F,C) for faces
    i = 0..nx, j = 0..ny; d u/dz, d w/dx at (F,C,F), k = 0..nz; d v/dz,
    d w/dy at (C,F,F)."""
    dx, dy, dzc, dzf = _grid(ph)
    p = _P(ph)
    u, v, w = s["u"], s["v"], s["w"]
    g = {}
    g["ux"] = (p.v(u, di=1) - p.v(u)) / dx
    g["vy"] = (p.v(v, dj=1) - p.v(v)) / dy
    g["wz"] = (p.v(w, dk=1) - p.v(w)) / dzc[:, None, None]
    # (F,F,C) edges: x faces i = 0..nx, y faces j = 0..ny
    g["uy"] = (p.v(u, nj=1, ni=1) - p.v(u, dj=-1, nj=1, ni=1)) / dy
    g["vx"] = (p.v(v, nj=1, ni=1) - p.v(v, di=-1, nj=1, ni=1)) / dx
    # (F,C,F): x faces i = 0..nx, z faces k = 0..nz
    dzf3 = dzf[:, None, None]
    g["uz"] = (p.v(u, nk=1, ni=1) - p.v(u, dk=-1, nk=1, ni=1)) / dzf3
    g["wx"] = (p.v(w, nk=1, ni=1) - p.v(w, di=-1, nk=1, ni=1)) / dx
    # (C,F,F): y faces j = 0..ny, z faces k = 0..nz
    g["vz"] = (p.v(v, nk=1, nj=1) - p.v(v, dk=-1, nk=1, nj=1)) / dzf3
    g["wy"] = (p.v(w, nk=1, nj=1) - p.v(w, dj=-1, nk=1, nj=1)) / dy
    if ph.z_bounded:
        # wall faces: u, v mirror evenly and w vanishes, so these are zero
        for key in ("uz", "wx", "vz", "wy"):
            g[key][0] = 0.0
            g[key][ph.nz] = 0.0
    return g


def _avg_ffc(a):
    return 0.25 * (a[:, :-1, :-1] + a[:, 1:, :-1] + a[:, :-1, 1:] + a[:, 1:, 1:])


def _avg_fcf(a):
    return 0.25 * (a[:-1, :, :-1] + a[1:, :, :-1] + a[:-1, :, 1:] + a[1:, :, 1:])


def _avg_cff(a):
    return 0.25 * (a[:-1, :-1, :] + a[1:, :-1, :] + a[:-1, 1:, :] + a[1:, 1:, :])


def _buoyancy_gradient(s, ph):
    """N^2 = db/dz at centres: the mean of the face gradients (0 on walls)."""
    dx, dy, dzc, dzf = _grid(ph)
    p = _P(ph)
    b = ph.g * (ph.alpha * (s["T"] - ph.t_ref) - ph.beta * (s["S"] - ph.s_ref))
    gz = (p.v(b, nk=1) - p.v(b, dk=-1, nk=1)) / dzf[:, None, None]
    if ph.z_bounded:
        gz[0] = 0.0
        gz[ph.nz] = 0.0
    return 0.5 * (gz[1:] + gz[:-1])


def smagorinsky_viscosity(s, ph, cs=CS, cb=CB):
    dx, dy, dzc, _ = _grid(ph)
    g = velocity_gradients(s, ph)
    sxy2 = _avg_ffc((0.5 * (g["uy"] + g["vx"])) ** 2)
    sxz2 = _avg_fcf((0.5 * (g["uz"] + g["wx"])) ** 2)
    syz2 = _avg_cff((0.5 * (g["vz"] + g["wy"])) ** 2)
    s2 = 2.0 * (g["ux"] ** 2 + g["vy"] ** 2 + g["wz"] ** 2) + 4.0 * (sxy2 + sxz2 + syz2)
    delta = (dx * dy * dzc[:, None, None]) ** (1.0 / 3.0)
    n2 = _buoyancy_gradient(s, ph) if ph.buoyancy else np.zeros_like(s2)
    with np.errstate(divide="ignore", invalid="ignore"):
        fac = np.where(s2 > 0, np.maximum(0.0, 1.0 - cb * n2 / np.where(s2 > 0, s2, 1.0)), 0.0)
    return (cs * delta) ** 2 * np.sqrt(s2) * np.sqrt(fac)


def _centre_gradient_tensor(s, ph):
    """The nine d_k u_i at cell centres (edge components averaged from their
    four edges): G[i][k] = d u_i / d x_k."""
    g = velocity_gradients(s, ph)
    uy, vx = _avg_ffc(g["uy"]), _avg_ffc(g["vx"])
    uz, wx = _avg_fcf(g["uz"]), _avg_fcf(g["wx"])
    vz, wy = _avg_cff(g["vz"]), _avg_cff(g["wy"])
    return [[g["ux"], uy, uz], [vx, g["vy"], vz], [wx, wy, g["wz"]]]


def amd_nu_from_gradients(G, D, c=CAMD):
    """AMD eddy viscosity from the velocity gradient tensor G[i][k] =
    d u_i / d x_k and the filter widths D[k]."""
    S = [[0.5 * (G[i][j] + G[j][i]) for j in range(3)] for i in range(3)]
    num = 0.0
    for k in range(3):
        for i in range(3):
            for j in range(3):
                num = num + D[k] ** 2 * G[i][k] * G[j][k] * S[i][j]
    den = sum(G[i][k] ** 2 for i in range(3) for k in range(3))
    num, den = np.asarray(num, dtype=float), np.asarray(den, dtype=float)
    with np.errstate(divide="ignore", invalid="ignore"):
        nu = np.where(den > 0, -c * num / np.where(den > 0, den, 1.0), 0.0)
    return np.maximum(nu, 0.0)


def amd_kappa_from_gradients(G, gc, D, c=CAMD):
    """AMD eddy diffusivity from G and the tracer gradient gc[k]."""
    num = 0.0
    for k in range(3):
        for i in range(3):
            num = num + D[k] ** 2 * G[i][k] * gc[k] * gc[i]
    den = gc[0] ** 2 + gc[1] ** 2 + gc[2] ** 2
    num, den = np.asarray(num, dtype=float), np.asarray(den, dtype=float)
    with np.errstate(divide="ignore", invalid="ignore"):
        kap = np.where(den > 0, -c * num / np.where(den > 0, den, 1.0), 0.0)
    return np.maximum(kap, 0.0)


def _widths(ph):
    dx, dy, dzc, _ = _grid(ph)
    return [dx, dy, dzc[:, None, None]]


def amd_viscosity(s, ph, c=CAMD):
    return amd_nu_from_gradients(_centre_gradient_tensor(s, ph), _widths(ph), c)


def tracer_centre_gradient(s, name, ph):
    """d c / d x_k at centres: means of the two face gradients (0 on walls)."""
    dx, dy, dzc, dzf = _grid(ph)
    p = _P(ph)
    q = s[name]
    cx = (p.v(q, ni=1) - p.v(q, di=-1, ni=1)) / dx
    cy = (p.v(q, nj=1) - p.v(q, dj=-1, nj=1)) / dy
    cz = (p.v(q, nk=1) - p.v(q, dk=-1, nk=1)) / dzf[:, None, None]
    if ph.z_bounded:
        cz[0] = 0.0
        cz[ph.nz] = 0.0
    return [0.5 * (cx[:, :, 1:] + cx[:, :, :-1]), 0.5 * (cy[:, 1:] + cy[:, :-1]),
            0.5 * (cz[1:] + cz[:-1])]


def amd_diffusivity(s, name, ph, c=CAMD):
    """AMD eddy diffusivity of tracer `name` at centres."""
    return amd_kappa_from_gradients(_centre_gradient_tensor(s, ph),
                                    tracer_centre_gradient(s, name, ph), _widths(ph), c)


def _pad_centre(a, ph):
    """A centred interior field with periodic x, y and mirrored z images."""
    out = np.zeros((ph.nz + 2, ph.ny + 2, ph.nx + 2))
    out[1:-1, 1:-1, 1:-1] = a
    out[1:-1, 1:-1, 0] = a[:, :, -1]
    out[1:-1, 1:-1, -1] = a[:, :, 0]
    out[:, 0, :] = out[:, -2, :]
    out[:, -1, :] = out[:, 1, :]
    if ph.z_bounded:
        out[0] = out[1]
        out[-1] = out[-2]
    else:
        out[0] = out[-2]
        out[-1] = out[1]
    return out


def stress_divergence(s, nu_e, ph):
    """d_j (2 nu_e S_ij) for u, v, w (w: nz + 1 faces with zero wall faces)."""
    dx, dy, dzc, dzf = _grid(ph)
    nz = ph.nz
    g = velocity_gradients(s, ph)
    N = _pad_centre(nu_e, ph)            # index [k+1, j+1, i+1] = centre (k, j, i)
    nc = N[1:-1, 1:-1, 1:-1]
    # edge viscosities: four surrounding centres
    n_ffc = 0.25 * (N[1:-1, :-1, :-1] + N[1:-1, 1:, :-1] + N[1:-1, :-1, 1:] + N[1:-1, 1:, 1:])
    n_fcf = 0.25 * (N[:-1, 1:-1, :-1] + N[1:, 1:-1, :-1] + N[:-1, 1:-1, 1:] + N[1:, 1:-1, 1:])
    n_cff = 0.25 * (N[:-1, :-1, 1:-1] + N[1:, :-1, 1:-1] + N[:-1, 1:, 1:-1] + N[1:, 1:, 1:-1])
    # stresses 2 nu S at their locations
    txx = 2.0 * nc * g["ux"]
    tyy = 2.0 * nc * g["vy"]
    tzz = 2.0 * nc * g["wz"]
    txy = n_ffc * (g["uy"] + g["vx"])      # (F,F,C), i, j = 0..n
    txz = n_fcf * (g["uz"] + g["wx"])      # (F,C,F)
    tyz = n_cff * (g["vz"] + g["wy"])      # (C,F,F)
    if ph.z_bounded:
        txz[0] = txz[nz] = 0.0
        tyz[0] = tyz[nz] = 0.0
    dzc3, dzf3 = dzc[:, None, None], dzf[:, None, None]
    # u at face i: x flux at centres i-1, i (periodic), y flux at edges, z flux
    Gu = ((txx - np.roll(txx, 1, axis=2)) / dx
          + (txy[:, 1:, :-1] - txy[:, :-1, :-1]) / dy
          + (txz[1:, :, :-1] - txz[:-1, :, :-1]) / dzc3)
    Gv = ((txy[:, :-1, 1:] - txy[:, :-1, :-1]) / dx
          + (tyy - np.roll(tyy, 1, axis=1)) / dy
          + (tyz[1:, :-1, :] - tyz[:-1, :-1, :]) / dzc3)
    # w at face k (k = 0..nz-1 computed; the w cell about face k is dzf[k] thick)
    tzz_below = np.concatenate([tzz[:1] if not ph.z_bounded else tzz[:1], tzz], axis=0)
    if ph.z_bounded:
        # the centre below face 0 is the mirror image: w odd, so d w/dz even
        tzz_below[0] = tzz[0]
    else:
        tzz_below[0] = tzz[-1]
    Gw = ((txz[:nz, :, 1:] - txz[:nz, :, :-1]) / dx
          + (tyz[:nz, 1:, :] - tyz[:nz, :-1, :]) / dy
          + (tzz_below[1:] - tzz_below[:-1]) / dzf3[:nz])
    if ph.z_bounded:
        Gw = np.concatenate([Gw, np.zeros((1, ph.ny, ph.nx))], axis=0)
        Gw[0] = 0.0
        Gw[nz] = 0.0
    return Gu, Gv, Gw


def tracer_diffusion(s, name, kap_e, ph):
    """d_i (kappa_e d_i c) with face diffusivities (means of two centres) and
    no flux through the walls."""
    dx, dy, dzc, dzf = _grid(ph)
    p = _P(ph)
    q = s[name]
    K = _pad_centre(kap_e, ph)
    kx = 0.5 * (K[1:-1, 1:-1, :-1] + K[1:-1, 1:-1, 1:])      # faces i = 0..nx
    ky = 0.5 * (K[1:-1, :-1, 1:-1] + K[1:-1, 1:, 1:-1])
    kz = 0.5 * (K[:-1, 1:-1, 1:-1] + K[1:, 1:-1, 1:-1])      # faces k = 0..nz
    Fx = kx * (p.v(q, ni=1) - p.v(q, di=-1, ni=1)) / dx
    Fy = ky * (p.v(q, nj=1) - p.v(q, dj=-1, nj=1)) / dy
    Fz = kz * (p.v(q, nk=1) - p.v(q, dk=-1, nk=1)) / dzf[:, None, None]
    if ph.z_bounded:
        Fz[0] = 0.0
        Fz[ph.nz] = 0.0
    return ((Fx[:, :, 1:] - Fx[:, :, :-1]) / dx + (Fy[:, 1:] - Fy[:, :-1]) / dy
            + (Fz[1:] - Fz[:-1]) / dzc[:, None, None])


def les_tendencies(s, ph, kind):
    """The closure's contribution to G for kind 'smagorinsky' or 'amd'
    (constants from the physics record when it carries them)."""
    if kind == "smagorinsky":
        nu = smagorinsky_viscosity(s, ph, getattr(ph, "les_cs", CS), getattr(ph, "les_cb", CB))
        kap = {n: nu / getattr(ph, "les_pr", PR) for n in ph.tracers}
    elif kind == "amd":
        c = getattr(ph, "les_camd", CAMD)
        nu = amd_viscosity(s, ph, c)
        kap = {n: amd_diffusivity(s, n, ph, c) for n in ph.tracers}
    else:
        raise ValueError(kind)
    Gu, Gv, Gw = stress_divergence(s, nu, ph)
    out = {"u": Gu, "v": Gv, "w": Gw}
    for n in ph.tracers:
        out[n] = tracer_diffusion(s, n, kap[n], ph)
    return out
