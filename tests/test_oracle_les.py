"""Pins of the oracle's eddy-viscosity closures (Smagorinsky-Lilly and
anisotropic minimum dissipation) against closed forms and identities:
linear shear and stratification give the textbook viscosities, AMD vanishes
for pure shear and rotation and has a closed form for axisymmetric strain,
the stress divergence with a constant viscosity is the Laplacian of a
divergence-free velocity (the pinned constant closure), momentum and tracers
are conserved, and the kinetic-energy change equals minus the discrete
dissipation (summation by parts)."""
import dataclasses

import numpy as np
import pytest

from paper_2502_14148_amd import inputs
from oracle import fv, les, tendencies as td, timestep


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _phys(n=(8, 8, 16), stretched=False, **kw):
    ph = inputs.convection_physics(n, (2.0 * n[0], 3.0 * n[1], 1.0 * n[2]), **kw)
    if stretched:
        ph.z_faces = inputs.stretched_faces(n[2], ph.lz, ph.z0, 1.5)
    return ph


def _shear_state(ph, a, n2=0.0):
    """u = a z at the centres (uniform in x, y), v = w = 0; T linear in z so
    that db/dz = n2; S uniform."""
    nz, ny, nx = ph.nz, ph.ny, ph.nx
    zc = inputs.cell_centres_z(ph)
    s = {"u": np.broadcast_to((a * zc)[:, None, None], (nz, ny, nx)).copy(),
         "v": np.zeros((nz, ny, nx)), "w": np.zeros((nz + 1, ny, nx)),
         "T": np.broadcast_to((20.0 + n2 / (ph.g * ph.alpha) * zc)[:, None, None],
                              (nz, ny, nx)).copy(),
         "S": np.full((nz, ny, nx), 35.0)}
    return timestep.make_state(s, ph)


@pytest.mark.parametrize("stretched", [False, True])
def test_smagorinsky_linear_shear(stretched):
    """du/dz = a on every interior face: |S| = |a| away from the walls (the
    wall faces carry zero shear, so the wall cells see half of |S|^2), and
    nu_e = (C_s Delta)^2 |S| with Delta = (dx dy dzc)^(1/3)."""
    ph = _phys(stretched=stretched)
    ph.buoyancy = False
    a = 0.03
    nu = les.smagorinsky_viscosity(_shear_state(ph, a), ph)
    dx, dy, _ = ph.spacing
    dzc, _ = fv.z_spacings(ph)
    delta = (dx * dy * dzc) ** (1.0 / 3.0)
    want = (les.CS * delta) ** 2 * a
    want[0] /= np.sqrt(2.0)
    want[-1] /= np.sqrt(2.0)
    assert np.allclose(nu, want[:, None, None], rtol=1e-13, atol=0)


@pytest.mark.parametrize("n2,frac", [(2e-4, 1.0 - 2e-4 / 9e-4), (1e-3, 0.0)])
def test_smagorinsky_lilly_stratification(n2, frac):
    """Interior cells of a linearly stratified shear: the Lilly factor
    sqrt(max(0, 1 - C_b N^2 / |S|^2)), zero once N^2 exceeds |S|^2."""
    ph = _phys()
    a = 0.03
    nu = les.smagorinsky_viscosity(_shear_state(ph, a, n2), ph)
    dx, dy, dz = ph.spacing
    want = (les.CS * (dx * dy * dz) ** (1.0 / 3.0)) ** 2 * a * np.sqrt(frac)
    assert np.allclose(nu[1:-1], want, rtol=1e-12, atol=1e-20)


def test_amd_closed_forms():
    D = [1.0, 1.0, 1.0]
    a, c = 0.7, les.CAMD
    strain = [[a, 0, 0], [0, a, 0], [0, 0, -2 * a]]
    assert np.isclose(les.amd_nu_from_gradients(strain, D), c * a, rtol=1e-14)
    assert les.amd_nu_from_gradients([[0, 0, a], [0, 0, 0], [0, 0, 0]], D) == 0.0   # shear
    rot = [[0, -a, 0], [a, 0, 0], [0, 0, 0]]
    assert les.amd_nu_from_gradients(rot, D) == 0.0
    # stretching along z (a < 0 compresses x, y): no eddy viscosity
    assert les.amd_nu_from_gradients([[-a, 0, 0], [0, -a, 0], [0, 0, 2 * a]], D) == 0.0
    # anisotropic widths weight each direction by Delta_k^2
    Dz = [1.0, 1.0, 0.5]
    num = -(a ** 3 * (1 + 1) + (-2 * a) ** 3 * 0.25)
    assert np.isclose(les.amd_nu_from_gradients(strain, Dz), c * num / (6 * a * a), rtol=1e-14)
    # diffusivity: a vertical tracer gradient under axisymmetric strain
    g = 0.3
    assert np.isclose(les.amd_kappa_from_gradients(strain, [0, 0, g], D), 2 * c * a, rtol=1e-14)
    assert les.amd_kappa_from_gradients(strain, [g, 0, 0], D) == 0.0


def test_velocity_gradients_exact_for_linear_fields():
    """Linear profiles in z (centred u, v; w on faces) give their slopes."""
    ph = _phys(stretched=True)
    nz, ny, nx = ph.nz, ph.ny, ph.nx
    zc = inputs.cell_centres_z(ph)
    zf = np.asarray(ph.z_faces)
    s = timestep.make_state({"u": np.broadcast_to(0.2 * zc[:, None, None], (nz, ny, nx)).copy(),
                             "v": np.broadcast_to(-0.5 * zc[:, None, None], (nz, ny, nx)).copy(),
                             "w": np.zeros((nz + 1, ny, nx)),
                             "T": np.zeros((nz, ny, nx)), "S": np.zeros((nz, ny, nx))}, ph)
    g = les.velocity_gradients(s, ph)
    assert np.allclose(g["uz"][1:nz], 0.2, rtol=1e-13) and np.all(g["uz"][0] == 0)
    assert np.allclose(g["vz"][1:nz], -0.5, rtol=1e-13)
    w = np.broadcast_to((zf - zf[0])[:, None, None] * (zf[-1] - zf)[:, None, None], (nz + 1, ny, nx))
    s["w"] = fv.to_padded(np.ascontiguousarray(w), ph, "w")
    g = les.velocity_gradients(s, ph)
    assert np.allclose(g["wz"][:, 0, 0], np.diff(w[:, 0, 0]) / np.diff(zf), rtol=1e-13)


def _random(ph, seed, vel=1e-2):
    s = inputs.random_state(ph, seed=seed, vel=vel)
    s["T"] += 20.0
    s["S"] += 35.0
    return timestep.make_state(s, ph)


@pytest.mark.parametrize("stretched", [False, True])
def test_constant_viscosity_stress_is_the_laplacian(stretched):
    """With nu_e = nu constant, d_j(nu (d_j u_i + d_i u_j)) = nu lap u_i for a
    discretely divergence-free velocity: the constant closure of the pinned
    tendencies (advection, Coriolis and buoyancy off)."""
    ph = _phys((8, 12, 16), stretched=stretched, nu=0.37, kappa=0.0)
    ph.advection, ph.f, ph.buoyancy = "none", 0.0, False
    st = _random(ph, 4)
    nu = np.full((ph.nz, ph.ny, ph.nx), ph.nu)
    Gu, Gv, Gw = les.stress_divergence(st, nu, ph)
    G = td.tendencies(st, ph)
    assert rel(Gu, G["u"]) < 1e-12
    assert rel(Gv, G["v"]) < 1e-12
    assert rel(Gw, G["w"]) < 1e-12


@pytest.mark.parametrize("kind", ["smagorinsky", "amd"])
def test_les_conservation_and_dissipation(kind):
    """Sum of V G over u, v and each tracer vanishes (periodic sides, no flux
    through the walls); the kinetic-energy change of the viscous terms
    equals minus the discrete dissipation sum 2 nu S:S over the stress
    locations, and is negative."""
    ph = _phys((12, 8, 16), stretched=True)
    st = _random(ph, 7, vel=0.05)
    G = les.les_tendencies(st, ph, kind)
    dx, dy, _ = ph.spacing
    dzc, dzf = fv.z_spacings(ph)
    V = dx * dy * dzc[:, None, None]
    for n in ("u", "v", "T", "S"):
        scale = np.sum(np.abs(G[n]) * V)
        assert abs(np.sum(G[n] * V)) < 1e-12 * scale, n
    u = fv.interior(st["u"], ph, "u")
    v = fv.interior(st["v"], ph, "v")
    w = fv.interior(st["w"], ph, "w")
    dK = np.sum(u * G["u"] * V) + np.sum(v * G["v"] * V) + \
        np.sum((w * G["w"])[1:ph.nz] * dx * dy * dzf[1:ph.nz, None, None])
    nu = les.smagorinsky_viscosity(st, ph) if kind == "smagorinsky" else les.amd_viscosity(st, ph)
    g = les.velocity_gradients(st, ph)
    N = les._pad_centre(nu, ph)
    n_ffc = 0.25 * (N[1:-1, :-1, :-1] + N[1:-1, 1:, :-1] + N[1:-1, :-1, 1:] + N[1:-1, 1:, 1:])
    n_fcf = 0.25 * (N[:-1, 1:-1, :-1] + N[1:, 1:-1, :-1] + N[:-1, 1:-1, 1:] + N[1:, 1:-1, 1:])
    n_cff = 0.25 * (N[:-1, :-1, 1:-1] + N[1:, :-1, 1:-1] + N[:-1, 1:, 1:-1] + N[1:, 1:, 1:-1])
    D = np.sum(2 * nu * (g["ux"] ** 2 + g["vy"] ** 2 + g["wz"] ** 2) * V)
    D += np.sum((n_ffc * (g["uy"] + g["vx"]) ** 2)[:, :-1, :-1] * V)
    D += np.sum((n_fcf * (g["uz"] + g["wx"]) ** 2)[:, :, :-1] * dx * dy * dzf[:, None, None])
    D += np.sum((n_cff * (g["vz"] + g["wy"]) ** 2)[:, :-1, :] * dx * dy * dzf[:, None, None])
    assert D > 0
    assert abs(dK + D) < 1e-12 * D


def test_amd_nonsymmetric_gradient_closed_forms():
    """Strain plus shear with anisotropic widths (1, 1/2, 1): the weights
    Delta_k^2 attach to the derivative direction k, not to the component."""
    a, b, c = 0.7, 0.4, les.CAMD
    G = [[a, b, 0], [0, a, 0], [0, 0, -2 * a]]
    D = [1.0, 0.5, 1.0]
    want = c * (6.75 * a ** 3 - 0.5 * a * b * b) / (6 * a * a + b * b)
    assert np.isclose(les.amd_nu_from_gradients(G, D), want, rtol=1e-14)
    Gc = [[-a, b, 0], [0, -a, 0], [0, 0, 2 * a]]
    assert np.isclose(les.amd_kappa_from_gradients(Gc, [1.0, 1.0, 0.0], D),
                      c * (1.25 * a - 0.25 * b) / 2.0, rtol=1e-14)


@pytest.mark.parametrize("kind", ["smagorinsky", "amd"])
def test_tracer_variance_dissipation(kind):
    """sum V c d_i(kappa d_i c) = -sum over faces V_f kappa_f (d c)^2 with
    the face diffusivity the mean of its two centres."""
    ph = _phys((12, 8, 16), stretched=True)
    st = _random(ph, 9, vel=0.05)
    G = les.les_tendencies(st, ph, kind)
    dx, dy, _ = ph.spacing
    dzc, dzf = fv.z_spacings(ph)
    c = fv.interior(st["T"], ph, "T")
    kap = les.smagorinsky_viscosity(st, ph) / les.PR if kind == "smagorinsky" \
        else les.amd_diffusivity(st, "T", ph)
    lhs = np.sum(c * G["T"] * dzc[:, None, None]) * dx * dy
    rhs = 0.0
    kx = 0.5 * (kap + np.roll(kap, 1, axis=2))
    rhs += np.sum(kx * ((c - np.roll(c, 1, axis=2)) / dx) ** 2 * dzc[:, None, None]) * dx * dy
    ky = 0.5 * (kap + np.roll(kap, 1, axis=1))
    rhs += np.sum(ky * ((c - np.roll(c, 1, axis=1)) / dy) ** 2 * dzc[:, None, None]) * dx * dy
    kz = 0.5 * (kap[1:] + kap[:-1])
    rhs += np.sum(kz * ((c[1:] - c[:-1]) / dzf[1:ph.nz, None, None]) ** 2
                  * dzf[1:ph.nz, None, None]) * dx * dy
    assert rhs > 0
    assert abs(lhs + rhs) < 1e-12 * rhs
