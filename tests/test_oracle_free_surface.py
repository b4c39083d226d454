"""Pins of the oracle's split-explicit barotropic substeps: the closed-form
amplification matrix of a periodic gravity wave, exact volume conservation,
exact response to uniform forcing, and the depth-integral identity of the
baroclinic correction."""
import numpy as np
import pytest

from oracle import free_surface as fs


def test_gravity_wave_matrix():
    """A single Fourier mode on a uniform periodic grid evolves by
    M = [[1, -dtau D], [-gH dtau G, 1 + gH dtau^2 G D]] per substep, with
    D = G = 2 i sin(k dx / 2) / dx (det M = 1)."""
    nx, ny, dx = 64, 4, 2.5e3
    g, H, dtau = 9.81, 3000.0, 7.0
    m = fs.rectilinear_metrics(nx, ny, dx, dx, y_walls=False)
    kk = 5
    k = 2 * np.pi * kk / (nx * dx)
    xc = (np.arange(nx) + 0.5) * dx
    xf = np.arange(nx) * dx
    e0, u0 = 0.3 + 0.1j, -2.0 + 0.5j
    eta = np.broadcast_to((e0 * np.exp(1j * k * xc)).real, (ny, nx)).copy()
    U = np.broadcast_to((u0 * np.exp(1j * k * xf)).real, (ny, nx)).copy()
    V = np.zeros((ny, nx))
    zero = np.zeros((ny, nx))
    D = 2j * np.sin(k * dx / 2) / dx
    Mx = np.array([[1, -dtau * D], [-g * H * dtau * D, 1 + g * H * dtau ** 2 * D * D]])
    assert abs(np.linalg.det(Mx) - 1) < 1e-12
    nsub = 17
    for _ in range(nsub):
        eta, U, V = fs.substep(eta, U, V, zero, zero, g, H, dtau, m)
    amp = np.linalg.matrix_power(Mx, nsub) @ np.array([e0, u0])
    assert np.max(np.abs(eta[0] - (amp[0] * np.exp(1j * k * xc)).real)) < 1e-12 * abs(e0) * 10
    assert np.max(np.abs(U[0] - (amp[1] * np.exp(1j * k * xf)).real)) < 1e-12 * abs(u0) * 10
    assert np.max(np.abs(V)) == 0.0


def test_volume_conservation_latlon():
    m = fs.latlon_metrics(72, 28, -70.0, 140.0, 6.371e6)
    rng = np.random.default_rng(0)
    eta = rng.standard_normal((28, 72))
    U = rng.standard_normal((28, 72)) * 100
    V = rng.standard_normal((29, 72)) * 100
    V[0] = V[-1] = 0
    GU = rng.standard_normal((28, 72)) * 1e-3
    GV = rng.standard_normal((29, 72)) * 1e-3
    vol0 = np.sum(m.area[:, None] * eta)
    w = np.full(45, 1.0 / 45)
    e1, U1, V1, eb, ub, vb = fs.substeps(eta, U, V, GU, GV, 9.81, 3000.0, 600.0, 30, w, m)
    assert abs(np.sum(m.area[:, None] * e1) - vol0) < 1e-12 * np.sum(m.area[:, None] * np.abs(eta))
    assert abs(np.sum(m.area[:, None] * eb) - vol0) < 1e-12 * np.sum(m.area[:, None] * np.abs(eta))
    assert np.all(V1[0] == 0) and np.all(V1[-1] == 0) and np.all(vb[0] == 0)


def test_uniform_forcing_exact():
    """Uniform Gbar in x on a periodic-x domain drives no divergence:
    U^n = U^0 + n dtau Gbar exactly and eta stays put; the average of the
    substeps follows from the weights in closed form."""
    m = fs.latlon_metrics(36, 10, -60.0, 120.0, 6.371e6)
    eta = np.zeros((10, 36))
    U = np.full((10, 36), 3.0)
    V = np.zeros((11, 36))
    GU = np.full((10, 36), 2e-4)
    GV = np.zeros((11, 36))
    dt, N = 600.0, 30
    w = np.linspace(1, 2, 40)
    w /= w.sum()
    e1, U1, V1, eb, ub, vb = fs.substeps(eta, U, V, GU, GV, 9.81, 3000.0, dt, N, w, m)
    dtau = dt / N
    assert np.max(np.abs(U1 - (3.0 + len(w) * dtau * 2e-4))) < 1e-13
    assert np.max(np.abs(e1)) == 0.0
    expect = sum(a * (3.0 + (n + 1) * dtau * 2e-4) for n, a in enumerate(w))
    assert np.max(np.abs(ub - expect)) < 1e-13


def test_correction_matches_barotropic_transport():
    rng = np.random.default_rng(1)
    nz, ny, nx = 7, 5, 6
    dz = np.full(nz, 3000.0 / nz)
    u = rng.standard_normal((nz, ny, nx))
    Ubar = rng.standard_normal((ny, nx)) * 300
    u2 = fs.correct_baroclinic(u, dz, Ubar, 3000.0)
    assert np.max(np.abs(np.tensordot(dz, u2, axes=(0, 0)) - Ubar)) < 1e-10
    # the correction is depth-independent: shear is preserved
    assert np.max(np.abs(np.diff(u2 - u, axis=0))) < 1e-14
