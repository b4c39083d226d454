"""Pins of the oracle's pressure solve and projection: brute-force dense
solves of the 7-point operator, single-mode eigenvalues, direct transforms,
divergence after projection, and the projection of gradients."""
import numpy as np
import pytest
import scipy.fft as sfft

from paper_2502_14148_amd.inputs import Physics, random_state
from oracle import pressure, timestep, fv, diagnostics as dg


def _ph(n, bounded, L=(1.3, 0.9, 0.7)):
    return Physics(nx=n, ny=n + (2 if n >= 8 else 0), nz=n, lx=L[0], ly=L[1], lz=L[2],
                   z_bounded=bounded, tracers=("c",))


def dense_laplacian(ph):
    """The 7-point div(grad) operator as a dense matrix, assembled from its
    stencil: periodic x, y; periodic z or no-flux walls (a wall face carries
    no gradient)."""
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    dx, dy, dz = ph.spacing
    N = nx * ny * nz

    def idx(k, j, i):
        return (k * ny + j) * nx + i

    A = np.zeros((N, N))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(k, j, i)
                for (di, h) in ((1, dx), (-1, dx)):
                    A[r, idx(k, j, (i + di) % nx)] += 1 / h ** 2
                    A[r, r] -= 1 / h ** 2
                for (dj, h) in ((1, dy), (-1, dy)):
                    A[r, idx(k, (j + dj) % ny, i)] += 1 / h ** 2
                    A[r, r] -= 1 / h ** 2
                for dk in (1, -1):
                    kk = k + dk
                    if ph.z_bounded and not (0 <= kk < nz):
                        continue
                    A[r, idx(kk % nz, j, i)] += 1 / dz ** 2
                    A[r, r] -= 1 / dz ** 2
    return A


@pytest.mark.parametrize("bounded", [False, True])
def test_dense_8cubed_solve(bounded):
    ph = _ph(8, bounded)
    A = dense_laplacian(ph)
    rng = np.random.default_rng(2)
    rhs = rng.standard_normal((ph.nz, ph.ny, ph.nx))
    rhs -= rhs.mean()                      # compatible right-hand side
    p_dense = np.linalg.lstsq(A, rhs.ravel(), rcond=None)[0]  # min-norm = zero mean
    p_dense = p_dense.reshape(rhs.shape)
    p = pressure.solve_poisson(rhs, ph)
    assert np.max(np.abs(p - p_dense)) < 1e-13 * np.max(np.abs(p_dense)) * 10
    assert abs(p.mean()) < 1e-14 * np.max(np.abs(p))
    # the solution satisfies the operator exactly
    assert np.max(np.abs(A @ p.ravel() - rhs.ravel())) < 1e-12 * np.max(np.abs(rhs)) * 10


@pytest.mark.parametrize("bounded", [False, True])
def test_single_mode_eigenvalue(bounded):
    ph = _ph(12, bounded)
    dx, dy, dz = ph.spacing
    kx, ky, kz = 3, 2, 5
    xc = (np.arange(ph.nx) + 0.5) * dx
    yc = (np.arange(ph.ny) + 0.5) * dy
    zc = (np.arange(ph.nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    if bounded:
        zmode = np.cos(np.pi * kz * Z / ph.lz)
        lz = -(4 / dz ** 2) * np.sin(np.pi * kz / (2 * ph.nz)) ** 2
    else:
        zmode = np.cos(2 * np.pi * kz * Z / ph.lz)
        lz = -(4 / dz ** 2) * np.sin(np.pi * kz / ph.nz) ** 2
    mode = np.cos(2 * np.pi * kx * X / ph.lx) * np.sin(2 * np.pi * ky * Y / ph.ly) * zmode
    lam = (-(4 / dx ** 2) * np.sin(np.pi * kx / ph.nx) ** 2
           - (4 / dy ** 2) * np.sin(np.pi * ky / ph.ny) ** 2 + lz)
    p = pressure.solve_poisson(lam * mode, ph)
    assert np.max(np.abs(p - mode)) < 1e-13


def test_transforms_against_direct_sums():
    """The library DCT-II and FFT used as steps equal their O(N^2) defining
    sums at the odd length 96 = 2^5 * 3."""
    rng = np.random.default_rng(4)
    N = 96
    x = rng.standard_normal(N)
    n = np.arange(N)
    # phases reduced modulo the period with integer arithmetic keep the
    # direct sums accurate to round-off
    direct_dct = np.array([2 * np.sum(x * np.cos(np.pi * ((k * (2 * n + 1)) % (4 * N)) / (2 * N)))
                           for k in range(N)])
    assert np.max(np.abs(sfft.dct(x, type=2) - direct_dct)) < 1e-12
    direct_fft = np.array([np.sum(x * np.exp(-2j * np.pi * ((k * n) % N) / N)) for k in range(N)])
    assert np.max(np.abs(np.fft.fft(x) - direct_fft)) < 1e-12
    assert np.max(np.abs(sfft.idct(sfft.dct(x, type=2), type=2) - x)) < 1e-14


@pytest.mark.parametrize("bounded", [False, True])
def test_projection_leaves_divergence_free(bounded):
    ph = _ph(16, bounded)
    s = random_state(ph, seed=9, divergence_free=False)
    u, v, w, p = pressure.project(s["u"], s["v"], s["w"], 0.37, ph)
    d = pressure.divergence(u, v, w, ph)
    vmax = max(np.max(np.abs(u)), np.max(np.abs(v)), np.max(np.abs(w)))
    assert np.max(np.abs(d)) * min(ph.spacing) / vmax < 1e-13
    if bounded:
        assert np.all(w[0] == 0) and np.all(w[-1] == 0)
    # idempotent: projecting again changes nothing
    u2, v2, w2, _ = pressure.project(u, v, w, 0.37, ph)
    assert max(np.max(np.abs(u2 - u)), np.max(np.abs(w2 - w))) < 1e-13 * vmax


@pytest.mark.parametrize("bounded", [False, True])
def test_projection_removes_gradients(bounded):
    """P(grad phi) = 0 for any centred phi: a discrete gradient is pure pressure."""
    ph = _ph(12, bounded)
    rng = np.random.default_rng(6)
    phi = rng.standard_normal((ph.nz, ph.ny, ph.nx))
    dx, dy, dz = ph.spacing
    u = (phi - np.roll(phi, 1, axis=2)) / dx
    v = (phi - np.roll(phi, 1, axis=1)) / dy
    if bounded:
        w = np.zeros((ph.nz + 1, ph.ny, ph.nx))
        w[1:ph.nz] = (phi[1:] - phi[:-1]) / dz
    else:
        w = (phi - np.roll(phi, 1, axis=0)) / dz
    u2, v2, w2, p = pressure.project(u, v, w, 1.0, ph)
    scale = np.max(np.abs(u))
    for a in (u2, v2, w2):
        assert np.max(np.abs(a)) < 1e-12 * scale
    assert np.max(np.abs((p - p.mean()) - (phi - phi.mean()))) < 1e-12 * np.max(np.abs(phi))


def test_rk3_step_keeps_divergence_below_1e12():
    ph = Physics(nx=16, ny=16, nz=8, lx=32.0, ly=32.0, lz=8.0, z_bounded=True, z0=-8.0,
                 f=1e-4, alpha=2e-4, beta=8e-4, t_ref=20.0, s_ref=35.0, nu=1e-5,
                 kappa=1e-5, tracers=("T", "S"), buoyancy=True, top_flux={"T": 5e-6})
    s = random_state(ph, seed=3, vel=1e-3, tracer_scale=0.01)
    s["T"] = s["T"] + 20.0
    s["S"] = s["S"] + 25.0
    state = timestep.make_state(s, ph)
    st2, _ = timestep.rk3_step(state, 1.0, ph)
    assert dg.scaled_divergence(st2, ph) < 1e-12
