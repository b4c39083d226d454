"""Pins of the oracle's learned-closure pieces: BF16 rounding on exactly
representable cases, gradients against central finite differences, the
Adam first step in closed form, integral preservation of coarse-graining,
and conservation of the closure tendency."""
import numpy as np
import pytest

from paper_2502_14148_amd.inputs import Physics, random_state
from oracle import closure as cl
from oracle import pressure


def test_bf16_round_to_nearest_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3e38, 1e-40])
    got = cl.bf16(x)
    want = [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, None, None]
    for g, w in zip(got[:5], want[:5]):
        assert g == w
    # every result is representable in 8 bits of mantissa
    m, e = np.frexp(got[:5])
    assert np.all(np.abs(m * 2 ** 8 - np.round(m * 2 ** 8)) == 0)


def test_zero_weights_give_bias():
    p = cl.init_params(1)
    for k in ("W1", "W2", "W3"):
        p[k] = np.zeros_like(p[k])
    p["b3"] = np.array([0.5, -1.0, 2.0, 0.25])
    X = np.random.default_rng(0).standard_normal((7, cl.NIN))
    Y, _ = cl.forward(p, X)
    assert np.array_equal(Y, np.broadcast_to(p["b3"], Y.shape))


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = cl.init_params(2)
    p["b1"] = rng.standard_normal(cl.NH) * 0.1
    p["b2"] = rng.standard_normal(cl.NH) * 0.1
    X = rng.standard_normal((5, cl.NIN))
    T = rng.standard_normal((5, cl.NOUT))
    Y, cache = cl.forward(p, X, use_bf16=False)
    g = cl.backward(p, cache, Y, T, use_bf16=False)
    h = 1e-6
    for name, idx in (("W1", (3, 17)), ("W1", (200, 499)), ("b1", (9,)), ("W2", (100, 5)),
                      ("b2", (255,)), ("W3", (2, 77)), ("b3", (1,))):
        q = {k: v.copy() for k, v in p.items()}
        q[name][idx] += h
        lp = cl.mse(cl.forward(q, X, use_bf16=False)[0], T)
        q[name][idx] -= 2 * h
        lm = cl.mse(cl.forward(q, X, use_bf16=False)[0], T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[name][idx]) <= 1e-6 * max(abs(fd), 1e-6) + 1e-10, (name, idx, fd, g[name][idx])


def test_adam_first_step_closed_form():
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -1e-3, 0.0])}
    out = cl.adam_step(p, g, {}, lr=1e-2)
    # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(out["a"], p["a"] - 1e-2 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=0, atol=1e-15)


def _phys(n=16, bounded=True):
    return Physics(nx=n, ny=n, nz=n, lx=2.0 * n, ly=2.0 * n, lz=1.0 * n, z_bounded=bounded,
                   tracers=("T", "S"), g=9.81, alpha=2e-4, beta=8e-4)


def test_coarse_grain_preserves_integrals_and_divergence():
    ph = _phys(16)
    s = random_state(ph, seed=4)
    U, V, W, C = cl.coarse_grain(s["u"], s["v"], s["w"], s["T"], 4)
    assert abs(C.sum() * 64 - s["T"].sum()) < 1e-12 * np.abs(s["T"]).sum()
    phc = _phys(4)
    phc.lx, phc.ly, phc.lz = ph.lx, ph.ly, ph.lz
    d_fine = pressure.divergence(s["u"], s["v"], s["w"], ph)
    d_coarse = pressure.divergence(U, V, W, phc)
    assert np.max(np.abs(d_fine)) < 1e-12 * np.max(np.abs(s["u"]))
    assert np.max(np.abs(d_coarse)) < 1e-12 * np.max(np.abs(s["u"]))
    # coarse faces of w on the walls stay closed
    assert np.all(W[0] == 0) and np.all(W[-1] == 0)


def test_subgrid_flux_vanishes_for_box_constant_fields():
    ph = _phys(8)
    rng = np.random.default_rng(5)
    b = np.kron(rng.standard_normal((2, 2, 2)), np.ones((4, 4, 4)))
    s = random_state(ph, seed=6)
    F = cl.subgrid_fluxes(s["u"], s["v"], s["w"], b, 4)
    assert np.max(np.abs(F[3])) < 1e-14 * np.max(np.abs(b))
    assert np.all(F[2] >= -1e-15)     # <w w> - <w><w> is a variance


def test_closure_tendency_conserves_columns():
    ph = _phys(8)
    rng = np.random.default_rng(7)
    F = rng.standard_normal((4, ph.nz, ph.ny, ph.nx))
    G = cl.closure_tendency(F, ph)
    for k in ("u", "v", "T"):
        assert np.max(np.abs(G[k].sum(axis=0))) < 1e-10
    assert np.all(G["w"][0] == 0) and np.all(G["w"][-1] == 0)


def _box_cov(a, b, r):
    """Brute-force <a b> - <a><b> over each r^3 box with plain loops."""
    nz, ny, nx = a.shape
    out = np.zeros((nz // r, ny // r, nx // r))
    for K in range(nz // r):
        for J in range(ny // r):
            for I in range(nx // r):
                sa = sb = sab = 0.0
                for k in range(K * r, K * r + r):
                    for j in range(J * r, J * r + r):
                        for i in range(I * r, I * r + r):
                            sa += a[k, j, i]
                            sb += b[k, j, i]
                            sab += a[k, j, i] * b[k, j, i]
                n = r ** 3
                out[K, J, I] = sab / n - (sa / n) * (sb / n)
    return out


def test_subgrid_fluxes_centre_values_closed_form():
    """Face i lies on the left of cell i, so the centre value of a face field
    f(i) = i^2 is the mean of faces i and i + 1: i^2 + i + 1/2 (a mean with
    the left neighbour, i^2 - i + 1/2, changes every covariance below by
    2 Var(i)).  Same along y for v and along z for w (faces k and k + 1 of a
    walled column).  Coarse boxes away from the periodic seam are compared
    with the fluxes of those closed-form centre values."""
    n, r = 8, 4
    idx = np.arange(n, dtype=np.float64)
    one = np.ones((n, n, n))
    ii = one * idx[None, None, :]
    jj = one * idx[None, :, None]
    kk = one * idx[:, None, None]
    u = ii ** 2                                   # x faces
    v = jj ** 2                                   # y faces
    kf = np.arange(n + 1, dtype=np.float64)
    w = (np.ones((n + 1, n, n)) * kf[:, None, None]) ** 2 + ii[:1]   # z faces, varies in x too
    b = kk + 2.0 * jj - ii
    F = cl.subgrid_fluxes(u, v, w, b, r)
    uc = ii ** 2 + ii + 0.5
    vc = jj ** 2 + jj + 0.5
    wc = kk ** 2 + kk + 0.5 + ii
    want = [_box_cov(q, wc, r) for q in (uc, vc, wc, b)]
    # boxes whose x and y ranges do not reach the last (seam) column/row
    sel = (slice(None), slice(0, n // r - 1), slice(0, n // r - 1))
    for q in range(4):
        assert np.max(np.abs(F[q][sel] - want[q][sel])) < 1e-9, q
    # the left-neighbour mean would differ by 2 Var(i) = (r^2 - 1) / 6 in tau_uw
    # wherever wc varies with i inside the box as i itself does
    assert abs(_box_cov(ii ** 2 - ii + 0.5, wc, r)[0, 0, 0] - want[0][0, 0, 0]) > 0.1


def test_closure_tendency_of_a_single_flux_impulse():
    """One nonzero flux value d at centre (k0, j0, i0): tau_uw reaches the two
    x faces of that cell (i0, i0 + 1) at a quarter of d on the z faces k0 and
    k0 + 1 (half from the x average, half from the z average), so G_u is
    -d / (4 dz) at level k0 - 1, 0 at k0 and +d / (4 dz) at k0 + 1 on those
    two faces and zero elsewhere; v likewise on y faces j0, j0 + 1; J_bw
    reaches only the cell's own column (the z average alone), giving
    -+d / (2 dz g alpha) at k0 -+ 1; tau_ww differences to the w faces k0
    (-d / dz) and k0 + 1 (+d / dz)."""
    ph = _phys(8)
    dz = ph.spacing[2]
    k0, j0, i0, d = 3, 2, 5, 1.75
    for comp in range(4):
        F = np.zeros((4, ph.nz, ph.ny, ph.nx))
        F[comp, k0, j0, i0] = d
        G = cl.closure_tendency(F, ph)
        if comp in (0, 1):
            name = "u" if comp == 0 else "v"
            want = np.zeros((ph.nz, ph.ny, ph.nx))
            for e in (0, 1):
                jj, ii = (j0, i0 + e) if comp == 0 else (j0 + e, i0)
                want[k0 - 1, jj, ii] = -d / (4 * dz)
                want[k0 + 1, jj, ii] = d / (4 * dz)
        elif comp == 3:
            name = "T"
            c = d / (ph.g * ph.alpha)
            want = np.zeros((ph.nz, ph.ny, ph.nx))
            want[k0 - 1, j0, i0] = -c / (2 * dz)
            want[k0 + 1, j0, i0] = c / (2 * dz)
        else:
            name = "w"
            want = np.zeros((ph.nz + 1, ph.ny, ph.nx))
            want[k0, j0, i0] = -d / dz
            want[k0 + 1, j0, i0] = d / dz
        assert np.max(np.abs(G[name] - want)) < 1e-15, (comp, name)
        for other in ("u", "v", "w", "T"):
            if other != name:
                assert not np.any(G[other]), (comp, other)
