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
