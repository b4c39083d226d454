"""GPU parity with WENO reconstructions of orders 7 and 9 (stencil radius 4
and 5, halo 4 and 5 cells; centred advecting velocity of order 6 and 8):
tendencies, RK3 steps and a ten-step convection run through the C ABI
against the FP64 oracle on the same seeded inputs, the closure-carrying
kernel instantiation (with an LES closure), and 256^3 windows in the
launch configuration of the WENO9 benchmark.  Bars as for WENO5: relative
L2 1e-12 in FP64 and 1e-5 in FP32-mixed (tendencies 1e-4 in FP32; the FP32
run starts from the inputs rounded to FP32)."""
import dataclasses

import numpy as np
import pytest

from paper_2502_14148_amd import inputs
from oracle import fv, tendencies as td, timestep

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
SCHEMES = ["weno7z", "weno7_linear", "weno9z", "weno9_linear"]


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _prep(state, precision):
    if precision == "fp32":
        return {k: v.astype(np.float32).astype(np.float64) for k, v in state.items()}
    return state


def _conv(n, scheme, **kw):
    ph = inputs.convection_physics(n, (2.0 * n[0], 2.0 * n[1], 1.0 * n[2]), **kw)
    return dataclasses.replace(ph, advection=scheme)


def _box(n, scheme):
    return dataclasses.replace(inputs.periodic_box_physics(n), advection=scheme)


# (physics, state): wide 32 x 8 tiles, 8 x 8 tiles (16 wide), several k
# chunks with a ragged last one, periodic z, the smallest grid (8: images at
# both ends of an axis shorter than twice the halo)
CASES = {
    "conv_32x32x16": lambda s: (_conv((32, 32, 16), s),
                                lambda ph: inputs.random_state(ph, seed=3, vel=1e-2)),
    "conv_16x16x32": lambda s: (_conv((16, 16, 32), s),
                                lambda ph: inputs.random_state(ph, seed=8, vel=1e-2)),
    "conv_64x32x96": lambda s: (_conv((64, 32, 96), s, nu=1e-3, kappa=2e-3),
                                lambda ph: inputs.smooth_random_state(ph, seed=5)),
    "box16": lambda s: (_box(16, s), lambda ph: inputs.random_state(ph, seed=1)),
    "box8": lambda s: (_box(8, s), lambda ph: inputs.random_state(ph, seed=6)),
}


def make_case(name, scheme):
    ph, gen = CASES[name](scheme)
    s = gen(ph)
    if ph.z_bounded and "T" in s:
        s["T"] = s["T"] + 20.0
        s["S"] = s["S"] + 25.0
    return ph, s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("scheme", SCHEMES)
def test_tendency_parity(gpu_lib, scheme, case, precision):
    ph, s = make_case(case, scheme)
    s = _prep(s, precision)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.tendencies()
    G = td.tendencies(timestep.make_state(s, ph), ph)
    for name in m.fields:
        err = rel_l2(m.get_tendency(name), G[name])
        assert err <= TOL[precision] * (10 if precision == "fp32" else 1), (case, name, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case,dt,nsteps", [("conv_32x32x16", 1.0, 2), ("box16", 0.01, 1),
                                            ("conv_16x16x32", 1.0, 1)])
@pytest.mark.parametrize("scheme", ["weno7z", "weno9z"])
def test_rk3_step_parity(gpu_lib, scheme, case, dt, nsteps, precision):
    ph, s = make_case(case, scheme)
    s = _prep(s, precision)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.rk3_step(dt, nsteps)
    st = timestep.make_state(s, ph)
    for _ in range(nsteps):
        st, _ = timestep.rk3_step(st, dt, ph)
    for name in m.fields:
        err = rel_l2(m.get_state(name), fv.interior(st[name], ph, name))
        assert err <= TOL[precision], (case, name, err)


def test_convection_ten_steps_weno9(gpu_lib):
    """Free convection with WENO9 and no explicit closure beyond molecular
    values (implicit LES), 64 x 64 x 32 at 2 m x 2 m x 1 m, 10 steps of 1 s,
    FP64 and FP32-mixed against one oracle run, from the initial state of
    the WENO5 ten-step test."""
    ph = _conv((64, 64, 32), "weno9z")
    s = inputs.convection_initial(ph, seed=7)
    st = timestep.run(timestep.make_state(s, ph), 1.0, 10, ph)
    ref = {n: fv.interior(st[n], ph, n) for n in ("u", "v", "w", "T", "S")}
    for precision in ("fp64", "fp32"):
        m = gpu_lib.Model(ph, precision)
        m.set_states(_prep(s, precision))
        m.rk3_step(1.0, 10)
        for name in m.fields:
            err = rel_l2(m.get_state(name), ref[name])
            assert err <= TOL[precision], (precision, name, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_weno7_with_les_closure(gpu_lib, precision):
    """The kernel instantiation that adds closure tendencies, with WENO7 and
    the Smagorinsky-Lilly closure."""
    ph = dataclasses.replace(_conv((32, 32, 16), "weno7z"), les="smagorinsky")
    s = _prep(make_case("conv_32x32x16", "weno7z")[1], precision)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.tendencies()
    G = td.tendencies(timestep.make_state(s, ph), ph)
    for name in m.fields:
        err = rel_l2(m.get_tendency(name), G[name])
        assert err <= TOL[precision] * (10 if precision == "fp32" else 1), (name, err)


def test_weno_restrictions(gpu_lib):
    """Orders 7 and 9 are nonhydrostatic-only and ensembles take WENO5-Z."""
    m = gpu_lib.Model(_conv((32, 32, 16), "weno9z"), "fp32")
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_UNSUPPORTED"):
        gpu_lib.Ensemble([m])


N, B = 256, 24


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_weno9_windows(gpu_lib, precision):
    """The 256^3 free-convection LES with WENO9 (the benchmark's WENO9
    configuration): tendencies on 24 x 24 full-depth column windows, exact
    but in a margin of R + 1 = 6 cells, against the oracle on the window."""
    ph = _conv((N, N, N), "weno9z")
    s = inputs.convection_initial(ph, seed=0, tracer_noise=0.1)
    s = _prep(s, precision)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.tendencies()
    tol = 1e-12 if precision == "fp64" else 1e-4
    inner = slice(6, B - 6)
    dx, dy, _ = ph.spacing
    sub = dataclasses.replace(ph, nx=B, ny=B, lx=B * dx, ly=B * dy)
    G = {name: m.get_tendency(name) for name in ("u", "v", "w", "T", "S")}
    for i0, j0 in ((0, 0), (100, 37), (N - B, N - B)):
        st = {k: s[k][:, j0:j0 + B, i0:i0 + B] for k in ("u", "v", "w", "T", "S")}
        ref = td.tendencies(timestep.make_state(st, sub), sub)
        for name in G:
            got = G[name][:, j0:j0 + B, i0:i0 + B][:, inner, inner]
            err = rel_l2(got, ref[name][:, inner, inner])
            assert err <= tol, (precision, name, i0, j0, err)
