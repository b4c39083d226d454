"""Pins of the oracle's tendencies with WENO orders 7 and 9: the flux-form
tracer advection converges at the scheme's order, momentum self-advection
at the order of the centred advecting-velocity interpolation (one below:
a wrong interpolation order or a misplaced stencil offset shows as a lower
rate), conservation of tracer content and momentum, free-stream
preservation and the second-order convergence of every term together."""
import numpy as np
import pytest

from paper_2502_14148_amd.inputs import Physics, random_state
from oracle import fv, tendencies as td, timestep
from tests.test_oracle_tendencies import _phys, _tendency_errors

SCHEMES = {"weno5_linear": ([16, 32, 64], 5, 4), "weno7_linear": ([16, 32, 64], 7, 6),
           "weno7z": ([16, 32, 64], 7, 6), "weno9_linear": ([16, 24, 32], 9, 8),
           "weno9z": ([16, 24, 32], 9, 8)}


def _fit(errs, ns):
    return -np.polyfit(np.log(np.array(ns, float)), np.log(np.array(errs)), 1)[0]


def _tracer_error(n, scheme):
    """Constant velocity 0.8 along x; the tracer holds the exact cell averages
    of sin(x); the exact averaged tendency is -0.8 (sin(x_{i+1/2}) -
    sin(x_{i-1/2})) / h."""
    L = 2 * np.pi
    ph = Physics(nx=n, ny=4, nz=4, lx=L, ly=1.0, lz=1.0, z_bounded=False, tracers=("c",),
                 advection=scheme)
    h = L / n
    xf = np.arange(n) * h
    avg = (-np.cos(xf + h) + np.cos(xf)) / h
    c = np.broadcast_to(avg, (4, 4, n)).copy()
    zero = np.zeros((4, 4, n))
    st = timestep.make_state({"u": np.full((4, 4, n), 0.8), "v": zero, "w": zero, "c": c}, ph)
    G = td.tracer_tendency(st["c"], st, ph)
    return np.max(np.abs(G[0, 0] - (-0.8 * (np.sin(xf + h) - np.sin(xf)) / h)))


def _self_advection_error(n, scheme, axis):
    """u (axis x) or w (axis z) holds the exact averages of 0.7 + sin over
    its staggered cells; the exact averaged tendency of Burgers' flux form is
    -((q^2)(right) - (q^2)(left)) / h at that cell's faces."""
    L = 2 * np.pi
    ph = Physics(nx=n if axis == "x" else 4, ny=4, nz=n if axis == "z" else 4,
                 lx=L if axis == "x" else 1.0, ly=1.0, lz=L if axis == "z" else 1.0,
                 z_bounded=False, tracers=("c",), advection=scheme, nu=0.0, kappa=0.0, f=0.0,
                 buoyancy=False)
    h = L / n
    xs = np.arange(n) * h
    avg = 0.7 + (np.cos(xs - h / 2) - np.cos(xs + h / 2)) / h
    exact = -((0.7 + np.sin(xs + h / 2)) ** 2 - (0.7 + np.sin(xs - h / 2)) ** 2) / h
    if axis == "x":
        zero = np.zeros((4, 4, n))
        st = timestep.make_state({"u": np.broadcast_to(avg, (4, 4, n)).copy(), "v": zero,
                                  "w": zero, "c": zero}, ph)
        return np.max(np.abs(td.u_tendency(st, ph)[0, 0] - exact))
    zero = np.zeros((n, 4, 4))
    st = timestep.make_state({"u": zero, "v": zero, "c": zero,
                              "w": np.broadcast_to(avg[:, None, None], (n, 4, 4)).copy()}, ph)
    return np.max(np.abs(td.w_tendency(st, ph)[:, 0, 0] - exact))


@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_tracer_advection_order(scheme):
    ns, order, _ = SCHEMES[scheme]
    errs = [_tracer_error(n, scheme) for n in ns]
    assert _fit(errs, ns) >= order - 0.2, errs


@pytest.mark.parametrize("axis", ["x", "z"])
@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_momentum_self_advection_order(scheme, axis):
    ns, _, order = SCHEMES[scheme]
    errs = [_self_advection_error(n, scheme, axis) for n in ns]
    assert abs(_fit(errs, ns) - order) < 0.2, errs


@pytest.mark.parametrize("scheme", ["weno7z", "weno9z"])
@pytest.mark.parametrize("bounded", [False, True])
def test_conservation_over_rk3_step(scheme, bounded):
    kw = dict(advection=scheme, nu=0.01, kappa=0.02, f=0.0)
    if bounded:
        kw.update(buoyancy=False)
    ph = _phys(16, bounded, **kw)
    state = timestep.make_state(random_state(ph, seed=17), ph)
    st2, _ = timestep.rk3_step(state, 0.01, ph)
    names = list(ph.tracers) + (["u", "v"] if bounded else ["u", "v", "w"])
    for name in names:
        a = np.sum(fv.interior(state[name], ph, name))
        b = np.sum(fv.interior(st2[name], ph, name))
        scale = np.sum(np.abs(fv.interior(state[name], ph, name)))
        assert abs(a - b) <= 1e-12 * scale, name


@pytest.mark.parametrize("scheme", ["weno7z", "weno9z"])
def test_free_stream_preservation(scheme):
    ph = _phys(16, True, advection=scheme, nu=0.0, kappa=0.0)
    s = random_state(ph, seed=5)
    s["T"] = np.full_like(s["T"], 7.25)
    state = timestep.make_state(s, ph)
    G = td.tracer_tendency(state["T"], state, ph)
    assert np.max(np.abs(G)) < 1e-12 * 7.25 * np.max(np.abs(s["u"])) / min(ph.spacing)


@pytest.mark.parametrize("bounded", [False, True])
def test_all_terms_converge_weno9_linear(bounded):
    """Coriolis, buoyancy, diffusion and the walls together with WENO9: the
    tendencies converge to the continuous ones at second order."""
    ns = [16, 32, 64]
    errs = [_tendency_errors(n, bounded, "weno9_linear") for n in ns]
    for name in errs[0]:
        e = [er[name] for er in errs]
        assert np.log2(e[1] / e[2]) > 1.9, (name, e)
        assert e[2] < 0.01, (name, e)
