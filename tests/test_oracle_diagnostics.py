"""Pins of the oracle's global diagnostics (momentum integrals and the CFL
rate) against closed forms and invariants: uniform fields give value times
domain volume, a uniform flow on an f-plane turns by the RK3 stability
polynomial of -i f dt, and flux-form advection on a periodic box keeps the
integrals."""
import numpy as np
import pytest

from oracle import diagnostics as dg, fv, timestep
from paper_2502_14148_amd.inputs import Physics, random_state, stretched_faces


def _phys(n, bounded, stretched=False, **kw):
    zf = stretched_faces(n, 1.0, -1.0, 1.5) if stretched else None
    base = dict(nx=n, ny=n, nz=n, lx=2.0, ly=3.0, lz=1.0, z0=-1.0, z_bounded=bounded,
                advection="weno5z", nu=1e-3, kappa=1e-3, f=0.0, buoyancy=False,
                tracers=("T", "S"), z_faces=zf)
    base.update(kw)
    return Physics(**base)


@pytest.mark.parametrize("bounded,stretched", [(False, False), (True, False), (True, True)])
def test_uniform_fields_integrate_to_value_times_volume(bounded, stretched):
    ph = _phys(8, bounded, stretched)
    n = (ph.nz, ph.ny, ph.nx)
    nwf = fv.w_faces(ph)
    w = np.full((nwf, ph.ny, ph.nx), -0.7)
    if bounded:
        w[0] = w[-1] = 0.0
    st = timestep.make_state({"u": np.full(n, 1.25), "v": np.full(n, 0.5), "w": w,
                              "T": np.zeros(n), "S": np.zeros(n)}, ph)
    mu, mv, mw = dg.momentum_integrals(st, ph)
    vol = ph.lx * ph.ly * ph.lz
    assert abs(mu - 1.25 * vol) < 1e-14 * vol
    assert abs(mv - 0.5 * vol) < 1e-14 * vol
    if bounded:
        # interior faces only: the centres of the bottom and top cells bound them
        dzc, _ = fv.z_spacings(ph)
        span = ph.lz - 0.5 * dzc[0] - 0.5 * dzc[-1]
        assert abs(mw - (-0.7) * ph.lx * ph.ly * span) < 1e-14 * vol
    else:
        assert abs(mw - (-0.7) * vol) < 1e-14 * vol


def test_momentum_of_uniform_flow_turns_by_rk3_factor():
    f, dt = 0.11, 0.3
    ph = _phys(8, True, f=f)
    n = (ph.nz, ph.ny, ph.nx)
    s = {"u": np.full(n, 0.4), "v": np.full(n, -0.25), "w": np.zeros((ph.nz + 1, ph.ny, ph.nx)),
         "T": np.ones(n), "S": np.ones(n)}
    st = timestep.make_state(s, ph)
    st2, _ = timestep.rk3_step(st, dt, ph)
    vol = ph.lx * ph.ly * ph.lz
    z = -1j * f * dt
    amp = 1 + z + z ** 2 / 2 + z ** 3 / 6
    mu, mv, _ = dg.momentum_integrals(st2, ph)
    want = (0.4 - 0.25j) * amp * vol
    assert abs(mu - want.real) < 1e-13 * vol and abs(mv - want.imag) < 1e-13 * vol


def test_momentum_kept_by_periodic_advection():
    ph = _phys(16, False)
    st = timestep.make_state(random_state(ph, seed=3), ph)
    st2, _ = timestep.rk3_step(st, 0.01, ph)
    a, b = dg.momentum_integrals(st, ph), dg.momentum_integrals(st2, ph)
    dx, dy, dz = ph.spacing
    for q, name in enumerate(("u", "v", "w")):
        scale = np.sum(np.abs(fv.interior(st[name], ph, name))) * dx * dy * dz
        assert abs(a[q] - b[q]) <= 1e-12 * scale, name


def test_cfl_rate_closed_form():
    ph = _phys(8, True, stretched=True)
    n = (ph.nz, ph.ny, ph.nx)
    u, v = np.zeros(n), np.zeros(n)
    w = np.zeros((ph.nz + 1, ph.ny, ph.nx))
    u[2, 3, 4] = -0.9
    v[5, 1, 0] = 0.3
    w[4, 2, 2] = 0.02
    st = timestep.make_state({"u": u, "v": v, "w": w, "T": np.zeros(n), "S": np.zeros(n)}, ph)
    dzc, _ = fv.z_spacings(ph)
    want = max(0.9 / (ph.lx / 8), 0.3 / (ph.ly / 8), 0.02 / dzc.min())
    assert dg.cfl_rate(st, ph) == pytest.approx(want, rel=1e-15)
    assert dg.cfl(st, 0.5, ph) == pytest.approx(0.5 * want, rel=1e-15)
