"""GPU diagnostics (oc_diagnostics, oc_sync_check) against the oracle's
FP64 global diagnostics, and the NaN guard forced from the host: a state set
with one NaN must be reported as OC_ERR_NONFINITE."""
import numpy as np
import pytest

from paper_2502_14148_amd import inputs
from oracle import diagnostics as dg, timestep

pytestmark = pytest.mark.gpu


def _case(stretched):
    if stretched:
        ph = inputs.stretched_convection_physics((32, 32, 24), (64.0, 64.0, 24.0))
    else:
        ph = inputs.convection_physics((32, 32, 16), (64.0, 64.0, 16.0))
    s = inputs.random_state(ph, seed=12, vel=0.05, tracer_means=(ph.t_ref, ph.s_ref))
    return ph, s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("stretched", [False, True])
def test_diagnostics_match_oracle(gpu_lib, precision, stretched):
    ph, s = _case(stretched)
    if precision == "fp32":
        s = {k: v.astype(np.float32).astype(np.float64) for k, v in s.items()}
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.rk3_step(1.0, 1)   # a projected state (the divergence measure is then small)
    got = m.diagnostics()
    st = timestep.make_state({n: m.get_state(n) for n in m.fields}, ph)
    for key, name in (("max_u", "u"), ("max_v", "v"), ("max_w", "w")):
        want = float(np.max(np.abs(m.get_state(name))))
        assert got[key] == want, key
    mom = dg.momentum_integrals(st, ph)
    dx, dy, _ = ph.spacing
    for q, name in enumerate(("u", "v", "w")):
        scale = np.sum(np.abs(m.get_state(name))) * dx * dy * ph.lz / ph.nz
        assert abs(got["momentum"][q] - mom[q]) <= 1e-13 * scale, name
    for q, name in enumerate(ph.tracers):
        want = dg.volume_integral(m.get_state(name), ph)
        assert abs(got["tracer_integrals"][q] - want) <= 1e-13 * abs(want), name
    assert got["cfl_rate"] == pytest.approx(dg.cfl_rate(st, ph), rel=1e-15)
    vmax = max(got["max_u"], got["max_v"], got["max_w"])
    scaled = dg.scaled_divergence(st, ph)
    # the GPU reports max|div| * min spacing; the oracle divides by max|u| too.
    # After the projection both are the roundoff of the difference formula,
    # so they agree to that roundoff, not relatively
    assert abs(got["div_scaled_by_dx"] / vmax - scaled) <= 1e-14
    assert scaled < (1e-12 if precision == "fp64" else 1e-5)
    assert got["div_scaled_by_dx"] / vmax < (1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nan_guard_from_host(gpu_lib, precision):
    ph, s = _case(False)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.diagnostics()
    m.sync_check()
    bad = s["T"].copy()
    bad[3, 5, 7] = np.nan
    m.set_state("T", bad)
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_NONFINITE"):
        m.diagnostics()
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_NONFINITE"):
        m.sync_check()
    bad = s["u"].copy()
    bad[0, 0, 0] = np.inf
    m.set_state("T", s["T"])
    m.set_state("u", bad)
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_NONFINITE"):
        m.sync_check()
    m.set_state("u", s["u"])
    m.sync_check()
    m.diagnostics()


def test_diagnostics_reject_hydrostatic(gpu_lib):
    ph = inputs.sector_physics((32, 16, 8))
    m = gpu_lib.Model(ph, "fp32")
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_UNSUPPORTED"):
        m.diagnostics()
    m.sync_check()
