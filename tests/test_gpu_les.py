"""GPU parity of the eddy-viscosity LES closures (Smagorinsky-Lilly with the
Lilly stratification factor; anisotropic minimum dissipation with per-tracer
diffusivities) through the C ABI against the FP64 oracle: full tendencies
(constant closure + advection + LES), and RK3 steps.  Bars as for the other
tendencies: relative L2 1e-12 in FP64, 1e-4 in FP32 (1e-5 for states)."""
import numpy as np
import pytest

from paper_2502_14148_amd import inputs
from oracle import fv, tendencies as td, timestep

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(les, n=(32, 32, 16), stretched=False):
    ph = inputs.convection_physics(n, (2.0 * n[0], 2.0 * n[1], 1.0 * n[2]), nu=1e-4, kappa=1e-4)
    if stretched:
        ph.z_faces = inputs.stretched_faces(n[2], ph.lz, ph.z0, 1.5)
    ph.les = les
    s = inputs.random_state(ph, seed=11, vel=5e-2)
    s["T"] = 20.0 + 0.01 * np.broadcast_to(inputs.cell_centres_z(ph)[:, None, None], s["T"].shape) \
        + 0.05 * s["T"]
    s["S"] += 35.0
    return ph, s


def _prep(state, precision):
    if precision == "fp32":
        return {k: v.astype(np.float32).astype(np.float64) for k, v in state.items()}
    return state


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("les,stretched", [("smagorinsky", False), ("amd", False),
                                           ("smagorinsky", True), ("amd", True)])
def test_les_tendency_parity(gpu_lib, les, stretched, precision):
    ph, s = _case(les, stretched=stretched)
    s = _prep(s, precision)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.tendencies()
    G = td.tendencies(timestep.make_state(s, ph), ph)
    for name in m.fields:
        err = rel_l2(m.get_tendency(name), G[name])
        assert err <= TOL[precision] * (10 if precision == "fp32" else 1), (les, name, err)


def test_les_changes_the_tendency(gpu_lib):
    """The closure is not a no-op: the LES share of G_u is a sizable part."""
    ph, s = _case("smagorinsky")
    m = gpu_lib.Model(ph, "fp64")
    m.set_states(s)
    m.tendencies()
    g1 = m.get_tendency("u")
    ph.les = "none"
    m0 = gpu_lib.Model(ph, "fp64")
    m0.set_states(s)
    m0.tendencies()
    assert rel_l2(g1, m0.get_tendency("u")) > 1e-3


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("les", ["smagorinsky", "amd"])
def test_les_rk3_parity(gpu_lib, les, precision):
    ph, s = _case(les, n=(32, 16, 16), stretched=True)
    s = _prep(s, precision)
    m = gpu_lib.Model(ph, precision)
    m.set_states(s)
    m.rk3_step(0.5, 2)
    st = timestep.make_state(s, ph)
    for _ in range(2):
        st, _ = timestep.rk3_step(st, 0.5, ph)
    for name in m.fields:
        err = rel_l2(m.get_state(name), fv.interior(st[name], ph, name))
        assert err <= TOL[precision], (les, name, err)


def test_les_restrictions(gpu_lib):
    ph, s = _case("amd")
    m = gpu_lib.Model(ph, "fp32")
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_UNSUPPORTED"):
        gpu_lib.Ensemble([m])
