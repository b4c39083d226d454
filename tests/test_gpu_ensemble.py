"""GPU tests of the ensemble path: members stepped together (one fused
tendency launch per substage over all members, batched Poisson passes,
graph replay, autotuned launch shape) give bit-for-bit the states of the
same members stepped one by one with oc_rk3_step, which are themselves held
to the FP64 oracle; one member is also compared with the oracle directly."""
import os

import numpy as np
import pytest

from paper_2502_14148_amd import inputs
from oracle import timestep

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "w", "T", "S")


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _members(sizes, seed=0):
    """Small uneven members: (nx, ny, nz) triples, convection physics."""
    rng = np.random.default_rng(seed)
    out = []
    for k, (nx, ny, nz) in enumerate(sizes):
        ph = inputs.convection_physics((nx, ny, nz), (2.0 * nx, 2.0 * ny, 1.0 * nz),
                                       surface_buoyancy_flux=float(rng.uniform(0.5e-8, 2e-8)))
        out.append((ph, inputs.convection_initial(ph, seed=seed * 100 + k, noise=1e-2)))
    return out


def _models(gpu_lib, members, precision):
    ms = []
    for ph, st in members:
        m = gpu_lib.Model(ph, precision)
        m.set_states(st)
        ms.append(m)
    return ms


def _assert_same(ms_a, ms_b):
    for ia, (a, b) in enumerate(zip(ms_a, ms_b)):
        for f in FIELDS:
            x, y = a.get_state(f), b.get_state(f)
            assert np.array_equal(x, y), (ia, f, np.abs(x - y).max())
        # the last substage's pressure, kept as a spectrum until it is read
        assert np.array_equal(a.get_pressure(), b.get_pressure()), ia


SIZES = [(32, 32, 32), (64, 32, 16), (32, 32, 32), (16, 16, 64), (96, 96, 32)]
# uneven members that every column tile (32 x 8, 16 x 8, 8 x 8) divides
SIZES_WIDE = [(32, 32, 32), (64, 32, 16), (32, 32, 32), (32, 16, 64), (96, 96, 32)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tune,graph", [(False, False), (True, True), (False, True)])
def test_ensemble_equals_members_stepped_alone(gpu_lib, precision, tune, graph):
    mem = _members(SIZES, seed=1)
    ens_models = _models(gpu_lib, mem, precision)
    ref_models = _models(gpu_lib, mem, precision)
    e = gpu_lib.Ensemble(ens_models, tune=tune, graph=graph)
    dt = 2.0
    e.step(dt, 3)
    for m in ref_models:
        m.rk3_step(dt, 3)
    _assert_same(ens_models, ref_models)
    # odd and even step counts alternate the buffer parity; keep going
    e.step(dt, 2)
    for m in ref_models:
        m.rk3_step(dt, 2)
    _assert_same(ens_models, ref_models)


def test_member_stepped_alone_and_dt_change(gpu_lib):
    mem = _members(SIZES[:3], seed=2)
    ens_models = _models(gpu_lib, mem, "fp32")
    ref_models = _models(gpu_lib, mem, "fp32")
    e = gpu_lib.Ensemble(ens_models, graph=True)
    e.step(1.0, 1)
    ens_models[1].rk3_step(1.0, 1)     # one member advances on its own
    e.step(1.5, 2)                      # and dt changes
    for k, m in enumerate(ref_models):
        m.rk3_step(1.0, 1)
        if k == 1:
            m.rk3_step(1.0, 1)
        m.rk3_step(1.5, 2)
    _assert_same(ens_models, ref_models)


def test_ensemble_member_matches_oracle(gpu_lib):
    mem = _members([(32, 32, 32), (16, 16, 32)], seed=3)
    ms = _models(gpu_lib, mem, "fp64")
    e = gpu_lib.Ensemble(ms, tune=True, graph=True)
    e.step(2.0, 2)
    ph, st = mem[0]
    ref = timestep.make_state(st, ph)
    for _ in range(2):
        ref, _ = timestep.rk3_step(ref, 2.0, ph)
    from oracle import fv
    for f in FIELDS:
        got = ms[0].get_state(f)
        want = fv.interior(ref[f], ph, f)
        assert rel_l2(got, want) < 1e-12, (f, rel_l2(got, want))


def test_autotune_cache_roundtrip(gpu_lib, tmp_path):
    path = tmp_path / "tune.jsonl"
    mem = _members(SIZES[:3], seed=4)
    ms = _models(gpu_lib, mem, "fp32")
    e1 = gpu_lib.Ensemble(ms)
    assert e1.tuning()["source"] == "default"
    t1 = e1.autotune(path)
    assert t1["source"] == "timed" and path.exists()
    e2 = gpu_lib.Ensemble(ms)
    t2 = e2.autotune(path)
    assert t2["source"] == "cache"
    for k in ("tile", "persistent", "kc_div"):
        assert t1[k] == t2[k]
    # no cache: timed again, nothing written
    n_lines = len(path.read_text().splitlines())
    assert e2.autotune(None)["source"] == "timed"
    assert len(path.read_text().splitlines()) == n_lines


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("tile,kc_div", [("32x8", 1024), ("16x8", 256), ("8x8", 4096)])
def test_persistent_grid_equals_members_stepped_alone(gpu_lib, precision, tile, kc_div):
    """The persistent work-queue launch (workgroups resident on every CU
    drain an atomic counter, reset inside the captured graph), forced through
    oc_ensemble_set_tuning, gives the members' own oc_rk3_step results bit
    for bit, over several graph replays and across a change of the launch
    configuration."""
    mem = _members(SIZES_WIDE, seed=6)
    ens_models = _models(gpu_lib, mem, precision)
    ref_models = _models(gpu_lib, mem, precision)
    e = gpu_lib.Ensemble(ens_models, graph=True)
    t = e.set_tuning(tile, persistent=True, kc_div=kc_div)
    assert t["persistent"] and t["source"] == "set" and t["tile"] == tile
    assert t["nblocks"] >= 256
    dt = 2.0
    e.step(dt, 3)
    for m in ref_models:
        m.rk3_step(dt, 3)
    _assert_same(ens_models, ref_models)
    # the flat grid of the same tile continues from there
    e.set_tuning(tile, persistent=False, kc_div=kc_div)
    e.step(dt, 2)
    for m in ref_models:
        m.rk3_step(dt, 2)
    _assert_same(ens_models, ref_models)
    # and the persistent grid again, without graphs
    e2 = gpu_lib.Ensemble(ens_models, graph=False)
    e2.set_tuning(tile, persistent=True, kc_div=kc_div)
    e2.step(dt, 1)
    for m in ref_models:
        m.rk3_step(dt, 1)
    _assert_same(ens_models, ref_models)


def test_set_tuning_rejects_bad_values(gpu_lib):
    mem = _members([(32, 32, 32), (16, 16, 16)], seed=7)
    e = gpu_lib.Ensemble(_models(gpu_lib, mem, "fp32"))
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_ARG"):
        e.set_tuning("32x8", kc_div=1024)   # does not divide the 16 x 16 member
    with pytest.raises(gpu_lib.OcError, match="OC_ERR_ARG"):
        e.set_tuning("8x8", kc_div=0)
    assert e.set_tuning("16x8", kc_div=1024)["tile"] == "16x8"


def test_full_size_uneven_ensemble(gpu_lib):
    # 16 x 64^3, 16 x 96^3, 16 x 128^3 free-convection members in FP32, one
    # step under the tuned graph path; one member of each size checked
    # against its own oc_rk3_step, the 64^3 member also against the oracle
    members = inputs.ensemble_physics()
    ms = []
    for ph, seed in members:
        m = gpu_lib.Model(ph, "fp32")
        m.set_states(inputs.convection_initial(ph, seed=seed))
        ms.append(m)
    e = gpu_lib.Ensemble(ms, tune=True, graph=True)
    dt = 1.0
    e.step(dt, 1)
    for idx in (0, 16, 32):
        ph, seed = members[idx]
        r = gpu_lib.Model(ph, "fp32")
        r.set_states(inputs.convection_initial(ph, seed=seed))
        r.rk3_step(dt, 1)
        _assert_same([ms[idx]], [r])
    ph, seed = members[0]
    st = inputs.convection_initial(ph, seed=seed)
    ref, _ = timestep.rk3_step(timestep.make_state(st, ph), dt, ph)
    from oracle import fv
    for f in ("u", "v", "w"):
        got = ms[0].get_state(f)
        assert rel_l2(got, fv.interior(ref[f], ph, f)) < 1e-5, f
    for f in ("T", "S"):
        assert rel_l2(ms[0].get_state(f), fv.interior(ref[f], ph, f)) < 1e-5, f
