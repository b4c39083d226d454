"""Error bars of the FP32-mixed path that follow from its arithmetic.

The FP32 state is rounded to FP32 every time a substage stores it (stored
value = x - offset, the offset being the equation of state's reference for
T and S, 0 otherwise).  One rounding errs by at most half a unit in the last
place of the stored value, with an RMS of ulp / sqrt(12) for values that
fill their binade; 3 n stores in n RK3 steps add up like a random walk.  A
field whose change over the run is small against its stored magnitude
therefore cannot match the FP64 oracle's change to better than

    rel_anom ~ sqrt(3 n) * ||ulp(x - offset)||_2 / sqrt(12) / ||x - x0||_2.

The same holds for FP64 storage with its own ulp and a 1e-12 base.
anomaly_tolerance returns 1e-5 plus three times that floor: where the run
changes the fields by more than about one percent the bar is 1e-5 in effect;
where it barely changes them the bar says what FP32 storage alone allows, and
a field that was never updated (relative anomaly error 1) still fails as long
as the bar stays below 0.1, which the callers assert.
"""
import numpy as np


def storage_offset(ph, name, precision):
    if precision != "fp32" or not getattr(ph, "buoyancy", False):
        return 0.0
    return {"T": ph.t_ref, "S": ph.s_ref}.get(name, 0.0)


def anomaly_tolerance(ref, x0, nsteps, offset=0.0, stores_per_step=3, base=1e-5,
                      dtype=np.float32):
    ulp = np.spacing(np.abs(np.asarray(ref - offset, dtype=dtype))).astype(np.float64)
    change = np.linalg.norm(ref - x0)
    if change == 0.0:
        return np.inf
    floor = np.sqrt(stores_per_step * nsteps) * np.linalg.norm(ulp) / np.sqrt(12.0) / change
    return base + 3.0 * floor


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def check_anomaly(got, ref, x0, nsteps, ph, name, precision, label=""):
    """Relative L2 of the change over the run, x - x0, against the oracle's;
    returns (error, bar)."""
    if precision == "fp32":
        tol = anomaly_tolerance(ref, x0, nsteps, storage_offset(ph, name, precision))
    else:
        tol = anomaly_tolerance(ref, x0, nsteps, base=1e-12, dtype=np.float64)
    assert tol < 0.1, (label, name, "the run changes the field too little to test", tol)
    err = rel_l2(got - x0, ref - x0)
    assert err <= tol, (label, name, err, tol)
    return err, tol
