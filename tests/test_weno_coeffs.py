"""The constants the tendency kernels use for WENO7/9 and the centred
advecting-velocity interpolations (weno_coeffs.h, written by
csrc/gen_weno_coeffs.py through the primitive-function construction) must be
exactly those of the oracle's independent derivation (cell-average
Vandermonde inverses), and the committed header must be what the generator
writes."""
import importlib.util
import os
import subprocess
import sys

import pytest

from oracle import weno

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_2502_14148_amd", "csrc", "gen_weno_coeffs.py")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_weno_coeffs", GEN)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_header_is_current():
    assert subprocess.run([sys.executable, GEN, "--check"]).returncode == 0


@pytest.mark.parametrize("r", [4, 5])
def test_device_constants_equal_oracle_derivation(r):
    g = _gen()
    d, cand, full = g.ideal(r)
    assert tuple(d) == weno.ideal_weights(r)
    assert tuple(tuple(c) for c in cand) == weno.candidate_coefficients(r)
    assert tuple(full) == tuple(weno.interface_stencil(list(range(-r, r - 1))))
    assert tuple(g.interface_weights(list(range(-(r - 1), r - 1)))) == \
        weno.centred_coefficients(2 * r - 2)
    assert tuple(g.TAU[r]) == weno.TAU[r]
    n = r - 1
    for k in range(r):
        L, D = g.indicator_factors(list(range(-r + k, k)))
        # L D L^T must rebuild the oracle's quadratic form in the differences
        N = [[sum(L[a][m] * D[m] * L[b][m] for m in range(n)) for b in range(n)]
             for a in range(n)]
        assert tuple(tuple(row) for row in N) == weno.difference_forms(r)[k]
        assert all(x > 0 for x in D)
