"""The FP64 conditioning floor of the benchmark grid, measured on the oracle alone.

Two evaluations of one Allen-Cahn step that are both correct in exact arithmetic -- the
oracle as written (LU solves) and the same oracle with explicit inverses in place of its
LU solves (``tests/inverse_oracle.py``; the GPU library also applies explicit inverses) --
are compared.  Their relative difference is how closely any FP64 implementation can be
expected to reproduce the oracle at that size.  It fixes the parity bar of the full-size
GPU tests: at 64x64 leaves, p = 16 (gamma dt = 2.5e-4) the stage operator I - gamma dt L_h
has condition number ~1e5 and the spread exceeds the 1e-11 target, so those tests compare
against 1e-10 and against a small multiple of this spread; at 16x16 leaves the spread is
below 1e-12 and the 1e-11 bar applies.
"""
import numpy as np
import pytest

from inverse_oracle import explicit_inverses
from oracle.ark import ARK, ark436l2sa, tableau_float
from oracle.grid import Grid
from oracle.hps import HPS
from paper_2306_02526_amd import workloads


def _step_both_ways(n, p, dt=1e-3):
    g = Grid(0, 1, 0, 1, n, n, p)
    x, y = g.coordinates()
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, c0 = wl.L_coeffs(x[: g.n_int], y[: g.n_int])
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    tab = tableau_float(ark436l2sa())
    u0 = wl.u0(x, y)
    a = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt, workloads.AllenCahn.gpoly).step(u0)
    with explicit_inverses():
        b = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt, workloads.AllenCahn.gpoly).step(u0)
    return np.abs(a - b).max() / np.abs(a).max()


def test_explicit_inverse_variant_is_the_same_solution():
    """The variant is a valid evaluation: on a small grid it agrees with the LU oracle to
    rounding (and it really is a different evaluation: not bitwise equal)."""
    s = _step_both_ways(4, 8)
    assert 0.0 < s <= 1e-13, s


def test_conditioning_floor_at_16x16_is_below_the_fp64_target():
    s = _step_both_ways(16, 16)
    assert s <= 1e-12, s   # measured 6.9e-13


@pytest.mark.slow
def test_conditioning_floor_at_the_benchmark_grid_exceeds_the_fp64_target():
    """64x64 leaves, p = 16: measured 1.81e-11 (about 75 s of oracle time on one core).
    No FP64 evaluation order can be held to 1e-11 of the LU oracle here; 1e-10 leaves the
    GPU path a margin of 5x over this spread."""
    s = _step_both_ways(64, 16)
    assert 1e-11 <= s <= 5e-11, s
