"""Checkpoint and resume: a run of 5 steps, saved as (u^n, t^n) on the host and resumed on
an operator rebuilt from the same key (grid, coefficients, gamma dt) in a fresh context,
equals 10 uninterrupted steps bit for bit.  The build and the steps are deterministic
(fixed reduction orders, no atomics in any sum), so a stored state is all a restart needs.
"""
import sys

import numpy as np
import pytest

from oracle.grid import Grid
from paper_2306_02526_amd import hps, workloads
from paper_2306_02526_amd.tableau import ark436l2sa as product_tableau

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return _t


def make(torch, key):
    n, p, dt = key
    tab = product_tableau()
    g = hps.make_grid(0, 1, 0, 1, n, n, p)
    og = Grid(0, 1, 0, 1, n, n, p)
    x, y = hps.hps_nodes(g)
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, c0 = wl.L_coeffs(x[: og.n_int], y[: og.n_int])
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, tab["gamma"] * dt)
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    return op, ctx, wl.u0(x, y)


@pytest.mark.parametrize("key", [(16, 10, 1e-3), (32, 8, 2e-3)])
def test_five_plus_five_steps_equal_ten(torch, key):
    say(f"[resume] Allen-Cahn {key[0]}x{key[0]} p={key[1]} dt={key[2]}")
    dt = key[2]
    op, ctx, u0 = make(torch, key)
    ref = torch.tensor(u0, device="cuda")
    for n in range(10):
        hps.ark_step(ctx, n * dt, ref)
    ref = ref.cpu().numpy()
    del ctx
    op.free()
    # first half, then a checkpoint on the host
    op, ctx, u0 = make(torch, key)
    u = torch.tensor(u0, device="cuda")
    for n in range(5):
        hps.ark_step(ctx, n * dt, u)
    saved_u, saved_t = u.cpu().numpy().copy(), 5 * dt
    del ctx, u
    op.free()
    # resume on a rebuilt operator and a new context
    op, ctx, _ = make(torch, key)
    u = torch.tensor(saved_u, device="cuda")
    for n in range(5):
        hps.ark_step(ctx, saved_t + n * dt, u)
    out = u.cpu().numpy()
    say(f"   max |difference| {np.abs(out - ref).max():.1e}")
    assert np.array_equal(out, ref)
    del ctx
    op.free()
