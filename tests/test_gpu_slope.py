"""Slope formulation with flux-jump penalisation (ark_step_slope) through the C ABI against
the oracle's SlopeARK on the same seeded inputs: FP64 <= 1e-11, FP32+IR <= 1e-10."""
import math
import sys

import numpy as np
import pytest

from oracle.ark import InterfaceSolver, SlopeARK, ark436l2sa, tableau_float
from oracle.grid import Grid
from oracle.hps import HPS
from paper_2306_02526_amd import hps, workloads
from paper_2306_02526_amd.tableau import ark436l2sa as product_tableau

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32IR = 1e-10


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return _t


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def var_coefs(x, y):
    return dict(cxx=1.0 + 0.3 * np.sin(x + 2 * y), cyy=1.2 + 0.2 * np.cos(3 * x), cx=0.5 * np.sin(y),
                cy=-0.4 * np.cos(x), c0=0.3 * np.sin(x * y))


def problem(torch, n1, n2, p, dt, flags=hps.HPS_FP64, gpoly=None):
    tab = product_tableau()
    gdt = tab["gamma"] * dt
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    og = Grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    co = var_coefs(x[: og.n_int], y[: og.n_int])
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt, flags)
    ctx = hps.ark_create(op, tab, dt, g=gpoly)
    orc = SlopeARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt, gpoly)
    return tab, og, x, y, op, ctx, orc


def test_slope_time_dependent_boundary_and_flux_jumps(torch):
    """Variable coefficients on a 4x2 rectangle, stage sources, time-dependent boundary slopes
    and a start vector with flux jumps (the penalty is active), 3 steps."""
    say("[slope] 4x2 p=9, sources, boundary slopes, penalty")
    dt = 0.01
    tab, og, x, y, op, ctx, orc = problem(torch, 4, 2, 9, dt)
    rng = np.random.default_rng(31)
    u = rng.standard_normal(og.N)
    ug = torch.tensor(u, device="cuda")
    jump0 = np.abs(InterfaceSolver(og).jump(u)).max()
    for n in range(3):
        q = rng.standard_normal((tab["s"], og.n_int))
        fd = rng.standard_normal((tab["s"], op.n_bdry))
        hps.ark_step_slope(ctx, n * dt, ug, q_stages=torch.tensor(q, device="cuda"),
                           fdot_stages=torch.tensor(fd, device="cuda"))
        u = orc.step(u, q_stages=q, fdot_stages=fd)
        e = rel(ug.cpu().numpy(), u)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL64
    jump3 = np.abs(InterfaceSolver(og).jump(ug.cpu().numpy())).max()
    say(f"   flux jump {jump0:.2e} -> {jump3:.2e}")
    assert jump3 <= 1e-11 * jump0


def test_slope_with_nonlinearity_and_separable_source(torch):
    """Allen-Cahn type g = u - u^3 with zero boundary data, separable source q_time q_space,
    on 8x8 leaves, p = 10, 4 steps."""
    say("[slope] 8x8 p=10, g = u - u^3, separable source")
    dt = 1e-3
    gp = workloads.AllenCahn.gpoly
    tab, og, x, y, op, ctx, orc = problem(torch, 8, 8, 10, dt, gpoly=gp)
    wl = workloads.AllenCahn(workloads.rng_for(2))
    u = wl.u0(x, y)
    ug = torch.tensor(u, device="cuda")
    qs = np.sin(3 * x[: og.n_int]) * np.cos(y[: og.n_int])
    qsd = torch.tensor(qs, device="cuda")
    for n in range(4):
        t = n * dt
        qt = [math.exp(-(t + c * dt)) for c in tab["c"]]
        hps.ark_step_slope(ctx, t, ug, q_space=qsd, q_time=qt)
        u = orc.step(u, q_stages=np.array([v * qs for v in qt]))
        e = rel(ug.cpu().numpy(), u)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL64


def test_slope_fp32_ir(torch):
    say("[slope] FP32 operators + FP64 refinement, 4x4 p=8")
    dt = 1e-3
    tab, og, x, y, op, ctx, orc = problem(torch, 4, 4, 8, dt, flags=hps.HPS_FP32_IR,
                                          gpoly=workloads.AllenCahn.gpoly)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(og.N)
    u[og.boundary_indices()] = 0.0
    ug = torch.tensor(u, device="cuda")
    for n in range(2):
        hps.ark_step_slope(ctx, n * dt, ug)
        u = orc.step(u)
        e = rel(ug.cpu().numpy(), u)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL32IR


def test_slope_graph_replay_equals_eager(torch, monkeypatch):
    """The FP64 slope step is captured into a HIP graph and replayed; replays (with eager
    torch work between them) equal the eagerly enqueued steps bit for bit."""
    say("[slope] graph replay vs eager, 8x4 p=8")
    dt = 1e-3
    res = []
    for graphs in ("1", "0"):
        monkeypatch.setenv("HPS_GRAPHS", graphs)
        tab, og, x, y, op, ctx, orc = problem(torch, 8, 4, 8, dt, gpoly=workloads.AllenCahn.gpoly)
        u = torch.tensor(np.sin(math.pi * x) * np.sin(2 * math.pi * y), device="cuda")
        out = []
        for n in range(4):
            hps.ark_step_slope(ctx, n * dt, u)
            junk = torch.randn(1000, device="cuda").sum()
            torch.cuda.synchronize()
            out.append(u.clone())
        res.append(out)
    for a, b in zip(*res):
        assert torch.equal(a, b)
