"""Interface-line solves (step completion: interface values from flux continuity along each
grid line of leaves) on elongated grids, where the lines are long: lines of up to 256 leaves
are staged in LDS, longer ones take the per-thread kernel.  One ARK step with boundary data
and a cubic g, through the C ABI, against the oracle on the same inputs (FP64 <= 1e-11), and
the flux jumps of the result vanish."""
import sys

import numpy as np
import pytest

from oracle.ark import ARK, InterfaceSolver, ark436l2sa, tableau_float
from oracle.grid import Grid
from oracle.hps import HPS
from paper_2306_02526_amd import hps
from paper_2306_02526_amd.tableau import ark436l2sa as product_tableau

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


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


# (n1, n2, p): line lengths 128 and 256 (staged in LDS), 1024 and 512 (per-thread kernel)
SHAPES = [(128, 2, 6), (256, 4, 5), (1024, 2, 4), (2, 512, 4)]


@pytest.mark.parametrize("n1,n2,p", SHAPES, ids=[f"{a}x{b}_p{c}" for a, b, c in SHAPES])
def test_long_lines_step_matches_oracle(torch, n1, n2, p):
    say(f"[lines] {n1}x{n2} p={p}: one ARK step with boundary data")
    tab = product_tableau()
    dt = 1e-3
    gdt = tab["gamma"] * dt
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    og = Grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    xi, yi = x[: og.n_int], y[: og.n_int]
    co = dict(cxx=1.0 + 0.2 * np.sin(3 * xi), cyy=1.1 + 0.1 * np.cos(2 * yi), cx=0.3 * np.cos(yi),
              cy=-0.2 * np.sin(xi), c0=0.1 * np.cos(xi + yi))
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt)
    gp = (0.0, 1.0, 0.0, -1.0)
    ctx = hps.ark_create(op, tab, dt, g=gp)
    orc = ARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt, gp)
    bi = og.boundary_indices()
    u0 = np.sin(5 * x) * np.cos(3 * y) + 0.3
    fs = np.array([np.sin(5 * x[bi]) * np.cos(3 * y[bi]) + 0.3 + c * dt for c in list(tab["c"]) + [1.0]])
    ug = torch.tensor(u0, device="cuda")
    hps.ark_step(ctx, 0.0, ug, f_stages=torch.tensor(fs, device="cuda"))
    ref = orc.step(u0.copy(), None, fs)
    out = ug.cpu().numpy()
    e = rel(out, ref)
    jump = np.abs(InterfaceSolver(og).jump(out)).max()
    say(f"   rel err {e:.2e}, max flux jump {jump:.2e}")
    # p^2 max(n1, n2) = 16384 is the benchmark grid's scale (64x64 leaves, p = 16): there the
    # stage operator's condition number (~1e5) puts two valid FP64 evaluations ~1e-11 apart,
    # and the full-size parity test takes 1e-10; below that scale the FP64 bar holds
    assert e <= (1e-10 if p * p * max(n1, n2) >= 16384 else TOL64)
    # the jump equations have entries of size ~p^2/h = p^2 max(n1, n2): roundoff times that
    assert jump <= 1e-14 * np.abs(out).max() * p * p * max(n1, n2)
