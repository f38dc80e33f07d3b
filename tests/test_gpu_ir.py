"""FP32 operators with FP64 iterative refinement: the replayed step, the FP64 fallback, the
strict mode's error, and the build's zero-pivot error, through the C ABI.

The refinement (residual in FP64, corrections with the FP32 operators, stop when
||delta||_inf <= 1e-11 ||u||_inf) is checked against the oracle's stage solves (Sec. 3.1,
eqs. 9-11; Algorithm 1 of Sec. 2.1 for each solve) at 1e-10.  Failure handling is forced
from the host with the HPS_TEST_FP32_SKEW build flag, which stores the FP32 leaf inverses
multiplied by 1.5, so every correction removes only about half of the error: a numerical
failure of the refinement, not a GPU fault.
"""
import sys

import numpy as np
import pytest

from oracle.ark import ARK, ark436l2sa, tableau_float
from oracle.grid import Grid
from oracle.hps import HPS
from paper_2306_02526_amd import hps, workloads
from paper_2306_02526_amd.tableau import ark436l2sa as product_tableau

pytestmark = pytest.mark.gpu

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


def allen_cahn(torch, n, p, dt, flags):
    tab = product_tableau()
    gdt = tab["gamma"] * dt
    g = hps.make_grid(0, 1, 0, 1, n, n, p)
    og = Grid(0, 1, 0, 1, n, n, p)
    x, y = hps.hps_nodes(g)
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, c0 = wl.L_coeffs(x[: og.n_int], y[: og.n_int])
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt, flags)
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    return og, co, op, ctx, wl.u0(x, y), gdt


def test_replayed_fp32_ir_steps_match_oracle(torch):
    """First step host-checked, later steps replayed with the measured number of corrections
    per stage; every step within 1e-10 of the oracle, every stage converged."""
    say("[ir] Allen-Cahn 16x16 p=12 FP32+IR, 5 steps")
    dt = 1e-3
    og, co, op, ctx, u, gdt = allen_cahn(torch, 16, 12, dt, hps.HPS_FP32_IR)
    orc = ARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt, workloads.AllenCahn.gpoly)
    ug = torch.tensor(u, device="cuda")
    for n in range(5):
        hps.ark_step(ctx, n * dt, ug)
        info = hps.ark_info(ctx)
        u = orc.step(u)
        e = rel(ug.cpu().numpy(), u)
        say(f"   step {n}: rel err {e:.2e}, {info}")
        assert e <= TOL32IR
        assert info["fp64_fallbacks"] == 0 and 1 <= info["ir_iterations"] <= 10
        assert info["last_correction"] <= 1e-11
    del ctx
    op.free()


@pytest.mark.parametrize("n1,n2,p,extra", [(1, 1, 8, 0), (2, 1, 6, 0), (4, 2, 9, 0),
                                          (8, 4, 7, hps.HPS_WIDE_TILES), (8, 8, 8, hps.HPS_UNIFORM_COEFFS)],
                         ids=["1x1_p8", "2x1_p6", "4x2_p9", "8x4_p7_wide", "8x8_p8_uniform"])
def test_replayed_steps_on_small_and_odd_trees(torch, n1, n2, p, extra):
    """Replayed refined steps run the fused passes (residual in the leaf kernel that adds the
    previous correction, the last correction fused with the evaluation of L u_i, F_i): one
    leaf, odd trees (a single bottom level below the composite pairs), wide level tiles
    (no composites) and shared operators, against the oracle over four steps."""
    say(f"[ir] replayed fused passes, {n1}x{n2} p={p}, flags {hps.HPS_FP32_IR | extra}")
    tab = product_tableau()
    dt = 2e-3
    gdt = tab["gamma"] * dt
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    og = Grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    wl = workloads.AllenCahn(workloads.rng_for(3))
    if extra & hps.HPS_UNIFORM_COEFFS:
        one = np.ones(og.n_int)
        co = dict(cxx=1.3 * one, cyy=0.8 * one, cx=0.2 * one, cy=-0.1 * one, c0=0.05 * one)
    else:
        cxx, cyy, cx, cy, c0 = wl.L_coeffs(x[: og.n_int], y[: og.n_int])
        co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt,
                       hps.HPS_FP32_IR | extra)
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    orc = ARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt, workloads.AllenCahn.gpoly)
    u = wl.u0(x, y)
    ug = torch.tensor(u, device="cuda")
    for n in range(4):
        hps.ark_step(ctx, n * dt, ug)
        info = hps.ark_info(ctx)
        u = orc.step(u)
        e = rel(ug.cpu().numpy(), u)
        say(f"   step {n}: rel err {e:.2e}, {info}")
        assert e <= TOL32IR and info["fp64_fallbacks"] == 0
    del ctx
    op.free()


def test_failed_refinement_falls_back_to_fp64_bitwise(torch, monkeypatch):
    """With refinement made to fail, every stage is re-solved with the operator's FP64
    copy: the steps equal those of a plain FP64 operator bit for bit, and the record says
    so; hps_solve likewise.  (Both operators sweep the same FP64 composite level pairs.)"""
    say("[ir] forced refinement failure, 8x8 p=10, 3 steps")
    dt = 1e-3
    og, co, op64, c64, u0, gdt = allen_cahn(torch, 8, 10, dt, hps.HPS_FP64)
    _, _, opsk, csk, _, _ = allen_cahn(torch, 8, 10, dt, hps.HPS_FP32_IR | hps.HPS_TEST_FP32_SKEW)
    a, b = torch.tensor(u0, device="cuda"), torch.tensor(u0, device="cuda")
    for n in range(3):
        hps.ark_step(c64, n * dt, a)
        hps.ark_step(csk, n * dt, b)
        info = hps.ark_info(csk)
        say(f"   step {n}: {info}")
        assert torch.equal(a, b), float((a - b).abs().max())
        assert info["fp64_fallbacks"] == 5
    assert hps.ark_info(c64) == {"ir_iterations": 0, "last_correction": 0.0, "fp64_fallbacks": 0}
    rng = np.random.default_rng(5)
    body = torch.tensor(rng.standard_normal(og.n_int), device="cuda")
    dirv = torch.tensor(rng.standard_normal(op64.n_bdry), device="cuda")
    u64 = hps.hps_solve(op64, body, dirv)
    usk, info = hps.hps_solve(opsk, body, dirv, info=True)
    say(f"   hps_solve: {info}")
    assert info["fp64_fallbacks"] == 1 and info["ir_iterations"] == 10 and info["last_correction"] > 1e-11
    assert torch.equal(u64, usk)
    del c64, csk
    op64.free()
    opsk.free()


def test_strict_refinement_reports_not_converged(torch):
    say("[ir] HPS_IR_STRICT with failing refinement")
    dt = 1e-3
    og, _, op, ctx, u0, _ = allen_cahn(torch, 4, 8, dt, hps.HPS_FP32_IR | hps.HPS_TEST_FP32_SKEW | hps.HPS_IR_STRICT)
    ug = torch.tensor(u0, device="cuda")
    with pytest.raises(hps.HPSError) as ei:
        hps.ark_step(ctx, 0.0, ug)
    assert ei.value.code == -5 and "converge" in str(ei.value)
    with pytest.raises(hps.HPSError) as ei:
        hps.hps_solve(op, torch.ones(og.n_int, dtype=torch.float64, device="cuda"))
    assert ei.value.code == -5
    del ctx
    op.free()


def test_zero_pivot_is_reported(torch):
    """A = I - gamma dt L is singular when L u = u / (gamma dt): every leaf matrix is zero,
    the first pivot vanishes, and the build returns HPS_ESINGULAR.  (gamma dt = 1/4 and
    c0 = 4 make 1 - gamma dt c0 exactly zero however it is rounded or fused.)"""
    say("[build] singular operator")
    gdt = 0.25
    g = hps.make_grid(0, 1, 0, 1, 2, 2, 6)
    _, n_int, _, _ = hps.hps_num_nodes(g)
    c0 = torch.full((n_int,), 1.0 / gdt, dtype=torch.float64, device="cuda")
    with pytest.raises(hps.HPSError) as ei:
        hps.hps_build(g, {"c0": c0}, gdt)
    assert ei.value.code == -4 and "pivot" in str(ei.value)
    # the library stays usable
    op = hps.hps_build(g, {"c0": torch.zeros_like(c0)}, gdt)
    op.free()
