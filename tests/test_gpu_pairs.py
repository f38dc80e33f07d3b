"""Composite level-pair sweeps through the C ABI (the default for FP64 real operators;
the tests set HPS_COMPOSE=1 explicitly, HPS_COMPOSE=0 turns them off).

The upward and downward products of two adjacent tree levels (the merge formulas after
eqs. (7)-(8), Algorithm 1 of Sec. 2.1) are multiplied out at build time and swept by one
launch per pair and direction.  The result is the same solve, rounded differently, so it
is held to the FP64 bar against the oracle on trees with an even and an odd number of
levels (top pair only; top pair plus a single bottom level; several pairs), with
Dirichlet data and interface jumps; through stepping, graph replay and the
allocation-free entry point; and at the benchmark size in tests/test_gpu_parity.py
(which also holds the per-level sweeps to the same bar there).
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

TOL64 = 1e-11
PAIR_FAMILIES = {"pair_up_fp64", "pair_top_fp64", "pair_down_fp64"}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return _t


def var_coefs(x, y):
    return dict(cxx=1.0 + 0.3 * np.sin(x + 2 * y), cyy=1.2 + 0.2 * np.cos(3 * x),
                cx=0.5 * np.sin(y), cy=-0.4 * np.cos(x), c0=0.3 * np.sin(x * y))


def setup(torch, n1, n2, p, gdt, flags=hps.HPS_FP64):
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0.0, n1 * h, 0.0, n2 * h, n1, n2, p)
    og = Grid(0.0, n1 * h, 0.0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    co = var_coefs(x[: og.n_int], y[: og.n_int])
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt, flags)
    return g, og, x, y, co, op


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def families(op, torch, fn):
    hps.hps_profile_enable(op, True)
    hps.hps_profile_read(op)
    out = fn()
    torch.cuda.synchronize()
    fam = set(hps.hps_profile_read(op))
    hps.hps_profile_enable(op, False)
    return out, fam


# (n1, n2, p): tree levels L = log2(n1 n2) = 2 (the top pair only), 3 (top pair and a
# single bottom level), 4, 5, 6, 7 and 10; the smallest and largest orders (p = 3: one
# interior node per leaf; p = 24)
SHAPES = [(2, 2, 8), (4, 2, 6), (4, 4, 8), (8, 4, 10), (4, 8, 7), (8, 8, 12), (16, 8, 7), (32, 32, 6),
          (4, 4, 3), (2, 4, 24)]


@pytest.mark.parametrize("n1,n2,p", SHAPES, ids=[f"{a}x{b}_p{c}" for a, b, c in SHAPES])
def test_pair_solve_matches_oracle(torch, monkeypatch, n1, n2, p):
    monkeypatch.setenv("HPS_COMPOSE", "1")
    say(f"[pairs] solve {n1}x{n2} p={p}")
    rng = np.random.default_rng(4000 + 100 * n1 + 10 * n2 + p)
    gdt = 0.01
    g, og, x, y, co, op = setup(torch, n1, n2, p, gdt)
    body = rng.standard_normal(og.n_int)
    dirv = rng.standard_normal(op.n_bdry)
    jump = rng.standard_normal(op.n_iface)
    T = lambda a: torch.tensor(a, device="cuda")
    u, fam = families(op, torch, lambda: hps.hps_solve(op, T(body), T(dirv), T(jump)))
    assert PAIR_FAMILIES & fam, fam
    e = rel(u.cpu().numpy(), HPS(og, co, gdt).solve(body, dirv, jump))
    say(f"   kernels {sorted(fam)}; rel err vs oracle {e:.2e}")
    assert e <= TOL64
    op.free()


PAIR_FAMILIES32 = {"pair_up_fp32", "pair_top_fp32", "pair_down_fp32"}


@pytest.mark.parametrize("n1,n2,p", [(4, 2, 6), (8, 8, 10), (16, 8, 7)], ids=["4x2_p6", "8x8_p10", "16x8_p7"])
def test_pair_fp32_ir_solve_matches_oracle(torch, monkeypatch, n1, n2, p):
    """FP32+IR operators sweep FP32 copies of the composites (each pass of the refinement),
    with Dirichlet data and interface jumps: the refined solve meets the 1e-10 bar."""
    monkeypatch.setenv("HPS_COMPOSE", "1")
    say(f"[pairs] FP32+IR solve {n1}x{n2} p={p}")
    rng = np.random.default_rng(4100 + 100 * n1 + 10 * n2 + p)
    gdt = 0.01
    g, og, x, y, co, op = setup(torch, n1, n2, p, gdt, hps.HPS_FP32_IR)
    body, dirv, jump = rng.standard_normal(og.n_int), rng.standard_normal(op.n_bdry), rng.standard_normal(op.n_iface)
    T = lambda a: torch.tensor(a, device="cuda")
    u, fam = families(op, torch, lambda: hps.hps_solve(op, T(body), T(dirv), T(jump)))
    assert PAIR_FAMILIES32 & fam, fam
    e = rel(u.cpu().numpy(), HPS(og, co, gdt).solve(body, dirv, jump))
    say(f"   kernels {sorted(fam)}; rel err vs oracle {e:.2e}")
    assert e <= 1e-10
    op.free()


def test_pairs_not_used_where_they_do_not_apply(torch, monkeypatch):
    """One tree level (no pair) and wide tiles keep the single-level sweeps; the solve is
    still the oracle's."""
    monkeypatch.setenv("HPS_COMPOSE", "1")
    rng = np.random.default_rng(5)
    gdt = 0.01
    for (n1, n2, p, flags, tol) in [(2, 1, 8, hps.HPS_FP64, TOL64), (8, 8, 10, hps.HPS_WIDE_TILES, TOL64)]:
        say(f"[pairs] not applicable: {n1}x{n2} p={p} flags={flags}")
        g, og, x, y, co, op = setup(torch, n1, n2, p, gdt, flags)
        body = rng.standard_normal(og.n_int)
        u, fam = families(op, torch, lambda: hps.hps_solve(op, torch.tensor(body, device="cuda")))
        assert not ((PAIR_FAMILIES | PAIR_FAMILIES32) & fam), fam
        e = rel(u.cpu().numpy(), HPS(og, co, gdt).solve(body))
        say(f"   rel err {e:.2e}")
        assert e <= tol
        op.free()


def test_pair_steps_match_oracle_and_replay_exactly(torch, monkeypatch):
    """Allen-Cahn steps (ARK4(3)6L[2]SA, 8x8 leaves, p = 10) on a composed operator: the
    same as the oracle's to the FP64 bar, and the graph-replayed step equal to the eagerly
    enqueued one bit for bit."""
    monkeypatch.setenv("HPS_COMPOSE", "1")
    say("[pairs] Allen-Cahn 8x8 p=10 steps")
    dt = 1e-3
    tab = product_tableau()
    gdt = tab["gamma"] * dt
    g = hps.make_grid(0, 1, 0, 1, 8, 8, 10)
    og = Grid(0, 1, 0, 1, 8, 8, 10)
    x, y = hps.hps_nodes(g)
    xi, yi = x[: og.n_int], y[: og.n_int]
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, c0 = wl.L_coeffs(xi, yi)
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt)
    ctx_g = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    ctx_e = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    ark = ARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt, workloads.AllenCahn.gpoly)
    u0 = wl.u0(x, y)
    ug = torch.tensor(u0, device="cuda")
    ue = ug.clone()
    ur = u0.copy()
    for n in range(5):
        monkeypatch.setenv("HPS_GRAPHS", "1")
        if n == 0:
            _, fam = families(op, torch, lambda: hps.ark_step(ctx_g, n * dt, ug))
            assert PAIR_FAMILIES & fam, fam
        else:
            hps.ark_step(ctx_g, n * dt, ug)
        torch.cuda.synchronize()
        monkeypatch.setenv("HPS_GRAPHS", "0")
        hps.ark_step(ctx_e, n * dt, ue)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), n
        ur = ark.step(ur)
        e = rel(ug.cpu().numpy(), ur)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL64
    del ctx_g, ctx_e
    op.free()


def test_pair_noalloc_equals_solve(torch, monkeypatch):
    """The allocation-free entry point runs the same composite sweeps (its scratch holds
    the per-level data), so it equals hps_solve bit for bit."""
    monkeypatch.setenv("HPS_COMPOSE", "1")
    say("[pairs] noalloc 8x4 p=10")
    rng = np.random.default_rng(6)
    g, og, x, y, co, op = setup(torch, 8, 4, 10, 0.01)
    T = lambda a: torch.tensor(a, device="cuda")
    body, dirv, jump = rng.standard_normal(og.n_int), rng.standard_normal(op.n_bdry), rng.standard_normal(op.n_iface)
    u1 = hps.hps_solve(op, T(body), T(dirv), T(jump))
    u2 = hps.hps_solve_noalloc(op, T(body), T(dirv), T(jump))
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    op.free()


def test_uniform_operator_pairs_stored_once(torch, monkeypatch):
    """Constant coefficients (HPS_UNIFORM_COEFFS): every node's composite is the same, so it
    is computed and stored once; the sweeps use it and equal the per-node operator's bit
    for bit."""
    monkeypatch.setenv("HPS_COMPOSE", "1")
    say("[pairs] uniform coefficients, 8x8 p=10")
    const = lambda x, y: dict(cxx=1.3 + 0 * x, cyy=0.8 + 0 * x, cx=0.2 + 0 * x, cy=-0.1 + 0 * x, c0=0.05 + 0 * x)
    h = 1.0 / 8
    g = hps.make_grid(0.0, 1.0, 0.0, 1.0, 8, 8, 10)
    og = Grid(0.0, 1.0, 0.0, 1.0, 8, 8, 10)
    x, y = hps.hps_nodes(g)
    co = const(x[: og.n_int], y[: og.n_int])
    dco = {k: torch.tensor(v, device="cuda") for k, v in co.items()}
    full = hps.hps_build(g, dco, 0.01, hps.HPS_FP64)
    uni = hps.hps_build(g, dco, 0.01, hps.HPS_UNIFORM_COEFFS)
    assert uni.bytes()[1] * 4 < full.bytes()[1]
    rng = np.random.default_rng(8)
    T = lambda a: torch.tensor(a, device="cuda")
    body, dirv, jump = rng.standard_normal(og.n_int), rng.standard_normal(full.n_bdry), rng.standard_normal(full.n_iface)
    a = hps.hps_solve(full, T(body), T(dirv), T(jump))
    b, fam = families(uni, torch, lambda: hps.hps_solve(uni, T(body), T(dirv), T(jump)))
    assert PAIR_FAMILIES & fam, fam
    assert torch.equal(a, b)
    e = rel(b.cpu().numpy(), HPS(og, co, 0.01).solve(body, dirv, jump))
    say(f"   rel err vs oracle {e:.2e}")
    assert e <= TOL64
    full.free()
    uni.free()


@pytest.mark.parametrize("compose,flags", [("1", hps.HPS_FP64), ("0", hps.HPS_FP64), ("0", hps.HPS_FP32_IR)],
                         ids=["pairs", "levels", "fp32ir"])
def test_zero_dirichlet_data_skips_nothing_that_matters(torch, monkeypatch, compose, flags):
    """Without Dirichlet data the top pair (or the fused root) does not stream the columns
    that multiply the (zero) boundary values: the solve equals the one given explicit zeros
    bit for bit, for one right-hand side and for several."""
    monkeypatch.setenv("HPS_COMPOSE", compose)
    say(f"[pairs] no Dirichlet data vs explicit zeros, 8x8 p=12, compose={compose} flags={flags}")
    rng = np.random.default_rng(10)
    g, og, x, y, co, op = setup(torch, 8, 8, 12, 0.01, flags)
    T = lambda a: torch.tensor(a, device="cuda")
    body, jump = rng.standard_normal(og.n_int), rng.standard_normal(op.n_iface)
    zeros = torch.zeros(op.n_bdry, dtype=torch.float64, device="cuda")
    a = hps.hps_solve(op, T(body), None, T(jump))
    b = hps.hps_solve(op, T(body), zeros, T(jump))
    assert torch.equal(a, b)
    bodies = T(rng.standard_normal((3, og.n_int)))
    am = hps.hps_solve(op, bodies)
    bm = hps.hps_solve(op, bodies, torch.zeros((3, op.n_bdry), dtype=torch.float64, device="cuda"))
    assert torch.equal(am, bm)
    e = rel(a.cpu().numpy(), HPS(og, co, 0.01).solve(body, None, jump))
    say(f"   rel err vs oracle {e:.2e}")
    assert e <= (TOL64 if flags == hps.HPS_FP64 else 1e-10)
    op.free()
