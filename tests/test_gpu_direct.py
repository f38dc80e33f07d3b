"""The direct sweep of small trees through the C ABI.

With no boundary or jump data the interface values of a solve are a linear function of the
leaves' particular fluxes alone (Algorithm 1 of Sec. 2.1), so a small tree's whole level
sweep is one product with a matrix the build takes from the operator's own sweeps of unit
vectors.  The solve is the same one, rounded differently: it is held to the FP64 bar against
the oracle and to rounding against the level sweeps (HPS_DIRECT=0), and the sweep is used
only where it applies (no Dirichlet or jump data, FP64 real operators of small trees).
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


def setup(torch, monkeypatch, n1, n2, p, gdt, direct, flags=hps.HPS_FP64):
    monkeypatch.setenv("HPS_DIRECT", "1" if direct else "0")
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0.0, n1 * h, 0.0, n2 * h, n1, n2, p)
    og = Grid(0.0, n1 * h, 0.0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    xi, yi = x[: og.n_int], y[: og.n_int]
    co = dict(cxx=1.0 + 0.3 * np.sin(xi + 2 * yi), cyy=1.2 + 0.2 * np.cos(3 * xi), cx=0.5 * np.sin(yi),
              cy=-0.4 * np.cos(xi), c0=0.3 * np.sin(xi * yi))
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt, flags)
    monkeypatch.delenv("HPS_DIRECT")
    return og, co, op


def families(op, torch, fn):
    hps.hps_profile_enable(op, True)
    hps.hps_profile_read(op)
    out = fn()
    torch.cuda.synchronize()
    fam = set(hps.hps_profile_read(op))
    hps.hps_profile_enable(op, False)
    return out, fam


# trees of 2 to 5 levels, one interior node per leaf (p = 3) to p = 12
SHAPES = [(2, 2, 8), (4, 2, 6), (4, 4, 8), (8, 4, 8), (4, 4, 3), (4, 4, 12), (2, 8, 5)]


@pytest.mark.parametrize("n1,n2,p", SHAPES, ids=[f"{a}x{b}_p{c}" for a, b, c in SHAPES])
def test_direct_solve_matches_oracle_and_level_sweeps(torch, monkeypatch, n1, n2, p):
    say(f"[direct] solve {n1}x{n2} p={p}")
    gdt = 0.01
    og, co, op = setup(torch, monkeypatch, n1, n2, p, gdt, True)
    _, _, ref_op = setup(torch, monkeypatch, n1, n2, p, gdt, False)
    body = np.random.default_rng(5000 + 100 * n1 + 10 * n2 + p).standard_normal(og.n_int)
    T = lambda a: torch.tensor(a, device="cuda")
    u, fam = families(op, torch, lambda: hps.hps_solve(op, T(body)))
    assert "direct_fp64" in fam, fam
    ul, faml = families(ref_op, torch, lambda: hps.hps_solve(ref_op, T(body)))
    assert "direct_fp64" not in faml, faml
    e = rel(u.cpu().numpy(), HPS(og, co, gdt).solve(body))
    d = rel(u.cpu().numpy(), ul.cpu().numpy())
    say(f"   rel err vs oracle {e:.2e}, vs the level sweeps {d:.2e}")
    assert e <= TOL64 and d <= 1e-13
    op.free()
    ref_op.free()


def test_direct_sweep_only_where_it_applies(torch, monkeypatch):
    """Dirichlet data, interface jumps, several right-hand sides, FP32+IR and wide tiles take
    the level sweeps; results stay at the oracle's."""
    gdt = 0.01
    og, co, op = setup(torch, monkeypatch, 4, 4, 8, gdt, True)
    rng = np.random.default_rng(17)
    T = lambda a: torch.tensor(a, device="cuda")
    body, dirv, jump = rng.standard_normal(og.n_int), rng.standard_normal(op.n_bdry), rng.standard_normal(op.n_iface)
    H = HPS(og, co, gdt)
    for name, fn, ref in [("dirichlet", lambda: hps.hps_solve(op, T(body), T(dirv)), H.solve(body, dirv)),
                          ("jump", lambda: hps.hps_solve(op, T(body), None, T(jump)), H.solve(body, None, jump))]:
        u, fam = families(op, torch, fn)
        e = rel(u.cpu().numpy(), ref)
        say(f"   {name}: {sorted(fam)}, rel err {e:.2e}")
        assert "direct_fp64" not in fam and e <= TOL64
    bodies = rng.standard_normal((3, og.n_int))
    um, fam = families(op, torch, lambda: hps.hps_solve(op, T(bodies)))
    assert "direct_fp64" not in fam
    for r in range(3):
        assert rel(um[r].cpu().numpy(), H.solve(bodies[r])) <= TOL64
    op.free()
    for flags in (hps.HPS_FP32_IR, hps.HPS_WIDE_TILES):
        _, _, o2 = setup(torch, monkeypatch, 4, 4, 8, gdt, True, flags)
        _, fam = families(o2, torch, lambda: hps.hps_solve(o2, T(body)))
        assert "direct_fp64" not in fam, (flags, fam)
        o2.free()


def test_direct_steps_match_oracle_and_replay_exactly(torch, monkeypatch):
    """The config-1 heat problem (4x4 leaves, p = 8, manufactured solution, zero boundary
    data): stage solves through the direct sweep, the oracle's steps to the FP64 bar, and
    the graph-replayed step equal to the eagerly enqueued one bit for bit."""
    say("[direct] heat 4x4 p=8 steps")
    tab = product_tableau()
    dt = 0.01
    gdt = tab["gamma"] * dt
    monkeypatch.setenv("HPS_DIRECT", "1")
    g = hps.make_grid(0, 1, 0, 1, 4, 4, 8)
    og = Grid(0, 1, 0, 1, 4, 4, 8)
    x, y = hps.hps_nodes(g)
    pr = workloads.HeatManufactured(workloads.rng_for(1))
    cxx, cyy, cx, cy, c0 = pr.L_coeffs(x[: og.n_int], y[: og.n_int])
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt)
    monkeypatch.delenv("HPS_DIRECT")
    ctx_g = hps.ark_create(op, tab, dt)
    ctx_e = hps.ark_create(op, tab, dt)
    ark = ARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt)
    qs = pr.q_space(x[: og.n_int], y[: og.n_int])
    qsd = torch.tensor(qs, device="cuda")
    u0 = pr.exact(0.0, x, y)
    ug, ue, ur = torch.tensor(u0, device="cuda"), torch.tensor(u0, device="cuda"), u0.copy()
    for n in range(10):
        t = n * dt
        qt = [pr.q_time(t + c * dt) for c in tab["c"]]
        monkeypatch.setenv("HPS_GRAPHS", "1")
        if n == 0:
            _, fam = families(op, torch, lambda: hps.ark_step(ctx_g, t, ug, q_space=qsd, q_time=qt))
            assert "direct_fp64" in fam, fam
        else:
            hps.ark_step(ctx_g, t, ug, q_space=qsd, q_time=qt)
        monkeypatch.setenv("HPS_GRAPHS", "0")
        hps.ark_step(ctx_e, t, ue, q_space=qsd, q_time=qt)
        assert torch.equal(ug, ue), n
        ur = ark.step(ur, q_stages=np.array([v * qs for v in qt]))
        e = rel(ug.cpu().numpy(), ur)
        assert e <= TOL64, (n, e)
    say(f"   10 steps: rel err vs oracle {e:.2e}")
    del ctx_g, ctx_e
    op.free()


def test_grouped_batch_and_noalloc_take_the_direct_product(torch, monkeypatch):
    """Grouped batched steps (HPS_GROUP=1) of Allen-Cahn problems: two contexts on one small
    operator (each with a workspace of its own), another small operator and a tree too large
    for the direct product, each equal to its single step bit for bit and to the oracle; and
    the allocation-free solve without boundary or jump data equal to hps_solve."""
    say("[direct] grouped batch with small and large trees; allocation-free solve")
    tab = product_tableau()
    dt = 2e-3
    gdt = tab["gamma"] * dt
    built = {}
    for n1, n2, p in [(4, 4, 8), (8, 4, 6), (16, 16, 10)]:
        og, co, op = setup(torch, monkeypatch, n1, n2, p, gdt, True)
        built[(n1, n2, p)] = (og, co, op)
    keys = [(4, 4, 8), (4, 4, 8), (8, 4, 6), (16, 16, 10)]
    ctxs = [hps.ark_create(built[k][2], tab, dt, g=workloads.AllenCahn.gpoly) for k in keys]
    singles = [hps.ark_create(built[k][2], tab, dt, g=workloads.AllenCahn.gpoly) for k in keys]
    arks = {k: ARK(HPS(og, co, gdt), co, tableau_float(ark436l2sa()), dt, workloads.AllenCahn.gpoly)
            for k, (og, co, _) in built.items()}
    us, refs = [], []
    for b, k in enumerate(keys):
        h = 1.0 / max(k[0], k[1])
        x, y = hps.hps_nodes(hps.make_grid(0.0, k[0] * h, 0.0, k[1] * h, *k))
        u0 = np.sin(3 * x + b) * np.cos(2 * y)
        us.append(torch.tensor(u0, device="cuda"))
        refs.append(u0)
    want = [u.clone() for u in us]
    monkeypatch.setenv("HPS_GROUP", "1")
    for n in range(2):
        hps.ark_step_batched(ctxs, [n * dt] * len(keys), us)
        for b in range(len(keys)):
            hps.ark_step(singles[b], n * dt, want[b])
            refs[b] = arks[keys[b]].step(refs[b])
        torch.cuda.synchronize()
        for b in range(len(keys)):
            assert torch.equal(us[b], want[b]), (n, b)
            e = rel(us[b].cpu().numpy(), refs[b])
            say(f"   step {n} problem {b} {keys[b]}: bitwise equal to its single step, rel err {e:.2e}")
            assert e <= TOL64
    monkeypatch.delenv("HPS_GROUP")
    del ctxs, singles
    rng = np.random.default_rng(23)
    for k in [(4, 4, 8), (8, 4, 6)]:
        og, co, op = built[k]
        body = torch.tensor(rng.standard_normal(og.n_int), device="cuda")
        u_na = hps.hps_solve_noalloc(op, body)
        torch.cuda.synchronize()
        u_ref = hps.hps_solve(op, body)
        torch.cuda.synchronize()
        assert torch.equal(u_na, u_ref), k
    for _, _, op in built.values():
        op.free()
