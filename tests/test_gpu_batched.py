"""Batched entry points (include/hps_batch.h) through the C ABI: every problem of a batch
must give what the single-problem entry point gives (FP64: bitwise, the same kernels run)
and what the CPU oracle gives (relative max-norm <= 1e-11, FP32+IR <= 1e-10)."""
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


def coefs(x, y, k):
    return dict(cxx=1.0 + 0.3 * np.sin(x + k * y), cyy=1.1 + 0.2 * np.cos(2 * x + k),
                cx=0.4 * np.sin(y + k), cy=-0.3 * np.cos(x), c0=0.2 * np.sin(x * y + k))


def build(torch, n1, n2, p, gdt, k, flags=hps.HPS_FP64):
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    og = Grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    co = coefs(x[: og.n_int], y[: og.n_int], k)
    op = hps.hps_build(g, {c: torch.tensor(v, device="cuda") for c, v in co.items()}, gdt, flags)
    return og, co, op


# (n1, n2, p, gamma_dt, flags): squares and rectangles, several orders, both precisions
MIX = [(4, 4, 12, 1e-2, hps.HPS_FP64), (2, 1, 6, 1e-3, hps.HPS_FP64), (1, 1, 5, 5e-3, hps.HPS_FP64),
       (8, 8, 10, 1e-2, hps.HPS_FP64), (2, 4, 8, 1e-3, hps.HPS_FP64), (4, 4, 8, 1e-2, hps.HPS_FP32_IR),
       (16, 8, 7, 2e-3, hps.HPS_FP64)]


def test_solve_batched_matches_single_and_oracle(torch):
    say(f"[batched] hps_solve_batched over {len(MIX) + 1} problems ({hps.hps_batch_streams()} streams)")
    probs = [build(torch, *m[:4], k, m[4]) for k, m in enumerate(MIX)]
    ops = [op for _, _, op in probs] + [probs[0][2]]       # the first operator twice
    ogs = [og for og, _, _ in probs] + [probs[0][0]]
    cos = [co for _, co, _ in probs] + [probs[0][1]]
    rng = np.random.default_rng(11)
    body = [rng.standard_normal(og.n_int) for og in ogs]
    dirichlet = [rng.standard_normal(op.n_bdry) for op in ops]
    jump = [rng.standard_normal(op.n_iface) if op.n_iface else None for op in ops]
    dev = lambda a: None if a is None else torch.tensor(a, device="cuda")
    db, dd, dj = [dev(v) for v in body], [dev(v) for v in dirichlet], [dev(v) for v in jump]
    u_b, info = hps.hps_solve_batched(ops, db, dd, dj, info=True)
    torch.cuda.synchronize()
    for b, (op, og, co) in enumerate(zip(ops, ogs, cos)):
        u_s = hps.hps_solve(op, db[b], dd[b], dj[b])
        gdt = MIX[b][3] if b < len(MIX) else MIX[0][3]
        ref = HPS(og, co, gdt).solve(body[b], dirichlet[b], jump[b])
        e = rel(u_b[b].cpu().numpy(), ref)
        tol = TOL32IR if op.flags == hps.HPS_FP32_IR else TOL64
        say(f"   problem {b}: {og.n1}x{og.n2} p={og.p} flags={op.flags}: oracle {e:.2e}, "
            f"IR passes {info[b]['ir_iterations']}")
        assert e <= tol, (b, e)
        if op.flags == hps.HPS_FP64:
            assert torch.equal(u_b[b], u_s), b


def test_ark_step_batched_mix_matches_oracle(torch):
    """The batched workload recipe (heat with manufactured solution / Allen-Cahn, smooth
    random diffusivity, square leaves on rectangles) at sizes the oracle runs quickly."""
    mix = workloads.batched_mix(n_problems=6, sides=(1, 2, 4), orders=(6, 8))
    tab = product_tableau()
    otab = tableau_float(ark436l2sa())
    ctxs, us, refs, orcs, probs = [], [], [], [], []
    for m in mix:
        x0, x1, y0, y1 = m["domain"]
        g = hps.make_grid(x0, x1, y0, y1, m["n1"], m["n2"], m["p"])
        og = Grid(x0, x1, y0, y1, m["n1"], m["n2"], m["p"])
        x, y = hps.hps_nodes(g)
        pr = m["problem"]
        cxx, cyy, cx, cy, c0 = pr.L_coeffs(x[: og.n_int], y[: og.n_int])
        co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
        gdt = m["gamma_dt"]
        dt = gdt / tab["gamma"]
        op = hps.hps_build(g, {c: torch.tensor(v, device="cuda") for c, v in co.items()}, gdt)
        gp = None if m["kind"] == "heat" else workloads.AllenCahn.gpoly
        ctxs.append(hps.ark_create(op, tab, dt, g=gp))
        u0 = pr.exact(0.0, x, y) if m["kind"] == "heat" else pr.u0(x, y)
        us.append(torch.tensor(u0, device="cuda"))
        refs.append(u0.copy())
        orcs.append(ARK(HPS(og, co, gdt), co, otab, dt, gp))
        probs.append((m, x, y, og, dt))
        say(f"   {m['kind']} {m['n1']}x{m['n2']} p={m['p']} gamma_dt={gdt:g}")
    qsp = [torch.tensor(m["problem"].q_space(x[: og.n_int], y[: og.n_int]), device="cuda")
           if m["kind"] == "heat" else None for m, x, y, og, dt in probs]
    singles = [u.clone() for u in us]
    for n in range(3):
        ts = [n * dt for _, _, _, _, dt in probs]
        qt = [[workloads.HeatManufactured.q_time(t + c * dt) for c in tab["c"]] if m["kind"] == "heat" else None
              for (m, _, _, _, dt), t in zip(probs, ts)]
        hps.ark_step_batched(ctxs, ts, us, q_space=qsp, q_time=qt)
        for b, ctx in enumerate(ctxs):
            hps.ark_step(ctx, ts[b], singles[b], q_space=qsp[b], q_time=qt[b])
            q_st = None
            if qt[b] is not None:
                qs = qsp[b].cpu().numpy()
                q_st = np.array([v * qs for v in qt[b]])
            refs[b] = orcs[b].step(refs[b], q_stages=q_st)
        torch.cuda.synchronize()
        for b in range(len(ctxs)):
            e = rel(us[b].cpu().numpy(), refs[b])
            assert e <= TOL64, (n, b, e)
            assert torch.equal(us[b], singles[b]), (n, b)
    say("   3 batched steps: parity with the oracle and bitwise equal to single steps")


def test_batched_rejects_missing_entries(torch):
    g = hps.make_grid(0, 1, 0, 1, 2, 2, 6)
    og = Grid(0, 1, 0, 1, 2, 2, 6)
    x, y = hps.hps_nodes(g)
    co = coefs(x[: og.n_int], y[: og.n_int], 0)
    op = hps.hps_build(g, {c: torch.tensor(v, device="cuda") for c, v in co.items()}, 1e-2)
    body = torch.zeros(og.n_int, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        hps.hps_solve_batched([op, op], [body, None])
    assert hps.hps_solve_batched([], []) == []


@pytest.mark.parametrize("flags", [hps.HPS_FP64, hps.HPS_WIDE_TILES, hps.HPS_FP32_IR,
                                   hps.HPS_FP32_IR | hps.HPS_WIDE_TILES],
                         ids=["thin", "wide", "fp32ir_thin", "fp32ir_wide"])
def test_grouped_batched_steps_match_single_steps_and_oracle(torch, monkeypatch, flags):
    """Problems with at least two leaves run as grouped launches (one launch per leaf
    phase and per tree level for all problems; two of them share one operator and use
    workspaces of their own): the same bits as single steps, and the oracle's result; the
    plan and its graph are reused on later steps.  Both level tilings (thin tiles for one
    problem, wide tiles for many), FP64 and FP32+IR (after each context's first,
    host-checked step, the refined steps of all problems are grouped too: each problem
    keeps its own number of corrections per stage)."""
    ir = bool(flags & hps.HPS_FP32_IR)
    tol = TOL32IR if ir else TOL64
    mix = workloads.batched_mix(n_problems=7, stream=6, sides=(2, 4, 8), orders=(6, 8, 10))
    tab = product_tableau()
    otab = tableau_float(ark436l2sa())
    res = {}
    for mode in ("grouped", "streams"):
        monkeypatch.setenv("HPS_GROUP", "1" if mode == "grouped" else "0")
        ctxs, us, probs, orcs, refs = [], [], [], [], []
        for m in mix:
            x0, x1, y0, y1 = m["domain"]
            g = hps.make_grid(x0, x1, y0, y1, m["n1"], m["n2"], m["p"])
            og = Grid(x0, x1, y0, y1, m["n1"], m["n2"], m["p"])
            x, y = hps.hps_nodes(g)
            pr = m["problem"]
            cxx, cyy, cx, cy, c0 = pr.L_coeffs(x[: og.n_int], y[: og.n_int])
            co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
            dt = m["gamma_dt"] / tab["gamma"]
            op = hps.hps_build(g, {c: torch.tensor(v, device="cuda") for c, v in co.items()}, m["gamma_dt"],
                               flags)
            gp = None if m["kind"] == "heat" else workloads.AllenCahn.gpoly
            ctxs.append(hps.ark_create(op, tab, dt, g=gp))
            u0 = pr.exact(0.0, x, y) if m["kind"] == "heat" else pr.u0(x, y)
            us.append(torch.tensor(u0, device="cuda"))
            probs.append((m, x, y, og, dt))
            if mode == "grouped":
                orcs.append(ARK(HPS(og, co, m["gamma_dt"]), co, otab, dt, gp))
                refs.append(u0.copy())
            if len(ctxs) == 1:   # a second problem on the first operator, other initial data
                ctxs.append(hps.ark_create(op, tab, dt, g=gp))
                us.append(torch.tensor(0.5 * u0, device="cuda"))
                probs.append((m, x, y, og, dt))
                if mode == "grouped":
                    orcs.append(orcs[-1])
                    refs.append(0.5 * u0)
        qsp = [torch.tensor(m["problem"].q_space(x[: og.n_int], y[: og.n_int]), device="cuda")
               if m["kind"] == "heat" else None for m, x, y, og, dt in probs]
        out = []
        for n in range(4 if ir else 3):
            ts = [n * dt for *_, dt in probs]
            qt = [[workloads.HeatManufactured.q_time(t + c * dt) for c in tab["c"]] if m["kind"] == "heat" else None
                  for (m, _, _, _, dt), t in zip(probs, ts)]
            hps.ark_step_batched(ctxs, ts, us, q_space=qsp, q_time=qt)
            torch.cuda.synchronize()
            out.append([u.clone() for u in us])
            if mode == "grouped":
                for b in range(len(ctxs)):
                    q_st = None
                    if qt[b] is not None:
                        qs = qsp[b].cpu().numpy()
                        q_st = np.array([v * qs for v in qt[b]])
                    refs[b] = orcs[b].step(refs[b], q_stages=q_st)
                    e = rel(us[b].cpu().numpy(), refs[b])
                    assert e <= tol, (n, b, e)
        res[mode] = out
        if ir:
            say(f"   refinement records: {[hps.ark_info(c) for c in ctxs[:3]]}")
        say(f"   {mode}: {len(ctxs)} problems ({len(mix)} operators), {len(out)} steps")
    for a, b in zip(res["grouped"], res["streams"]):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
