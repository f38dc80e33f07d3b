"""The fifth-order pair ARK5(4)8L[2]SA (8 stages, 7 implicit stage solves per step; Sec. 3
names it and Sec. 5.4 integrates the rotating flow with it) through the C ABI: every entry
point that takes a tableau (stage and slope formulations, FP32+IR, the Burgers system,
complex operators, batched and grouped steps, graph replay), against the oracle stepping
with the same tableau on the same inputs: FP64 relative max-norm <= 1e-11, FP32+IR <= 1e-10;
at the benchmark size (64x64 leaves, p = 16) one step element by element to the FP64
conditioning floor of that size (1e-10, derived in test_gpu_parity)."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle.ark import ARK, InterfaceSolver, SlopeARK, ark548l2sa, tableau_float
from oracle.burgers import BurgersARK
from oracle.grid import Grid
from oracle.hps import HPS
from oracle.nls import NLSARK
from paper_2306_02526_amd import hps, workloads
from paper_2306_02526_amd.tableau import ark436l2sa as product_ark4
from paper_2306_02526_amd.tableau import ark548l2sa as product_tableau

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32IR = 1e-10
TOL_FULL = 1e-10
OTAB = tableau_float(ark548l2sa())


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


def real_problem(torch, n1, n2, p, dt, flags=hps.HPS_FP64, coef_fn=var_coefs, gpoly=None, slope=False):
    tab = product_tableau()
    assert tab["s"] == 8
    gdt = tab["gamma"] * dt
    h = 1.0 / max(n1, n2)
    g = hps.make_grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    og = Grid(0, n1 * h, 0, n2 * h, n1, n2, p)
    x, y = hps.hps_nodes(g)
    co = coef_fn(x[: og.n_int], y[: og.n_int])
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt, flags)
    ctx = hps.ark_create(op, tab, dt, g=gpoly)
    cls = SlopeARK if slope else ARK
    orc = cls(HPS(og, co, gdt), co, OTAB, dt, gpoly)
    return tab, g, og, x, y, co, op, ctx, orc


def allen_cahn_coefs(x, y):
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, c0 = wl.L_coeffs(x, y)
    return dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)


def test_ark5_allen_cahn_matches_oracle(torch):
    say("[ark5] Allen-Cahn 8x8 p=10, g = u - u^3, 5 steps")
    dt = 1e-3
    tab, g, og, x, y, co, op, ctx, orc = real_problem(torch, 8, 8, 10, dt, coef_fn=allen_cahn_coefs,
                                                      gpoly=workloads.AllenCahn.gpoly)
    assert hps.ark_stage_solves_per_step(ctx) == 7
    u0 = workloads.AllenCahn(workloads.rng_for(2)).u0(x, y)
    ug, ur = torch.tensor(u0, device="cuda"), u0.copy()
    for n in range(5):
        hps.ark_step(ctx, n * dt, ug)
        ur = orc.step(ur)
        e = rel(ug.cpu().numpy(), ur)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL64


def test_ark5_inhomogeneous_boundary_and_stage_source(torch):
    """Variable coefficients on a 4x2 rectangle, q given per stage (8 rows), Dirichlet data at
    the 8 stage times and t + dt (9 rows), a cubic g with all four terms."""
    say("[ark5] 4x2 p=9, stage sources, boundary data")
    dt = 0.02
    gp = (0.1, -0.3, 0.2, -0.5)
    tab, g, og, x, y, co, op, ctx, orc = real_problem(torch, 4, 2, 9, dt, gpoly=gp)
    bi = og.boundary_indices()
    u0 = np.sin(x + y) * np.cos(2 * y)
    ug, ur = torch.tensor(u0, device="cuda"), u0.copy()
    for n in range(4):
        t = n * dt
        qs = np.array([np.cos(x[: og.n_int] * (1 + c)) * math.exp(-(t + c * dt)) for c in tab["c"]])
        fs = np.array([np.sin(x[bi] + y[bi]) * np.cos(2 * y[bi]) * (1 + t + c * dt)
                       for c in list(tab["c"]) + [1.0]])
        assert qs.shape[0] == 8 and fs.shape[0] == 9
        hps.ark_step(ctx, t, ug, q_stages=torch.tensor(qs, device="cuda"), f_stages=torch.tensor(fs, device="cuda"))
        ur = orc.step(ur, qs, fs)
        e = rel(ug.cpu().numpy(), ur)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL64


def test_ark5_fp32_ir_matches_oracle(torch):
    say("[ark5 fp32+ir] Allen-Cahn 16x16 p=12, 3 steps")
    dt = 1e-3
    tab, g, og, x, y, co, op, ctx, orc = real_problem(torch, 16, 16, 12, dt, flags=hps.HPS_FP32_IR,
                                                      coef_fn=allen_cahn_coefs, gpoly=workloads.AllenCahn.gpoly)
    u0 = workloads.AllenCahn(workloads.rng_for(3)).u0(x, y)
    ug, ur = torch.tensor(u0, device="cuda"), u0.copy()
    for n in range(3):
        hps.ark_step(ctx, n * dt, ug)
        ur = orc.step(ur)
        e = rel(ug.cpu().numpy(), ur)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL32IR


def test_ark5_slope_formulation_matches_oracle(torch):
    """Slope formulation with flux-jump penalisation: random start with flux jumps, stage
    sources and boundary slopes, 3 steps; the jumps are removed."""
    say("[ark5 slope] 4x2 p=9, sources, boundary slopes, penalty")
    dt = 0.01
    tab, g, og, x, y, co, op, ctx, orc = real_problem(torch, 4, 2, 9, dt, slope=True)
    rng = np.random.default_rng(41)
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
    assert np.abs(InterfaceSolver(og).jump(ug.cpu().numpy())).max() <= 1e-11 * jump0


def test_ark5_rotating_flow_matches_oracle(torch):
    """The rotating-flow Burgers test, the configuration the paper integrates with this pair:
    [-pi, pi]^2, eps = 0.005, no-slip walls; 8x8 leaves, p = 12, 2 steps."""
    say("[ark5 burgers] rotating flow 8x8 p=12, 2 steps")
    rot = workloads.BurgersRotating()
    tab = product_tableau()
    dt = 0.01
    gdt = tab["gamma"] * dt
    g = hps.make_grid(*rot.domain, 8, 8, 12)
    og = Grid(*rot.domain, 8, 8, 12)
    x, y = hps.hps_nodes(g)
    cxx, cyy, cx, cy, c0 = workloads.burgers_coeffs(rot.eps, og.n_int)
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt)
    cu, cv = hps.ark_create(op, tab, dt), hps.ark_create(op, tab, dt)
    orc = BurgersARK(HPS(og, co, gdt), co, OTAB, dt)
    u, v = rot.u0(x, y)
    bnd = og.boundary_indices()
    u[bnd] = 0.0
    v[bnd] = 0.0
    ug, vg = torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda")
    for n in range(2):
        hps.ark_step_burgers(cu, cv, n * dt, ug, vg)
        u, v = orc.step(u, v)
        eu, ev = rel(ug.cpu().numpy(), u), rel(vg.cpu().numpy(), v)
        say(f"   step {n}: rel err u {eu:.2e}, v {ev:.2e}")
        assert eu <= TOL64 and ev <= TOL64


def test_ark5_nls_filamentation_matches_oracle(torch):
    say("[ark5 nls] filamentation 8x8 p=13, dt=0.005, 2 steps")
    nls = workloads.NLSFilamentation()
    tab = product_tableau()
    dt = 0.005
    og = Grid(*nls.domain, 8, 8, 13)
    x, y = og.coordinates()
    re, im = nls.coeffs(og.n_int)
    co = {k: re[k] + 1j * im[k] for k in re}
    g = hps.make_grid(*nls.domain, 8, 8, 13)
    op = hps.hps_build_complex(g, {k: torch.tensor(v, device="cuda") for k, v in re.items()},
                               {k: torch.tensor(v, device="cuda") for k, v in im.items()}, tab["gamma"] * dt)
    ctx = hps.ark_create(op, tab, dt, g=nls.g())
    orc = NLSARK(HPS(og, co, tab["gamma"] * dt), co, OTAB, dt, nls.b, nls.c, nls.eps)
    u = nls.u0(x, y)
    ug = torch.tensor(np.stack([u.real, u.imag]), device="cuda").contiguous()
    for n in range(2):
        hps.ark_step(ctx, n * dt, ug)
        u = orc.step(u)
        a = ug.cpu().numpy()
        e = rel(a[0] + 1j * a[1], u)
        say(f"   step {n}: rel err {e:.2e}")
        assert e <= TOL64


def test_ark5_graph_replay_equals_eager(torch, monkeypatch):
    say("[ark5] graph replay vs eager, 8x8 p=10")
    dt = 1e-3
    tab, g, og, x, y, co, op, ctx_g, orc = real_problem(torch, 8, 8, 10, dt, coef_fn=allen_cahn_coefs,
                                                        gpoly=workloads.AllenCahn.gpoly)
    ctx_e = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    ug = torch.tensor(workloads.AllenCahn(workloads.rng_for(2)).u0(x, y), device="cuda")
    ue = ug.clone()
    scratch = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    for n in range(4):
        monkeypatch.setenv("HPS_GRAPHS", "1")
        hps.ark_step(ctx_g, n * dt, ug)
        scratch.add_(1.0).mul_(0.5)
        torch.cuda.synchronize()
        monkeypatch.setenv("HPS_GRAPHS", "0")
        hps.ark_step(ctx_e, n * dt, ue)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), n


def test_ark5_batched_grouped_and_mixed_tableaux(torch, monkeypatch):
    """Three FP64 problems stepped with ARK5 in one batched call (grouped launches) equal
    their single steps bit for bit and the oracle; a batch mixing ARK5 and ARK4 contexts
    (different stage counts, so not grouped) equals single steps too."""
    say("[ark5 batched] grouped ARK5 batch and a mixed ARK4/ARK5 batch")
    monkeypatch.setenv("HPS_GROUP", "1")
    dt = 2e-3
    shapes = [(4, 4, 8), (8, 4, 10), (2, 2, 12)]
    probs = [real_problem(torch, n1, n2, p, dt, gpoly=workloads.AllenCahn.gpoly) for n1, n2, p in shapes]
    us = [torch.tensor(np.sin(3 * x) * np.cos(2 * y), device="cuda") for _, _, _, x, y, *_ in probs]
    refs = [u.cpu().numpy() for u in us]
    singles = [u.clone() for u in us]
    for n in range(2):
        hps.ark_step_batched([pr[7] for pr in probs], [n * dt] * 3, us)
        for b, pr in enumerate(probs):
            hps.ark_step(hps.ark_create(pr[6], pr[0], dt, g=workloads.AllenCahn.gpoly), n * dt, singles[b])
            refs[b] = pr[8].step(refs[b])
        torch.cuda.synchronize()
        for b in range(3):
            assert torch.equal(us[b], singles[b]), (n, b)
            e = rel(us[b].cpu().numpy(), refs[b])
            say(f"   step {n} problem {b}: rel err {e:.2e}")
            assert e <= TOL64
    # mixed stage counts: problem 0 with ARK4 (its own operator, gamma = 1/4), problems 1, 2 with ARK5
    t4 = product_ark4()
    g0, og0, x0 = probs[0][1], probs[0][2], probs[0][3]
    co0 = probs[0][5]
    op4 = hps.hps_build(g0, {k: torch.tensor(v, device="cuda") for k, v in co0.items()}, t4["gamma"] * dt)
    ctxs = [hps.ark_create(op4, t4, dt, g=workloads.AllenCahn.gpoly), probs[1][7], probs[2][7]]
    us2 = [torch.tensor(np.cos(x0), device="cuda"), us[1].clone(), us[2].clone()]
    want = [u.clone() for u in us2]
    hps.ark_step_batched(ctxs, [0.0] * 3, us2)
    hps.ark_step(hps.ark_create(op4, t4, dt, g=workloads.AllenCahn.gpoly), 0.0, want[0])
    for b in (1, 2):
        hps.ark_step(hps.ark_create(probs[b][6], probs[b][0], dt, g=workloads.AllenCahn.gpoly), 0.0, want[b])
    torch.cuda.synchronize()
    for b in range(3):
        assert torch.equal(us2[b], want[b]), b


ORACLE_FULL_STEP = """
import sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle.ark import ARK, ark548l2sa, tableau_float
from oracle.grid import Grid
from oracle.hps import HPS
from paper_2306_02526_amd import workloads
d = np.load(sys.argv[2])
og = Grid(0, 1, 0, 1, 64, 64, 16)
co = {k: d[k] for k in ("cxx", "cyy", "cx", "cy", "c0")}
t0 = time.perf_counter()
ark = ARK(HPS(og, co, float(d["gdt"])), co, tableau_float(ark548l2sa()), float(d["dt"]), workloads.AllenCahn.gpoly)
print(f"   oracle built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
np.save(sys.argv[3], ark.step(d["u0"]))
print(f"   oracle step done after {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
"""


def test_ark5_full_size_step_matches_oracle(torch, tmp_path):
    """64x64 leaves, p = 16 (the benchmark grid), one ARK5 step of Allen-Cahn element by
    element against the oracle run in a child process on one BLAS thread."""
    say("[ark5 full size] Allen-Cahn 64x64 p=16, one step")
    dt = 1e-3
    tab = product_tableau()
    gdt = tab["gamma"] * dt
    g = hps.make_grid(0, 1, 0, 1, 64, 64, 16)
    n_int = hps.hps_num_nodes(g)[1]
    x, y = hps.hps_nodes(g)
    co = allen_cahn_coefs(x[:n_int], y[:n_int])
    op = hps.hps_build(g, {k: torch.tensor(v, device="cuda") for k, v in co.items()}, gdt)
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    u0 = workloads.AllenCahn(workloads.rng_for(2)).u0(x, y)
    ug = torch.tensor(u0, device="cuda")
    hps.ark_step(ctx, 0.0, ug)
    u_gpu = ug.cpu().numpy()
    say("   GPU step done; oracle in a child process")
    inp, outp = tmp_path / "in.npz", tmp_path / "out.npy"
    np.savez(inp, u0=u0, gdt=gdt, dt=dt, **co)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, OPENBLAS_NUM_THREADS="1", OMP_NUM_THREADS="1", MKL_NUM_THREADS="1")
    subprocess.run([sys.executable, "-c", ORACLE_FULL_STEP, root, str(inp), str(outp)], env=env, check=True,
                   timeout=900)
    e = rel(u_gpu, np.load(outp))
    say(f"   rel err {e:.2e}")
    assert e <= TOL_FULL
