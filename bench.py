"""Benchmark of the RKHPS per-stage HPS solve on one MI355X.

Workload (default): variable-coefficient Allen-Cahn u_t = div(a grad u) + u - u^3 on
[0,1]^2, a = 1 + 0.5 sin(2 pi x) cos(2 pi y), 64 x 64 leaves, p = 16 (N = 919,296
corner-free nodes, 1,048,576 = p^2 n1 n2 with corners), dt = 1e-3, ARK4(3)6L[2]SA,
seeded sine-mode initial data, homogeneous Dirichlet data.  One bench step is one ARK
step = 5 implicit stage solves (each with its fused stage right-hand side, L u_i and
F_i) plus the step completion.  `value` = stage-solves/s in FP64 with everything
resident in HBM; the operator build is timed separately.

Also reported: the same steps with FP32 operators + FP64 iterative refinement, single
stage-solve latency percentiles, the roofline of the dominant kernel (the leaf
particular solve, measured with HIP events on its launch stream) and the CPU oracle
timed on a bounded sample on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def leaf_kernel_hash():
    """sha256 of the sources the fused per-leaf kernel is compiled from; stored counter
    traffic is only reported while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("hps_leaf_kernels.hip", "hps_device.h"):
        with open(os.path.join(ROOT, "paper_2306_02526_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="leaves per side")
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--fp32-steps", type=int, default=10)
    ap.add_argument("--latency-samples", type=int, default=100)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-slope", action="store_true")
    ap.add_argument("--slope-steps", type=int, default=10)
    ap.add_argument("--no-burgers", action="store_true")
    ap.add_argument("--burgers-steps", type=int, default=10)
    ap.add_argument("--no-heat", action="store_true")
    ap.add_argument("--no-nls", action="store_true")
    ap.add_argument("--nls-steps", type=int, default=10)
    ap.add_argument("--heat-steps", type=int, default=20)
    ap.add_argument("--no-ark5", action="store_true")
    ap.add_argument("--ark5-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config1", action="store_true", help="skip the 4x4 p=8 heat latency leg")
    ap.add_argument("--no-batched-leg", action="store_true", help="skip the reduced batched-mix leg")
    ap.add_argument("--batch-problems", type=int, default=24, help="problems of the batched leg")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-serving-leg", action="store_true", help="skip the short serving leg")
    ap.add_argument("--cpu-stage-solves", type=int, default=3)
    ap.add_argument("--workload", default="allen_cahn", choices=["allen_cahn", "batched", "serving"],
                    help="allen_cahn: the single-problem benchmark (default); batched: 256 seeded "
                         "problems stepped together; serving: Poisson job arrivals on the server")
    ap.add_argument("--problems", type=int, default=256, help="batched: number of problems")
    ap.add_argument("--level-tiles", default="auto", choices=["auto", "wide", "thin"],
                    help="level operators in few large row tiles (HPS_WIDE_TILES) or thin ones; "
                         "auto: thin for one problem, wide for the batched and serving workloads")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    ap.add_argument("--window", type=float, default=1.0, help="serving: seconds of arrivals at --rate")
    ap.add_argument("--normal-exit", action="store_true",
                    help="end through the interpreter's normal teardown (profilers write their "
                         "results then)")
    ap.add_argument("--counter-run", action="store_true",
                    help="short run for hardware-counter passes: build, 2 steps, then a plain "
                         "1 GiB device copy whose counters calibrate the byte counts")
    ap.add_argument("--build-runs", type=int, default=0,
                    help="only build the benchmark operator (FP64) this many times and print the "
                         "wall time of each build")
    return ap.parse_args()


def build_run(args):
    """Operator builds alone: the benchmark grid's FP64 operator built --build-runs times
    (the first includes one-time set-up), each timed from a synchronized start to a
    synchronized end."""
    import torch

    from paper_2306_02526_amd import hps, workloads
    from paper_2306_02526_amd.tableau import ark436l2sa

    dev = torch.device("cuda:0")
    n, p, dt = args.n, args.p, args.dt
    g = hps.make_grid(0.0, 1.0, 0.0, 1.0, n, n, p)
    N, n_int, _, _ = hps.hps_num_nodes(g)
    x, y = hps.hps_nodes(g)
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, _ = wl.L_coeffs(x[:n_int], y[:n_int])
    coefs = {k: torch.tensor(v, device=dev) for k, v in dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy).items()}
    times = []
    for _ in range(args.build_runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = hps.hps_build(g, coefs, ark436l2sa()["gamma"] * dt, hps.HPS_FP64)
        torch.cuda.synchronize()
        times.append(round(time.perf_counter() - t0, 4))
        log(f"build {n}x{n} p={p}: {times[-1]:.4f} s")
        op.free()
    print(json.dumps({"workload": f"operator_build_{n}x{n}_leaves_p{p}", "build_s": times}), flush=True)


def counter_run(args):
    """Build, two FP64 steps and a plain 1 GiB device-to-device copy (the copy's
    FETCH_SIZE / WRITE_SIZE per byte moved calibrates the counters)."""
    import torch

    from paper_2306_02526_amd import hps, workloads
    from paper_2306_02526_amd.tableau import ark436l2sa

    dev = torch.device("cuda:0")
    n, p, dt = args.n, args.p, args.dt
    tab = ark436l2sa()
    g = hps.make_grid(0.0, 1.0, 0.0, 1.0, n, n, p)
    N, n_int, _, _ = hps.hps_num_nodes(g)
    x, y = hps.hps_nodes(g)
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, _ = wl.L_coeffs(x[:n_int], y[:n_int])
    coefs = {k: torch.tensor(v, device=dev) for k, v in dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy).items()}
    op = hps.hps_build(g, coefs, tab["gamma"] * dt, hps.HPS_FP64)
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    u = torch.tensor(wl.u0(x, y), device=dev)
    for k in range(2):
        hps.ark_step(ctx, k * dt, u)
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("counter run done: 2 steps, 1 GiB copy")


def leaf_down_up_algorithmic_bytes(n_leaves, q, stages, elem_bytes):
    """Algorithmic HBM bytes per launch of the fused per-leaf kernel that closes stage i
    and opens stage i+1 (i = 2..s-1), averaged over those launches:
      operators  S_leaf (q^2 x 4q) and A_ii^{-1} (q^2 x q^2), elem_bytes each;
      reads      u_b (4q), w (q^2), the 5 coefficients of L (5 q^2), u^n (q^2) and the
                 2 (i-1) stage vectors L u_j, F_j, j < i, read from HBM (q^2 each);
      writes     L u_i, F_i (2 q^2), w (q^2), h (4q);  all field data FP64."""
    q2 = q * q
    launches = list(range(2, stages))            # closes stage i, opens i + 1
    field_reads = [4 * q + q2 + 5 * q2 + q2 + 2 * (i - 1) * q2 for i in launches]
    field = sum(field_reads) / len(field_reads) + 2 * q2 + q2 + 4 * q
    per_leaf = (q2 * 4 * q + q2 * q2) * elem_bytes + field * 8
    return n_leaves * per_leaf


def leaf2_down_up_algorithmic_bytes(n_leaves, q, stages, elem_bytes):
    """The same for the two-component leaf kernel: the operators and the 5 coefficients of
    L are read once, every field vector of the list above once per component."""
    q2 = q * q
    launches = list(range(2, stages))
    comp = [4 * q + q2 + q2 + 2 * (i - 1) * q2 + 2 * q2 + q2 + 4 * q for i in launches]
    field = 5 * q2 + 2 * sum(comp) / len(comp)
    return n_leaves * ((q2 * 4 * q + q2 * q2) * elem_bytes + field * 8)


def burgers_leg(args, torch, hps, workloads, g, x, y, n_int, tab, tiles, dev, uniform=True, profile=True):
    """Two-dimensional Burgers system (traveling-wave closed form, eps = 0.1, dt = 1e-3,
    boundary data from the closed form) on the bench grid: ark_step_burgers, which solves
    both components in every stage, 2 (s - 1) stage solves per step.  uniform: build with
    HPS_UNIFORM_COEFFS (L = eps Lap has constant coefficients: one stored copy of every
    leaf and level operator)."""
    import numpy as np
    sol = workloads.BurgersTravelingWave(0.1)
    dt = 1e-3
    co = dict(zip(("cxx", "cyy", "cx", "cy", "c0"), workloads.burgers_coeffs(sol.eps, n_int)))
    op = hps.hps_build(g, {k: torch.tensor(v, device=dev) for k, v in co.items()}, tab["gamma"] * dt,
                       hps.HPS_FP64 | tiles | (hps.HPS_UNIFORM_COEFFS if uniform else 0))
    wide = bool(tiles & hps.HPS_WIDE_TILES)
    _, op_bytes = op.bytes()
    cu, cv = hps.ark_create(op, tab, dt), hps.ark_create(op, tab, dt)
    N = len(x)
    x0, x1, y0, y1 = g.x0, g.x1, g.y0, g.y1
    on = lambda a, b: np.abs(a - b) < 1e-13
    bd = np.nonzero((np.arange(N) >= n_int) & (on(x, x0) | on(x, x1) | on(y, y0) | on(y, y1)))[0]
    assert len(bd) == op.n_bdry
    nsteps = args.warmup + args.burgers_steps + 4
    # boundary data of every step, resident on the GPU; copied into fixed arrays per step
    ts = [[k * dt + c * dt for c in tab["c"]] + [(k + 1) * dt] for k in range(nsteps)]
    ex = [[sol.exact(t, x[bd], y[bd]) for t in row] for row in ts]
    all_fu = torch.tensor(np.array([[e[0] for e in row] for row in ex]), device=dev)
    all_fv = torch.tensor(np.array([[e[1] for e in row] for row in ex]), device=dev)
    fu, fv = all_fu[0].clone(), all_fv[0].clone()
    u0, v0 = sol.exact(0.0, x, y)
    u, v = torch.tensor(u0, device=dev), torch.tensor(v0, device=dev)

    def step(k):
        fu.copy_(all_fu[k])
        fv.copy_(all_fv[k])
        hps.ark_step_burgers(cu, cv, k * dt, u, v, fu, fv)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.burgers_steps):
        step(k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k_end = args.warmup + args.burgers_steps
    ue, ve = sol.exact(k_end * dt, x, y)
    err = max(float(np.abs(u.cpu().numpy() - ue).max()), float(np.abs(v.cpu().numpy() - ve).max()))
    stages = tab["s"] - 1
    out = {"stage_solves_per_s": round(2 * stages * args.burgers_steps / el, 1),
           "ms_per_step": round(1e3 * el / args.burgers_steps, 3), "steps": args.burgers_steps,
           "components": 2, "eps": sol.eps, "dt": dt, "level_tiles": "wide" if wide else "thin",
           "operators": "one shared copy (uniform coefficients)" if uniform else "per node",
           "operator_bytes": op_bytes, "max_err_vs_closed_form": err}
    if not profile:
        op.free()
        return out
    # per-kernel durations (eager steps, HIP events on the launch stream)
    hps.hps_profile_enable(op, True)
    for k in range(k_end, k_end + 4):
        step(k)
    torch.cuda.synchronize()
    prof = hps.hps_profile_read(op)
    hps.hps_profile_enable(op, False)
    kern = {k: {"launches_per_step": v[0] // 4, "us_per_launch": round(1e3 * v[1] / v[0], 2)} for k, v in prof.items()}
    leaf_us = 1e3 * prof["leaf2_down_up_fp64"][1] / prof["leaf2_down_up_fp64"][0]
    out["kernels"] = kern
    out["leaf2_down_up_us_per_launch"] = round(leaf_us, 2)
    if not uniform:
        # every leaf's operators streamed from HBM: bytes as for the scalar kernel
        alg = leaf2_down_up_algorithmic_bytes(g.n1 * g.n2, g.p - 2, tab["s"], 8)
        out["leaf2_down_up"] = {"algorithmic_bytes_per_launch": int(alg),
                                "achieved_GBps": round(alg / (leaf_us * 1e-6) / 1e9, 1)}
    op.free()
    return out


def heat_leg(args, torch, hps, workloads, g, x, y, n_int, tab, dev, uniform):
    """The 2-D heat test (u_t = Lap u + q, manufactured solution, f = 0) on the bench grid:
    the scalar stage formulation with a separable source; uniform: one shared operator copy
    (L = Lap has constant coefficients)."""
    import numpy as np
    wl = workloads.HeatManufactured(workloads.rng_for(1))
    dt = 1e-3
    one = torch.ones(n_int, dtype=torch.float64, device=dev)
    op = hps.hps_build(g, {"cxx": one, "cyy": one}, tab["gamma"] * dt,
                       hps.HPS_FP64 | (hps.HPS_UNIFORM_COEFFS if uniform else 0))
    _, op_bytes = op.bytes()
    ctx = hps.ark_create(op, tab, dt)
    u = torch.tensor(wl.exact(0.0, x, y), device=dev)
    qs = torch.tensor(wl.q_space(x[:n_int], y[:n_int]), device=dev)

    def step(k):
        t = k * dt
        hps.ark_step(ctx, t, u, q_space=qs, q_time=[wl.q_time(t + c * dt) for c in tab["c"]])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.heat_steps):
        step(k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k_end = args.warmup + args.heat_steps
    err = float(np.abs(u.cpu().numpy() - wl.exact(k_end * dt, x, y)).max())
    hps.hps_profile_enable(op, True)
    for k in range(k_end, k_end + 2):
        step(k)
    torch.cuda.synchronize()
    prof = hps.hps_profile_read(op)
    hps.hps_profile_enable(op, False)
    op.free()
    stages = tab["s"] - 1
    return {"stage_solves_per_s": round(stages * args.heat_steps / el, 1),
            "ms_per_step": round(1e3 * el / args.heat_steps, 3), "steps": args.heat_steps, "dt": dt,
            "operators": "one shared copy (uniform coefficients)" if uniform else "per node",
            "operator_bytes": op_bytes, "max_err_vs_exact": err,
            "leaf_down_up_us_per_launch": round(1e3 * prof["leaf_down_up_fp64"][1] / prof["leaf_down_up_fp64"][0], 2)}


def nls_leg(args, torch, hps, workloads, n, p, tab, dev, uniform, steps, tiles=0):
    """The regularised NLS filamentation problem (Sec. 5.5: [0, 25.6]^2, u0 = 5 exp(-r^2),
    zero boundary data, dt = 0.005) on n x n leaves of order p: complex operators (real
    embedding), ark_step with the NLS nonlinearity; 5 complex stage solves per step."""
    import numpy as np
    nls = workloads.NLSFilamentation()
    dt = 0.005
    g = hps.make_grid(*nls.domain, n, n, p)
    N, n_int, _, _ = hps.hps_num_nodes(g)
    x, y = hps.hps_nodes(g)
    re, im = nls.coeffs(n_int)
    t0 = time.perf_counter()
    op = hps.hps_build_complex(g, {k: torch.tensor(v, device=dev) for k, v in re.items()},
                               {k: torch.tensor(v, device=dev) for k, v in im.items()}, tab["gamma"] * dt,
                               hps.HPS_FP64 | tiles | (hps.HPS_UNIFORM_COEFFS if uniform else 0))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    _, op_bytes = op.bytes()
    ctx = hps.ark_create(op, tab, dt, g=nls.g())
    u0 = nls.u0(x, y)
    u = torch.tensor(np.stack([u0.real, u0.imag]), device=dev).contiguous()
    for k in range(args.warmup):
        hps.ark_step(ctx, k * dt, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + steps):
        hps.ark_step(ctx, k * dt, u)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hps.hps_profile_enable(op, True)
    for k in range(2):
        hps.ark_step(ctx, (args.warmup + steps + k) * dt, u)
    torch.cuda.synchronize()
    prof = hps.hps_profile_read(op)
    hps.hps_profile_enable(op, False)
    finite = bool(torch.isfinite(u).all())
    mass = float((u[0] ** 2 + u[1] ** 2).max().sqrt())
    op.free()
    stages = tab["s"] - 1
    out = {"grid": f"{n}x{n}_p{p}", "level_tiles": "wide" if tiles else "thin",
           "stage_solves_per_s": round(stages * steps / el, 1),
           "ms_per_step": round(1e3 * el / steps, 3), "steps": steps, "dt": dt, "build_s": round(build_s, 2),
           "operators": "one shared copy (uniform coefficients)" if uniform else "per node",
           "operator_bytes": op_bytes, "max_abs_u": mass, "finite": finite,
           "kernels": {k: {"launches_per_step": v[0] // 2, "us_per_launch": round(1e3 * v[1] / v[0], 2)}
                       for k, v in prof.items()}}
    return out


def ark5_leg(args, torch, hps, workloads, g, x, y, n_int, coefs, u0, dt, tiles, dev):
    """The headline Allen-Cahn workload stepped with the fifth-order pair ARK5(4)8L[2]SA
    (Sec. 3): its own operator (gamma = 41/200), 7 stage solves per step."""
    from paper_2306_02526_amd.tableau import ark548l2sa
    tab = ark548l2sa()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = hps.hps_build(g, coefs, tab["gamma"] * dt, hps.HPS_FP64 | tiles)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
    u = u0.clone()
    for k in range(args.warmup):
        hps.ark_step(ctx, k * dt, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.ark5_steps):
        hps.ark_step(ctx, (args.warmup + k) * dt, u)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hps.hps_profile_enable(op, True)
    for k in range(2):
        hps.ark_step(ctx, k * dt, u)
    torch.cuda.synchronize()
    prof = hps.hps_profile_read(op)
    hps.hps_profile_enable(op, False)
    finite = bool(torch.isfinite(u).all())
    op.free()
    stages = tab["s"] - 1
    return {"tableau": "ARK5(4)8L[2]SA", "stage_solves_per_step": stages,
            "stage_solves_per_s": round(stages * args.ark5_steps / el, 1),
            "ms_per_step": round(1e3 * el / args.ark5_steps, 3), "steps": args.ark5_steps, "dt": dt,
            "build_s": round(build_s, 3), "finite": finite,
            "kernels": {k: {"launches_per_step": v[0] // 2, "us_per_launch": round(1e3 * v[1] / v[0], 2)}
                        for k, v in prof.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.counter_run:
        counter_run(args)
        return
    if args.build_runs > 0:
        build_run(args)
        return
    if args.workload == "batched":
        batched_run(args)
        return
    if args.workload == "serving":
        serving_run(args)
        return
    import numpy as np
    import torch

    from paper_2306_02526_amd import hps, workloads
    from paper_2306_02526_amd.tableau import ark436l2sa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n, p, dt = args.n, args.p, args.dt
    q = p - 2
    tab = ark436l2sa()
    gdt = tab["gamma"] * dt
    g = hps.make_grid(0.0, 1.0, 0.0, 1.0, n, n, p)
    N, n_int, n_iface, n_bdry = hps.hps_num_nodes(g)
    x, y = hps.hps_nodes(g)
    wl = workloads.AllenCahn(workloads.rng_for(2))
    cxx, cyy, cx, cy, c0 = wl.L_coeffs(x[:n_int], y[:n_int])
    coefs = {k: torch.tensor(v, device=dev) for k, v in dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy).items()}
    u0 = torch.tensor(wl.u0(x, y), device=dev)
    stages = tab["s"] - 1

    # ---- build (FP64) ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tiles = hps.HPS_WIDE_TILES if args.level_tiles == "wide" else 0
    op = hps.hps_build(g, coefs, gdt, hps.HPS_FP64 | tiles)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    total_bytes, op_bytes = op.bytes()
    log(f"build FP64: {build_s:.3f} s, operators {op_bytes / 1e9:.3f} GB")
    # the method's own operator bytes (one operator per tree level): what the roofline
    # counts; the composite level pairs the default sweeps stream instead are larger
    prev = os.environ.get("HPS_COMPOSE")
    os.environ["HPS_COMPOSE"] = "0"
    op_lv = hps.hps_build(g, coefs, gdt, hps.HPS_FP64 | tiles)
    per_level_op_bytes = op_lv.bytes()[1]
    op_lv.free()
    if prev is None:
        del os.environ["HPS_COMPOSE"]
    else:
        os.environ["HPS_COMPOSE"] = prev
    ctx = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)

    u = u0.clone()
    for k in range(args.warmup):
        hps.ark_step(ctx, k * dt, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        hps.ark_step(ctx, (args.warmup + k) * dt, u)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = stages * args.steps / elapsed
    log(f"FP64: {ms_per_step:.3f} ms/step, {value:.1f} stage-solves/s")
    assert torch.isfinite(u).all()

    # ---- per-kernel timing (HIP events on the launch stream), outside the timed region ----
    hps.hps_profile_enable(op, True)
    prof_steps = 4
    for k in range(prof_steps):
        hps.ark_step(ctx, k * dt, u)
    torch.cuda.synchronize()
    prof = hps.hps_profile_read(op)
    hps.hps_profile_enable(op, False)
    launches, tot_ms = prof["leaf_down_up_fp64"]
    leaf_us = 1e3 * tot_ms / launches
    alg = leaf_down_up_algorithmic_bytes(n * n, q, tab["s"], 8)
    achieved = alg / (leaf_us * 1e-6) / 1e9
    breakdown = {k: {"launches_per_step": v[0] // prof_steps, "us_per_launch": round(1e3 * v[1] / v[0], 2)}
                 for k, v in prof.items()}
    log(f"leaf_down_up_fp64: {leaf_us:.1f} us/launch, {achieved:.0f} GB/s; kernels: {breakdown}")
    # the level sweeps of one stage solve: the operator bytes outside the leaf panels (A_ii^-1
    # and S_leaf, q2 x q2 and q2 x 4q per leaf) over the up and down sweep times
    level_bytes = op.bytes()[1] - n * n * (q * q * q * q + q * q * 4 * q) * 8
    level_fams = ("level_up_fp64", "level_down_fp64", "pair_up_fp64", "pair_top_fp64", "pair_down_fp64")
    level_us = sum(1e3 * prof[k][1] / prof[k][0] for k in level_fams if k in prof)
    n_levels = int(math.log2(n * n))
    composed = "pair_top_fp64" in prof
    levels = {"bytes_per_stage": int(level_bytes), "us_per_stage": round(level_us, 2),
              "achieved_GBps": round(level_bytes / (level_us * 1e-6) / 1e9, 1),
              "frac": round(level_bytes / (level_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
              "launches_per_stage": (2 * (n_levels // 2 - 1) + 1 + 2 * (n_levels % 2)) if composed
              else 2 * (n_levels - 1) + 1,
              "composite_level_pairs": composed,
              "note": "latency-bound: one dependent launch per tree level (level pair, if composed) and direction"}
    traffic = None
    tr_path = os.path.join(ROOT, "profiles", "leaf_down_up_fp64_traffic.json")
    if os.path.exists(tr_path):
        try:
            tr = json.load(open(tr_path))
            if tr.get("workload") == f"allen_cahn_n{n}_p{p}" and tr.get("kernel_hash") == leaf_kernel_hash():
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    stage_solve_bytes = op_bytes   # operator bytes streamed by one stage solve
    # the whole stage solve against the HBM roofline: every stored operator once (leaf
    # A_ii^-1 and S_leaf, every level's [X; U] and S) plus the field traffic of the fused
    # leaf kernel that closes one stage and opens the next (averaged over stages 2..s-1);
    # the time is the measured step time over its stage solves (the step completion's
    # interface lines and stage 1's evaluation included)
    leaf_op_bytes = n * n * (q ** 4 + q * q * 4 * q) * 8
    # algorithmic bytes: the per-level operators (not the larger composites) plus fields
    stage_bytes = per_level_op_bytes + (alg - leaf_op_bytes)
    stage_us = 1e3 * ms_per_step / stages
    stage_roof = {"bound": "hbm", "bytes_per_stage_solve": int(stage_bytes), "us_per_stage_solve": round(stage_us, 2),
                  "achieved": round(stage_bytes / (stage_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(stage_bytes / (stage_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                  "stage_solves_per_s_at_0.6_peak": round(0.6 * HBM_PEAK_GBS * 1e9 / stage_bytes, 1),
                  "bytes_counted": "the method's per-level operators (leaf A_ii^-1 and S_leaf, every level's [X; U] "
                                   "and S) once, plus the fused leaf kernel's field traffic",
                  "operator_bytes_streamed": int(op_bytes),
                  "note": "the default sweeps stream composite level-pair operators instead of the per-level ones "
                          "(operator_bytes_streamed); without Dirichlet data the top pair skips its boundary columns"}
    log(f"stage solve: {stage_roof}")

    # ---- single stage-solve latency (hps_solve: one full up/down sweep) ----
    body = torch.randn(n_int, dtype=torch.float64, device=dev)
    uo = torch.empty(N, dtype=torch.float64, device=dev)
    for _ in range(5):
        hps.hps_solve(op, body, u=uo)
    lat = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.latency_samples)]
    for a, b in ev:
        a.record(stream)
        hps.hps_solve(op, body, u=uo)
        b.record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    log(f"hps_solve latency: p50 {p50:.3f} ms, p99 {p99:.3f} ms")

    # ---- several right-hand sides per solve: one leaf launch and one level sweep for all ----
    multi = {}
    for nrhs in (1, 2, 4, 8):
        bm = torch.randn(nrhs, n_int, dtype=torch.float64, device=dev)
        um = torch.empty(nrhs, N, dtype=torch.float64, device=dev)
        for _ in range(3):
            hps.hps_solve(op, bm, u=um)
        evm = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for a, b in evm:
            a.record(stream)
            hps.hps_solve(op, bm, u=um)
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evm]))
        multi[str(nrhs)] = {"ms_per_solve_call": round(ms, 4), "rhs_per_s": round(nrhs / (ms * 1e-3), 1)}
        # where the time goes (HIP events per kernel family, one call, outside the timing)
        hps.hps_profile_enable(op, True)
        hps.hps_profile_read(op)
        hps.hps_solve(op, bm, u=um)
        torch.cuda.synchronize()
        multi[str(nrhs)]["us_per_family"] = {k: round(1e3 * v[1], 1) for k, v in hps.hps_profile_read(op).items()}
        hps.hps_profile_enable(op, False)
    for k in multi:
        multi[k]["time_vs_one_rhs"] = round(multi[k]["ms_per_solve_call"] / multi["1"]["ms_per_solve_call"], 3)
    log(f"multi-rhs hps_solve: {multi}")

    # ---- slope formulation with flux-jump penalisation, same operator and start ----
    slope = None
    if not args.no_slope:
        ctxs = hps.ark_create(op, tab, dt, g=workloads.AllenCahn.gpoly)
        us = u0.clone()
        hps.ark_step_slope(ctxs, 0.0, us)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, args.slope_steps + 1):
            hps.ark_step_slope(ctxs, k * dt, us)
        torch.cuda.synchronize()
        els = time.perf_counter() - t0
        ust = u0.clone()
        for k in range(args.slope_steps + 1):
            hps.ark_step(ctx, k * dt, ust)
        torch.cuda.synchronize()
        slope = {"stage_solves_per_s": round(stages * args.slope_steps / els, 1),
                 "ms_per_step": round(1e3 * els / args.slope_steps, 3), "steps": args.slope_steps + 1,
                 "rel_diff_vs_stage_formulation": float((us - ust).abs().max() / ust.abs().max())}
        log(f"slope formulation: {slope}")
        del ctxs

    # ---- two-component Burgers system on the same grid ----
    burgers = None
    if not args.no_burgers:
        # two right-hand sides per level product; thin tiles (composite level pairs) unless wide
        # ones are asked for: measured 5886 against 5008 stage-solves/s with shared operators
        btiles = hps.HPS_WIDE_TILES if args.level_tiles == "wide" else 0
        burgers = burgers_leg(args, torch, hps, workloads, g, x, y, n_int, tab, btiles, dev)
        burgers["per_node_operators"] = burgers_leg(args, torch, hps, workloads, g, x, y, n_int, tab, btiles, dev,
                                                    uniform=False)
        log(f"burgers: {burgers}")

    # ---- the heat test (constant coefficients) on the same grid ----
    heat = None
    if not args.no_heat:
        heat = heat_leg(args, torch, hps, workloads, g, x, y, n_int, tab, dev, uniform=True)
        heat["per_node_operators"] = heat_leg(args, torch, hps, workloads, g, x, y, n_int, tab, dev, uniform=False)
        log(f"heat: {heat}")

    # ---- the regularised NLS (complex operators): bench grid and the paper's grid ----
    nls = None
    if not args.no_nls:
        nls = nls_leg(args, torch, hps, workloads, n, p, tab, dev, uniform=True, steps=args.nls_steps)
        nls["per_node_operators"] = nls_leg(args, torch, hps, workloads, n, p, tab, dev, uniform=False,
                                            steps=args.nls_steps)
        nls["filamentation_8x8_p13"] = nls_leg(args, torch, hps, workloads, 8, 13, tab, dev, uniform=True,
                                               steps=args.nls_steps)
        log(f"nls: {nls}")

    # ---- the fifth-order pair on the headline workload ----
    ark5 = None
    if not args.no_ark5:
        ark5 = ark5_leg(args, torch, hps, workloads, g, x, y, n_int, coefs, u0, dt, tiles, dev)
        log(f"ark5: {ark5}")

    # ---- FP32 operators + FP64 iterative refinement, same steps ----
    fp32 = None
    if not args.no_fp32:
        del ctx
        op.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op32 = hps.hps_build(g, coefs, gdt, hps.HPS_FP32_IR | tiles)
        torch.cuda.synchronize()
        b32 = time.perf_counter() - t0
        ctx32 = hps.ark_create(op32, tab, dt, g=workloads.AllenCahn.gpoly)
        op64 = hps.hps_build(g, coefs, gdt, hps.HPS_FP64 | tiles)
        ctx64 = hps.ark_create(op64, tab, dt, g=workloads.AllenCahn.gpoly)
        u32 = u0.clone()
        u64 = u0.clone()
        hps.ark_step(ctx32, 0.0, u32)
        hps.ark_step(ctx64, 0.0, u64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs = []
        for k in range(1, args.fp32_steps + 1):
            hps.ark_step(ctx32, k * dt, u32)
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t0
        for k in range(1, args.fp32_steps + 1):
            hps.ark_step(ctx64, k * dt, u64)
        torch.cuda.synchronize()
        rel32 = float((u32 - u64).abs().max() / u64.abs().max())
        # where an FP32+IR step's time goes (HIP events per kernel family; the profiled
        # steps run eagerly, outside the timing)
        hps.hps_profile_enable(op32, True)
        hps.hps_profile_read(op32)
        for k in range(2):
            hps.ark_step(ctx32, (args.fp32_steps + 1 + k) * dt, u32.clone())
        torch.cuda.synchronize()
        kern32 = {k: round(1e3 * v[1] / 2, 1) for k, v in hps.hps_profile_read(op32).items()}
        hps.hps_profile_enable(op32, False)
        fp32 = {"stage_solves_per_s": round(stages * args.fp32_steps / el32, 1),
                "ms_per_step": round(1e3 * el32 / args.fp32_steps, 3),
                "rel_err_vs_fp64_after_steps": rel32, "steps": args.fp32_steps + 1,
                "build_s": round(b32, 3), "refinement_last_step": hps.ark_info(ctx32),
                "us_per_step_by_family": kern32,
                "note": "first step host-checked, later steps replayed from a HIP graph with a fixed "
                        "number of corrections per stage and one stream wait per step"}
        log(f"FP32+IR: {fp32}")
        # the accuracy the refined FP32 path is held to
        assert rel32 <= 1e-10, f"FP32+IR differs from FP64 by {rel32:.3e} > 1e-10"
        del ctx32, ctx64
        op32.free()
        op64.free()

    # ---- the small heat configuration: per-step latency ----
    config1 = None
    if not args.no_config1:
        config1 = config1_leg(torch, hps, workloads, dev)
        log(f"config 1 (heat 4x4 p=8): {config1}")

    # ---- a reduced batched mix, FP64 (grouped launches) and FP32+IR ----
    batched = None
    if not args.no_batched_leg:
        batched = {"recipe": f"the first {args.batch_problems} problems of the seeded 256-problem mix "
                             "(leaves per side 8..64, p 8/12/16, gamma dt 1e-3/1e-2, heat or Allen-Cahn), "
                             f"{args.batch_steps} timed steps after 1 warm-up step"}
        batched["fp64"] = batched_measure(torch, hps, workloads, dev, args.batch_problems, args.batch_steps, 1,
                                          hps.HPS_FP64 | hps.HPS_WIDE_TILES, sequential=False)
        log(f"batched FP64: {batched['fp64']}")
        batched["fp32_ir"] = batched_measure(torch, hps, workloads, dev, args.batch_problems, args.batch_steps, 1,
                                             hps.HPS_FP32_IR | hps.HPS_WIDE_TILES, sequential=False)
        log(f"batched FP32+IR: {batched['fp32_ir']}")

    # ---- a short serving run ----
    serving = None
    if not args.no_serving_leg:
        serving = serving_measure(torch, hps, workloads, dev, burst=16, low_window=3.0, rate=200.0,
                                  rate_window=0.5)
        log(f"serving: {serving}")

    # ---- CPU oracle on a bounded sample of the same workload ----
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu oracle: one BLAS thread")
        cpu = cpu_baseline(n, p, dt, args.cpu_stage_solves, threads=1, limit_s=240)
        log(f"cpu oracle: {cpu}")
        # all host cores: one single-threaded oracle per core, all running the same sample at
        # once (threaded BLAS does not help the oracle's many small dense operations: with
        # 16 threads it did not finish the sample within 90 s)
        nproc = min(os.cpu_count() or 1, 16)
        log(f"cpu oracle: {nproc} concurrent single-threaded processes")
        cpu["all_cores"] = cpu_baseline(n, p, dt, args.cpu_stage_solves, threads=1, limit_s=150, procs=nproc)
        log(f"cpu oracle, all cores: {cpu['all_cores']}")
        cpu["config1"] = config1_oracle()
        log(f"cpu oracle, config 1: {cpu['config1']}")

    out = {
        "metric": "stage-solves/s at N\u22481M (FP64 vs FP32+IR @1e-10 rel); p50/p99 solve latency",
        "value": round(value, 2),
        "unit": "stage-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"allen_cahn_variable_coef_{n}x{n}_leaves_p{p}", "n_leaves": n * n, "p": p,
                   "N_corner_free": N, "N_with_corners": p * p * n * n, "dt": dt,
                   "tableau": "ARK4(3)6L[2]SA", "stage_solves_per_step": stages,
                   "parallelism": "single GPU", "level_tiles": "wide" if tiles else "thin"},
        "unknowns_per_s": round(value * N, 1),
        "build_s": round(build_s, 4),
        "operator_bytes_per_stage_solve": int(stage_solve_bytes),
        "latency_ms": {"hps_solve_p50": round(p50, 4), "hps_solve_p99": round(p99, 4)},
        "multi_rhs_solve": multi,
        "kernels": breakdown,
        "roofline": {"bound": "hbm", "kernel": "k_leaf<double> (down stage i + up stage i+1)",
                     "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": int(alg),
                     "avg_launch_us": round(leaf_us, 2)},
        "stage_roofline": stage_roof,
        "level_sweeps": levels,
        "fp32_ir": fp32,
        "slope_formulation": slope,
        "burgers_system": burgers,
        "heat_constant_coefficients": heat,
        "nls_complex": nls,
        "ark5": ark5,
        "config1_heat_latency": config1,
        "batched_mix": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _mix_problem(torch, m, dev):
    """Device data of one problem of the batched recipe."""
    from paper_2306_02526_amd import hps, workloads
    from paper_2306_02526_amd.tableau import ark436l2sa
    tab = ark436l2sa()
    g = hps.make_grid(*m["domain"], m["n1"], m["n2"], m["p"])
    N, n_int, _, _ = hps.hps_num_nodes(g)
    x, y = hps.hps_nodes(g)
    pr = m["problem"]
    cxx, cyy, cx, cy, c0 = pr.L_coeffs(x[:n_int], y[:n_int])
    coefs = {k: torch.tensor(v, device=dev) for k, v in dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy).items()}
    heat = m["kind"] == "heat"
    u0 = torch.tensor(pr.exact(0.0, x, y) if heat else pr.u0(x, y), device=dev)
    qsp = torch.tensor(pr.q_space(x[:n_int], y[:n_int]), device=dev) if heat else None
    return dict(grid=g, coefs=coefs, u0=u0, q_space=qsp, heat=heat, tab=tab,
                dt=m["gamma_dt"] / tab["gamma"], gpoly=None if heat else workloads.AllenCahn.gpoly)


def batched_measure(torch, hps, workloads, dev, problems, steps, warmup, flags, sequential=True):
    """`problems` seeded problems of the batched recipe (leaves per side 8..64, p 8/12/16,
    gamma*dt 1e-3/1e-2, heat or Allen-Cahn), built with `flags`, then `steps` steps of every
    problem per ark_step_batched call (timed after `warmup` such calls)."""
    mix = workloads.batched_mix(n_problems=problems)
    probs, ctxs, us, ops = [], [], [], []
    op_bytes = 0
    t0 = time.perf_counter()
    for k, m in enumerate(mix):
        if k and k % 32 == 0:
            log(f"   {k}/{len(mix)} problems built")
        d = _mix_problem(torch, m, dev)
        op = hps.hps_build(d["grid"], d["coefs"], m["gamma_dt"], flags)
        op_bytes += op.bytes()[1]
        ops.append(op)
        ctxs.append(hps.ark_create(op, d["tab"], d["dt"], g=d["gpoly"]))
        us.append(d["u0"].clone())
        probs.append(d)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"batched: {len(mix)} problems built in {setup_s:.1f} s, operators {op_bytes / 1e9:.2f} GB")
    qsp = [d["q_space"] for d in probs]
    s = probs[0]["tab"]["s"]
    c = probs[0]["tab"]["c"]

    def step(k):
        ts = [k * d["dt"] for d in probs]
        qt = [[math.exp(-(t + ci * d["dt"])) for ci in c] if d["heat"] else None for d, t in zip(probs, ts)]
        hps.ark_step_batched(ctxs, ts, us, q_space=qsp, q_time=qt)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(warmup + k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ss = (s - 1) * len(probs) * steps
    out = {"stage_solves_per_s": round(ss / el, 1), "problem_steps_per_s": round(len(probs) * steps / el, 1),
           "ms_per_batch_step": round(1e3 * el / steps, 3), "problems": len(probs), "steps": steps,
           "precision": "FP32+IR" if flags & hps.HPS_FP32_IR else "FP64",
           "operator_GBps": round(op_bytes * (s - 1) * steps / el / 1e9, 1), "operator_bytes": op_bytes,
           "setup_s": round(setup_s, 1), "streams": hps.hps_batch_streams()}
    if flags & hps.HPS_FP32_IR:
        infos = [hps.ark_info(cx) for cx in ctxs]
        out["ir_corrections_per_stage_max"] = max(i["ir_iterations"] for i in infos)
        out["fp64_fallbacks"] = sum(i["fp64_fallbacks"] for i in infos)
    if sequential:
        # the same steps one problem at a time on one stream, for comparison
        t1 = time.perf_counter()
        for k in range(steps):
            for b, d in enumerate(probs):
                t = (warmup + steps + k) * d["dt"]
                qt = [math.exp(-(t + ci * d["dt"])) for ci in c] if d["heat"] else None
                hps.ark_step(ctxs[b], t, us[b], q_space=qsp[b], q_time=qt)
        torch.cuda.synchronize()
        out["one_stream_sequential_stage_solves_per_s"] = round(ss / (time.perf_counter() - t1), 1)
    out["finite"] = all(bool(torch.isfinite(u).all()) for u in us)
    del ctxs
    for op in ops:
        op.free()
    return out


def batched_run(args):
    """The batched workload on its own: args.problems problems, args.steps steps each.
    Prints one JSON line."""
    import torch

    from paper_2306_02526_amd import hps, workloads
    dev = torch.device("cuda:0")
    flags = hps.HPS_FP64 | (0 if args.level_tiles == "thin" else hps.HPS_WIDE_TILES)
    r = batched_measure(torch, hps, workloads, dev, args.problems, args.steps, args.warmup, flags)
    out = {"metric": "stage-solves/s, batched mix", "value": r["stage_solves_per_s"], "unit": "stage-solves/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_batch_step"],
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batched_mix_{args.problems}", "problems": args.problems,
                      "streams": r["streams"], "level_tiles": args.level_tiles}, **r}
    print(json.dumps(out), flush=True)


def serving_measure(torch, hps, workloads, dev, burst, low_window, rate, rate_window):
    """Serving: 16 seeded keys from the batched recipe; a burst of `burst` jobs (steps
    ~ U{50..500}, keys uniform) measures the saturation rate, then jobs arrive as a Poisson
    process at 0.8x that rate for `low_window` seconds and at `rate` per second for
    `rate_window` seconds.  Latency = completion - submission."""
    import numpy as np
    keys = [_mix_problem(torch, m, dev) for m in workloads.batched_mix(n_problems=16)]
    rng = workloads.rng_for(5, 1000)
    stream = torch.cuda.current_stream()
    srv = hps.Server(max_active=128)

    def submit(kidx, steps):
        d = keys[kidx]
        u = d["u0"].clone()
        extra = dict(q_space=d["q_space"], q_amp=1.0, q_rate=-1.0) if d["heat"] else {}
        return srv.submit(d["grid"], kidx, d["coefs"], d["tab"], d["dt"], u, steps, g=d["gpoly"],
                          stream=stream, **extra)

    def drain(ids):
        lat, fin = [], []
        for k, j in enumerate(ids):
            if k and k % 50 == 0:
                log(f"   {k}/{len(ids)} jobs finished")
            st = srv.wait(j)
            assert st["state"] == hps.SRV_DONE, st
            lat.append(st["finish_s"] - st["submit_s"])
            fin.append(st["finish_s"])
            srv.release(j)
        return np.array(lat), np.array(fin)

    # warm the operator cache with one short job per key
    drain([submit(k, 1) for k in range(len(keys))])
    t0 = time.perf_counter()
    ids = [submit(int(rng.integers(0, len(keys))), int(rng.integers(50, 501))) for _ in range(burst)]
    lat_b, _ = drain(ids)
    sat = burst / (time.perf_counter() - t0)
    log(f"serving: saturation {sat:.2f} jobs/s from a burst of {burst}")

    def poisson(rate, window):
        arr, t = [], 0.0
        while True:
            t += float(rng.exponential(1.0 / rate))
            if t > window:
                return arr
            arr.append((t, int(rng.integers(0, len(keys))), int(rng.integers(50, 501))))

    def run(rate, window):
        arr = poisson(rate, window)
        t0 = time.perf_counter()
        ids = []
        for t, k, n in arr:
            dly = t - (time.perf_counter() - t0)
            if dly > 0:
                time.sleep(dly)
            ids.append(submit(k, n))
        backlog = sum(1 for j in ids if srv.poll(j)["state"] == hps.SRV_QUEUED)
        lat, _ = drain(ids)
        span = time.perf_counter() - t0
        return {"rate": round(rate, 2), "window_s": window, "jobs": len(ids),
                "p50_s": round(float(np.percentile(lat, 50)), 3), "p99_s": round(float(np.percentile(lat, 99)), 3),
                "completed_per_s": round(len(ids) / span, 2), "queued_at_window_end": backlog,
                "stable": bool(backlog <= 2)}

    r_low = run(0.8 * sat, low_window)
    log(f"serving at 0.8x saturation: {r_low}")
    r_hi = run(rate, rate_window) if rate_window > 0 else None
    log(f"serving at {rate}/s: {r_hi}")
    st = srv.stats()
    srv.close()
    return {"saturation_jobs_per_s": round(sat, 2), "burst": burst,
            "burst_p50_s": round(float(np.percentile(lat_b, 50)), 3),
            "burst_p99_s": round(float(np.percentile(lat_b, 99)), 3), "keys": len(keys),
            "at_0.8x_saturation": r_low, "at_rate": r_hi, "server_stats": st}


def serving_run(args):
    """The serving workload on its own (burst of 48, 0.8x saturation for max(window, 5) s,
    then args.rate for args.window s).  Prints one JSON line."""
    import torch

    from paper_2306_02526_amd import hps, workloads
    dev = torch.device("cuda:0")
    r = serving_measure(torch, hps, workloads, dev, 48, max(args.window, 5.0), args.rate, args.window)
    out = {"metric": "jobs/s at saturation (served ARK integrations); p50/p99 latency",
           "value": r["saturation_jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "serving_16_keys_steps_50_500", "keys": r["keys"], "burst": r["burst"]}, **r}
    print(json.dumps(out), flush=True)


def config1_leg(torch, hps, workloads, dev, steps=100):
    """The small heat configuration: u_t = Lap u + q on [0,1]^2, 4 x 4 leaves, p = 8
    (N = 816; 0.40 MB of operators, latency-bound), manufactured solution with the seeded
    Fourier mix (separable source), f = 0, dt = 0.01, T = 1 (100 steps), FP64.  Per-step
    latency from HIP events around every ark_step on the stream, and the error against the
    closed form at T."""
    import numpy as np
    from paper_2306_02526_amd.tableau import ark436l2sa
    tab = ark436l2sa()
    dt = 0.01
    g = hps.make_grid(0.0, 1.0, 0.0, 1.0, 4, 4, 8)
    N, n_int, _, _ = hps.hps_num_nodes(g)
    x, y = hps.hps_nodes(g)
    wl = workloads.HeatManufactured(workloads.rng_for(1))
    one = torch.ones(n_int, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = hps.hps_build(g, {"cxx": one, "cyy": one}, tab["gamma"] * dt)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ctx = hps.ark_create(op, tab, dt)
    qs = torch.tensor(wl.q_space(x[:n_int], y[:n_int]), device=dev)
    u_init = torch.tensor(wl.exact(0.0, x, y), device=dev)
    u = u_init.clone()
    qt = lambda t: [wl.q_time(t + c * dt) for c in tab["c"]]
    hps.ark_step(ctx, 0.0, u, q_space=qs, q_time=qt(0.0))   # captures the step's graph for u
    u.copy_(u_init)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (a, b) in enumerate(ev):
        a.record(stream)
        hps.ark_step(ctx, k * dt, u, q_space=qs, q_time=qt(k * dt))
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    ex = wl.exact(steps * dt, x, y)
    err = float(np.abs(u.cpu().numpy() - ex).max())
    stages = tab["s"] - 1
    op_bytes = op.bytes()[1]
    del ctx
    op.free()
    return {"workload": "heat_manufactured_4x4_leaves_p8", "N": N, "dt": dt, "steps": steps, "T": steps * dt,
            "latency_ms_per_step": {"p50": round(float(np.percentile(lat, 50)), 4),
                                    "p99": round(float(np.percentile(lat, 99)), 4),
                                    "mean": round(float(lat.mean()), 4)},
            "steps_per_s_wall": round(steps / wall, 1), "stage_solves_per_s_wall": round(stages * steps / wall, 1),
            "max_err_vs_exact_at_T": err, "rel_err_vs_exact_at_T": err / float(np.abs(ex).max()),
            "build_s": round(build_s, 4), "operator_bytes": op_bytes}


def config1_oracle(steps=100, threads=1, limit_s=120):
    """The oracle on the small heat configuration (100 steps, one BLAS thread): build time,
    per-step times and the error against the closed form at T."""
    import subprocess
    code = f"""
import sys, time, json
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle.grid import Grid
from oracle.hps import HPS
from oracle.ark import ARK, ark436l2sa, tableau_float
from paper_2306_02526_amd import workloads
g = Grid(0, 1, 0, 1, 4, 4, 8)
x, y = g.coordinates()
wl = workloads.HeatManufactured(workloads.rng_for(1))
one = np.ones(g.n_int); zero = np.zeros(g.n_int)
co = dict(cxx=one, cyy=one, cx=zero, cy=zero, c0=zero)
tab = tableau_float(ark436l2sa()); dt = 0.01
t0 = time.perf_counter(); ark = ARK(HPS(g, co, tab['gamma'] * dt), co, tab, dt); tb = time.perf_counter() - t0
qs = wl.q_space(x[:g.n_int], y[:g.n_int])
u = wl.exact(0.0, x, y); times = []
for k in range({steps}):
    t = k * dt
    q = np.array([wl.q_time(t + c * dt) * qs for c in tab['c']])
    t0 = time.perf_counter(); u = ark.step(u, q); times.append(time.perf_counter() - t0)
err = float(np.abs(u - wl.exact({steps} * dt, x, y)).max())
print(json.dumps(dict(build_s=tb, times=times, err=err)))
"""
    import numpy as np
    th = str(threads)
    try:
        r = subprocess.run([sys.executable, "-c", code], stdout=subprocess.PIPE, text=True, timeout=limit_s,
                           env=dict(os.environ, OPENBLAS_NUM_THREADS=th, OMP_NUM_THREADS=th, MKL_NUM_THREADS=th))
    except subprocess.TimeoutExpired:
        return {"error": f"not finished within {limit_s} s"}
    if r.returncode != 0:
        return {"error": f"exit status {r.returncode}"}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    ts = np.array(d["times"]) * 1e3
    return {"workload": "heat_manufactured_4x4_leaves_p8", "steps": steps, "cores": threads,
            "latency_ms_per_step": {"p50": round(float(np.percentile(ts, 50)), 3),
                                    "p99": round(float(np.percentile(ts, 99)), 3)},
            "stage_solves_per_s": round(5 * steps / (ts.sum() / 1e3), 1), "build_s": round(d["build_s"], 3),
            "max_err_vs_exact_at_T": d["err"]}


def cpu_baseline(n, p, dt, n_solves, threads=1, limit_s=150, procs=1):
    """The oracle (plain NumPy FP64) on this host with `threads` BLAS threads: its build on
    the full grid (timed, not counted), then n_solves implicit stages of the same step
    timed; value = stage-solves/s on those stages.  procs > 1: that many copies run at once
    (one per core), value = all their stages over the wall-clock span from the first
    stage's start to the last stage's end."""
    import subprocess
    code = f"""
import os, sys, time, json
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle.grid import Grid
from oracle.hps import HPS
from oracle.ark import ARK, apply_L, ark436l2sa, tableau_float, poly_g
from paper_2306_02526_amd import workloads
g = Grid(0, 1, 0, 1, {n}, {n}, {p})
x, y = g.coordinates()
wl = workloads.AllenCahn(workloads.rng_for(2))
cxx, cyy, cx, cy, c0 = wl.L_coeffs(x[:g.n_int], y[:g.n_int])
co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
tab = tableau_float(ark436l2sa()); dt = {dt}
t0 = time.perf_counter(); H = HPS(g, co, tab['gamma'] * dt); tb = time.perf_counter() - t0
print(f"   oracle build {{tb:.1f}} s", file=sys.stderr, flush=True)
bar, nbar = os.environ.get("ORACLE_BARRIER"), int(os.environ.get("ORACLE_BARRIER_N", "1"))
if bar:   # concurrent copies: every copy has built before any times its stages
    open(os.path.join(bar, str(os.getpid())), "w").close()
    while len(os.listdir(bar)) < nbar: time.sleep(0.005)
u = wl.u0(x, y); n_int = g.n_int
A, Ah = tab['A'], tab['Ahat']
Lu = [apply_L(g, co, u)]; F = [poly_g(workloads.AllenCahn.gpoly, u[:n_int])]
times = []
for i in range(1, 1 + {n_solves}):
    t0 = time.perf_counter()
    rhs = u[:n_int].copy()
    for j in range(i):
        rhs += dt * A[i, j] * Lu[j] + dt * Ah[i, j] * F[j]
    ui = H.solve(rhs)
    Lu.append(apply_L(g, co, ui)); F.append(poly_g(workloads.AllenCahn.gpoly, ui[:n_int]))
    times.append(time.perf_counter() - t0)
    if i == 1: start = time.time() - times[-1]
    print(f"   oracle stage {{i}}: {{times[-1]:.1f}} s", file=sys.stderr, flush=True)
print(json.dumps(dict(build_s=tb, times=times, start=start, end=time.time())))
"""
    t0 = time.perf_counter()
    th = str(threads)
    import tempfile
    bar = tempfile.mkdtemp(prefix="oracle_barrier_")
    env = dict(os.environ, OPENBLAS_NUM_THREADS=th, OMP_NUM_THREADS=th, MKL_NUM_THREADS=th)
    if procs > 1:
        env.update(ORACLE_BARRIER=bar, ORACLE_BARRIER_N=str(procs))
    # progress lines go straight to stderr; each result is its process's last stdout line
    ps = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, text=True, env=env)
          for _ in range(procs)]
    outs, err = [], None
    for pr in ps:
        try:
            out, _ = pr.communicate(timeout=max(1.0, limit_s - (time.perf_counter() - t0)))
            if pr.returncode != 0:
                err = err or {"error": f"exit status {pr.returncode}"}
            else:
                outs.append(json.loads(out.strip().splitlines()[-1]))
        except subprocess.TimeoutExpired:
            err = {"error": f"not finished within {limit_s} s ({procs} process(es), {threads} BLAS thread(s) each)"}
            break
    for pr in ps:   # nothing is left running
        if pr.poll() is None:
            pr.kill()
        pr.wait()
    import shutil
    shutil.rmtree(bar, ignore_errors=True)
    if err:
        return err
    try:
        model = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")][0]
    except Exception:
        model = "unknown"
    d = outs[0]
    ts = d["times"]
    res = {"value": round(len(ts) / sum(ts), 4), "unit": "stage-solves/s", "cores": threads, "kind": "oracle",
           "sample": f"oracle build on the full {n}x{n} p={p} grid ({d['build_s']:.1f} s, not counted), then "
                     f"{len(ts)} implicit stages of one step (rhs assembly, HPS solve, L u_i, F_i) timed",
           "build_s": round(d["build_s"], 2), "host_cpu": model, "host_nproc": os.cpu_count(),
           "wall_s": round(time.perf_counter() - t0, 1)}
    if procs > 1:
        span = max(o["end"] for o in outs) - min(o["start"] for o in outs)
        total = sum(len(o["times"]) for o in outs)
        res.update(value=round(total / span, 4), cores=procs * threads, processes=procs,
                   sample=f"{procs} concurrent copies of: " + res["sample"],
                   stage_span_s=round(span, 2), build_s_max=round(max(o["build_s"] for o in outs), 2),
                   per_process_stage_solves_per_s=round(sum(len(o["times"]) / sum(o["times"]) for o in outs) / procs, 4))
    return res


if __name__ == "__main__":
    main()
    sys.stdout.flush()
    sys.stderr.flush()
    # leave nothing behind: every child process has been waited for; end without the
    # interpreter's and the runtime's teardown, except under a profiler, whose results
    # are written at a normal exit
    if "--normal-exit" not in sys.argv and "--counter-run" not in sys.argv and \
            not any(k.startswith("ROCPROF") for k in os.environ):
        os._exit(0)
