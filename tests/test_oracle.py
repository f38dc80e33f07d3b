"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's own formulas: each compares it with
a closed form, a printed value, an independent assembly, or an invariant that
a dropped term, a wrong sign or index, or a transposed operand would break.
"""
import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.ark import ARK, InterfaceSolver, SlopeARK, apply_L, ark436l2sa, tableau_float
from oracle.cheb import cheb_diff_ref, cheb_points, leaf_diff_1d, leaf_points_1d
from oracle.dense import dense_solve, flux_jump_matrix
from oracle.grid import Grid
from oracle.hps import HPS, leaf_index_sets, leaf_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _coefs(g, kind="var"):
    x, y = g.coordinates()
    xi, yi = x[: g.n_int], y[: g.n_int]
    if kind == "heat":
        one, zero = np.ones(g.n_int), np.zeros(g.n_int)
        return dict(cxx=one, cyy=one.copy(), cx=zero, cy=zero.copy(), c0=zero.copy())
    return dict(cxx=1.0 + 0.3 * np.sin(xi + 2 * yi), cyy=1.2 + 0.2 * np.cos(3 * xi),
                cx=0.5 * np.sin(yi), cy=-0.4 * np.cos(xi), c0=0.3 * np.sin(xi * yi))


# ---------------------------------------------------------------------------------------
# O1-O2: nodes and derivative
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("p", [3, 4, 5, 8, 11, 16, 21])
def test_derivative_exact_on_polynomials(p):
    a, h = 0.3, 0.7
    x = leaf_points_1d(a, h, p)
    D = leaf_diff_1d(h, p)
    for k in range(p):
        exact = k * x ** (k - 1) if k else np.zeros(p)
        err = np.abs(D @ x ** k - exact).max()
        assert err <= 1e-11 * max(1.0, np.abs(exact).max()) * p * p, (p, k, err)
    # nodes: ascending, endpoints exact, symmetric Chebyshev spacing
    assert np.all(np.diff(x) > 0) and x[0] == a and abs(x[-1] - (a + h)) < 1e-15
    xi = cheb_points(p)
    assert np.allclose(xi, -xi[::-1], atol=1e-15)


@pytest.mark.parametrize("p", [12, 16, 21])
def test_second_derivative_spectrum(p):
    """Sec. 4.1: Dirichlet D^2 on [-1,1] has real, negative, distinct eigenvalues that
    approximate lambda_k = -k^2 pi^2 / 4 at the low end."""
    gold = json.load(open(os.path.join(GOLDEN, "cheb_d2_spectrum.json")))
    D = cheb_diff_ref(p)
    E = (D @ D)[1:-1, 1:-1]
    ev = np.linalg.eigvals(E)
    assert np.abs(ev.imag).max() < 1e-8 * np.abs(ev.real).max()
    ev = np.sort(ev.real)[::-1]
    assert np.all(ev < 0)
    assert np.min(np.abs(np.diff(ev))) > 1e-6
    for k in gold["checked_k"]:
        lam = -(k ** 2) * math.pi ** 2 / 4.0
        assert abs(ev[k - 1] - lam) < 1e-4 * abs(lam), (p, k, ev[k - 1], lam)


# ---------------------------------------------------------------------------------------
# grid
# ---------------------------------------------------------------------------------------
def test_dof_counts_match_printed_values():
    gold = json.load(open(os.path.join(GOLDEN, "dof_counts.json")))
    for c in gold["cases"]:
        g = Grid(0, c["n1"], 0, c["n2"], c["n1"], c["n2"], c["p"])
        assert g.N == (c["p"] - 2) * (c["p"] * c["n1"] * c["n2"] + c["n1"] + c["n2"])
        assert c["printed"] - (c["n1"] + 1) * (c["n2"] + 1) == g.N, c


def test_grid_numbering_is_a_bijection_without_corners():
    g = Grid(0, 2, 0, 1, 4, 2, 6)
    seen = np.zeros(g.N, dtype=int)
    for j in range(g.n2):
        for i in range(g.n1):
            for b in range(g.p):
                for a in range(g.p):
                    k = g.local_to_global(i, j, a, b)
                    if (a in (0, g.p - 1)) and (b in (0, g.p - 1)):
                        assert k is None
                    else:
                        seen[k] += 1
    # interior nodes belong to one leaf, edge nodes to one or two leaves
    assert np.all(seen[: g.n_int] == 1)
    nb = g.boundary_mask()
    assert np.all(seen[g.n_int:][nb[g.n_int:]] == 1)
    assert np.all(seen[g.n_int:][~nb[g.n_int:]] == 2)
    assert len(g.boundary_indices()) == 2 * g.q * (g.n1 + g.n2)
    x, y = g.coordinates()
    assert not np.any(np.isnan(x)) and x.min() > 0 - 1e-15 and x.max() < 2 + 1e-15
    assert np.all((x[g.boundary_indices()] == 0) | (x[g.boundary_indices()] == 2)
                  | (y[g.boundary_indices()] == 0) | (y[g.boundary_indices()] == 1))


def test_leaf_rows_never_touch_corners():
    """Sec. 2.1: with c12 = 0 no interior collocation row references a corner node."""
    p = 7
    A = leaf_matrix(0.5, p, {k: np.full((p - 2) ** 2, 1.3) for k in ("cxx", "cyy", "cx", "cy", "c0")}, 0.1)
    for f in (0, p - 1, (p - 1) * p, p * p - 1):
        assert np.all(A[:, f] == 0.0)
    Ji, Jb = leaf_index_sets(p)
    assert len(set(Ji) | set(Jb)) == p * p - 4


# ---------------------------------------------------------------------------------------
# O4-O6: HPS = the global collocation system (Sec. 2.1 eq. 4; Sec. 3.1.1)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("n1,n2,p", [(1, 1, 6), (2, 1, 6), (1, 2, 5), (2, 2, 7), (4, 2, 6), (4, 4, 8), (2, 4, 5)])
def test_hps_equals_dense_global_solve(n1, n2, p):
    rng = np.random.default_rng(11 + n1 + 10 * n2 + 100 * p)
    g = Grid(0, n1 * 0.5, 0.25, 0.25 + n2 * 0.5, n1, n2, p)
    co = _coefs(g)
    H = HPS(g, co, 0.05)
    body = rng.standard_normal(g.n_int)
    dirv = rng.standard_normal(len(g.boundary_indices()))
    jump = rng.standard_normal(len(g.interface_indices()))
    for (bd, dv, jp) in [(body, dirv, jump), (body, None, None), (0 * body, dirv, None), (0 * body, None, jump)]:
        u1 = H.solve(bd, dv, jp)
        u2 = dense_solve(g, co, 0.05, bd, dv, jp)
        assert np.abs(u1 - u2).max() <= 1e-12 * np.abs(u2).max(), (n1, n2, p)


@pytest.mark.parametrize("n1,n2,p", [(2, 2, 6), (4, 2, 7), (4, 4, 5)])
def test_hps_exact_for_polynomials(n1, n2, p):
    """Collocation is exact for u = x^a y^b with a, b <= p-1 on every leaf, so with the
    body load A u evaluated in closed form the discrete solution is u at every node."""
    g = Grid(-0.5, -0.5 + n1 * 0.4, 0.1, 0.1 + n2 * 0.4, n1, n2, p)
    x, y = g.coordinates()
    xi, yi = x[: g.n_int], y[: g.n_int]
    co = _coefs(g)
    gdt = 0.07
    for (ea, eb) in [(p - 1, 0), (0, p - 1), (p - 1, p - 1), (2, 3), (1, 1)]:
        u = x ** ea * y ** eb
        ux = ea * xi ** max(ea - 1, 0) * yi ** eb if ea else 0 * xi
        uy = eb * xi ** ea * yi ** max(eb - 1, 0) if eb else 0 * xi
        uxx = ea * (ea - 1) * xi ** max(ea - 2, 0) * yi ** eb if ea > 1 else 0 * xi
        uyy = eb * (eb - 1) * xi ** ea * yi ** max(eb - 2, 0) if eb > 1 else 0 * xi
        Lu = co["cxx"] * uxx + co["cyy"] * uyy + co["cx"] * ux + co["cy"] * uy + co["c0"] * u[: g.n_int]
        body = u[: g.n_int] - gdt * Lu
        sol = HPS(g, co, gdt).solve(body, u[g.boundary_indices()], None)
        assert np.abs(sol - u).max() <= 1e-11 * np.abs(u).max(), (ea, eb)
        # and the collocation apply of L is exact on the same polynomial
        assert np.abs(apply_L(g, co, u) - Lu).max() <= 1e-10 * max(1.0, np.abs(Lu).max())


def test_hps_is_linear_and_flux_continuous():
    rng = np.random.default_rng(5)
    g = Grid(0, 1, 0, 1, 4, 4, 6)
    co = _coefs(g)
    H = HPS(g, co, 0.02)
    b1, b2 = rng.standard_normal((2, g.n_int))
    u1, u2, u12 = H.solve(b1), H.solve(b2), H.solve(b1 + 2 * b2)
    assert np.abs(u12 - (u1 + 2 * u2)).max() < 1e-12 * np.abs(u12).max()
    J = flux_jump_matrix(g)
    assert np.abs((J @ u12)[g.interface_indices()]).max() < 1e-9 * np.abs(u12).max() * g.p ** 2


def test_spatial_spectral_convergence():
    """Elliptic solve against a smooth exact solution: the error falls geometrically with p."""
    errs = []
    for p in (6, 9, 12, 15):
        g = Grid(0, 1, 0, 1, 2, 2, p)
        x, y = g.coordinates()
        co = _coefs(g, "heat")
        gdt = 0.1
        u = np.sin(2 * x + y) * np.exp(0.5 * y)
        xi, yi = x[: g.n_int], y[: g.n_int]
        # u = sin(2x+y) e^{y/2}: Lap u = (-5 sin + cos(2x+y) + 0.25 sin) e^{y/2}
        s, c = np.sin(2 * xi + yi), np.cos(2 * xi + yi)
        lap = (-4 * s + (-s + c + 0.25 * s)) * np.exp(0.5 * yi)
        body = u[: g.n_int] - gdt * lap
        sol = HPS(g, co, gdt).solve(body, u[g.boundary_indices()])
        errs.append(np.abs(sol - u).max())
    assert errs[1] < 1e-2 * errs[0] and errs[2] < 1e-2 * errs[1] and errs[3] < 1e-10


# ---------------------------------------------------------------------------------------
# O7: the tableau and the stage formulation
# ---------------------------------------------------------------------------------------
def _mv(M, v):
    return [sum(M[i][j] * v[j] for j in range(len(v))) for i in range(len(M))]


def _dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def test_ark436_order_conditions():
    """ARK4(3)6L[2]SA: row sums, order conditions to 4 for both tableaux and the coupling
    conditions, checked in rational arithmetic; stiffly accurate; L-stable."""
    t = ark436l2sa()
    s, A, Ah, b, bh, c = t["s"], t["A"], t["Ahat"], t["b"], t["bhat"], t["c"]
    one = [Fr(1)] * s
    tol = Fr(1, 10 ** 20)
    assert _mv(A, one) == c                                   # exact for the ESDIRK part
    assert all(abs(x - y) < tol for x, y in zip(_mv(Ah, one), c))
    assert all(A[i][i] == t["gamma"] for i in range(1, s)) and A[0][0] == 0
    assert A[s - 1][: s] == b                                  # stiffly accurate
    assert all(Ah[i][j] == 0 for i in range(s) for j in range(i, s))
    c2 = [x * x for x in c]
    c3 = [x * x * x for x in c]
    for bb in (b, bh):
        assert abs(_dot(bb, one) - 1) < tol
        assert abs(_dot(bb, c) - Fr(1, 2)) < tol
        assert abs(_dot(bb, c2) - Fr(1, 3)) < tol
        assert abs(_dot(bb, c3) - Fr(1, 4)) < tol
        for M in (A, Ah):
            Mc = _mv(M, c)
            assert abs(_dot(bb, Mc) - Fr(1, 6)) < tol
            assert abs(_dot(bb, [x * y for x, y in zip(c, Mc)]) - Fr(1, 8)) < tol
            assert abs(_dot(bb, _mv(M, c2)) - Fr(1, 12)) < tol
            for M2 in (A, Ah):
                assert abs(_dot(bb, _mv(M, _mv(M2, c))) - Fr(1, 24)) < tol
    # stability function of the ESDIRK part: R(z) = 1 + z b^T (I - z A)^{-1} 1
    Af = np.array([[float(x) for x in r] for r in A])
    bf = np.array([float(x) for x in b])

    def R(z):
        return 1 + z * bf @ np.linalg.solve(np.eye(s) - z * Af, np.ones(s))

    assert abs(R(-1e9)) < 1e-8
    assert max(abs(R(1j * w)) for w in np.logspace(-3, 4, 200)) <= 1 + 1e-12
    assert max(abs(R(-x)) for x in np.logspace(-3, 6, 200)) <= 1 + 1e-12


def _flux_continuous_state(g, u_int):
    u = np.zeros(g.N)
    u[: g.n_int] = u_int
    return InterfaceSolver(g).fill(u)


def test_ark_step_equals_stability_function():
    """q = g = f = 0: one stage-formulation step is R(dt K) u^n, K the interior operator
    with the interface values eliminated by flux continuity."""
    rng = np.random.default_rng(3)
    g = Grid(0, 1, 0, 1, 2, 2, 6)
    co = _coefs(g)
    tab = tableau_float(ark436l2sa())
    dt = 0.05
    ark = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt)
    u0 = _flux_continuous_state(g, rng.standard_normal(g.n_int))
    u1 = ark.step(u0)
    # dense K: columns are L applied to flux-continuous unit interior states
    n = g.n_int
    K = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        K[:, k] = apply_L(g, co, _flux_continuous_state(g, e))
    s, A, b = tab["s"], tab["A"], tab["b"]
    big = np.eye(s * n) - dt * np.kron(A, K)
    Ustages = np.linalg.solve(big, np.tile(u0[:n], s)).reshape(s, n)
    ref = u0[:n] + dt * sum(b[j] * (K @ Ustages[j]) for j in range(s))
    assert np.abs(u1[:n] - ref).max() <= 1e-11 * np.abs(ref).max()


def test_ark_temporal_order_four_on_a_decaying_mode():
    """q = g = 0, u = sin(pi x) sin(pi y) e^{-2 pi^2 t}: ESDIRK4 gives fourth order."""
    g = Grid(0, 1, 0, 1, 2, 2, 12)
    x, y = g.coordinates()
    co = _coefs(g, "heat")
    tab = tableau_float(ark436l2sa())
    ex = lambda t: np.sin(np.pi * x) * np.sin(np.pi * y) * np.exp(-2 * np.pi ** 2 * t)
    errs = []
    for dt in (0.04, 0.02, 0.01):
        ark = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt)
        u = ex(0.0)
        for _ in range(int(round(0.2 / dt))):
            u = ark.step(u)
        errs.append(np.abs(u - ex(0.2)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.7) and np.all(orders < 4.4), orders


def test_ark_converges_with_source_and_explicit_term():
    """Manufactured heat problem with a time-dependent source (ERK part active) and
    inhomogeneous boundary data: the step converges as dt shrinks."""
    g = Grid(0, 1, 0, 1, 2, 2, 12)
    x, y = g.coordinates()
    xi, yi = x[: g.n_int], y[: g.n_int]
    bi = g.boundary_indices()
    co = _coefs(g, "heat")
    tab = tableau_float(ark436l2sa())
    # exact u = sin(pi x) exp(-t (y - 1/2)^2)  (the paper's inhomogeneous-BC heat solution)
    ex = lambda t, X, Y: np.sin(np.pi * X) * np.exp(-t * (Y - 0.5) ** 2)

    def q(t, X, Y):
        E = np.exp(-t * (Y - 0.5) ** 2)
        s = np.sin(np.pi * X)
        return -(Y - 0.5) ** 2 * s * E + np.pi ** 2 * s * E - s * (4 * t * t * (Y - 0.5) ** 2 - 2 * t) * E

    errs = []
    for dt in (0.1, 0.05, 0.025):
        ark = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt)
        u, t = ex(0.0, x, y), 0.0
        for _ in range(int(round(0.4 / dt))):
            qs = np.array([q(t + c * dt, xi, yi) for c in tab["c"]])
            fs = np.array([ex(t + c * dt, x[bi], y[bi]) for c in list(tab["c"]) + [1.0]])
            u = ark.step(u, qs, fs)
            t += dt
        errs.append(np.abs(u - ex(t, x, y)).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-4
    assert np.log2(errs[1] / errs[2]) > 1.5


# ---------------------------------------------------------------------------------------
# O9: step completion
# ---------------------------------------------------------------------------------------
def test_step_update_equals_last_stage_without_sources():
    rng = np.random.default_rng(8)
    g = Grid(0, 1, 0, 2, 2, 4, 6)
    co = _coefs(g)
    tab = tableau_float(ark436l2sa())
    dt = 0.03
    ark = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt)
    nb = len(g.boundary_indices())
    fs = rng.standard_normal((tab["s"] + 1, nb))
    fs[-1] = fs[-2]     # c_s = 1: the last stage and t^{n+1} share the boundary data
    u0 = rng.standard_normal(g.N)
    u1, stages = ark.step(u0, None, fs, return_stages=True)
    assert np.abs(u1 - stages[-1]).max() <= 1e-12 * np.abs(u1).max()


def test_interface_fill_equals_identity_operator_hps():
    """Sec. 3.1.1: the explicit equation u = RHS with Dirichlet data, solved on the tree
    with the identity operator, gives the same interface values as the direct solve."""
    rng = np.random.default_rng(9)
    g = Grid(0, 2, 0, 1, 4, 2, 7)
    u = np.zeros(g.N)
    u[: g.n_int] = rng.standard_normal(g.n_int)
    bi = g.boundary_indices()
    u[bi] = rng.standard_normal(len(bi))
    direct = InterfaceSolver(g).fill(u.copy())
    zero = {k: np.zeros(g.n_int) for k in ("cxx", "cyy", "cx", "cy", "c0")}
    via_tree = HPS(g, zero, 0.3).solve(u[: g.n_int], u[bi], None)
    assert np.abs(direct - via_tree).max() <= 1e-12 * np.abs(direct).max()


# ---------------------------------------------------------------------------------------
# Theorem 1 (Sec. 4.2)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("h", [1.0, 1e-2, 1e-4, 1e-6])
def test_backward_euler_step_map_is_stable(h):
    g = Grid(0, 1, 0, 1, 2, 2, 6)
    co = _coefs(g, "heat")
    H = HPS(g, co, h)
    n = g.n_int
    M = np.zeros((g.N, g.N))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = H.solve(e)
    ev = np.linalg.eigvals(M)
    assert np.abs(ev).max() <= 1.0 + 1e-12
    # the columns of edge nodes vanish: at least one zero eigenvalue per interface node
    assert np.sum(np.abs(ev) < 1e-12) >= len(g.interface_indices())
    # and the interior-to-interior block contracts in the 2-norm
    assert np.linalg.norm(M[:n, :n], 2) <= 1.0 + 1e-12


# ---------------------------------------------------------------------------------------
# slope formulation with flux-jump penalisation (Sec. 3.1)
# ---------------------------------------------------------------------------------------
def _slope_coefs(x, y):
    return dict(cxx=1.0 + 0.3 * np.sin(x + 2 * y), cyy=1.2 + 0.2 * np.cos(3 * x), cx=0.5 * np.sin(y),
                cy=-0.4 * np.cos(x), c0=0.3 * np.sin(x * y))


def test_slope_equals_stage_for_flux_continuous_data():
    """Without sources and with fixed zero boundary data the two formulations are the same
    discrete map when u^n has a continuous flux: k_i = L u_i at interior nodes, and
    u^n + dt sum_j a_ij k_j solves the stage equation (uniqueness of the HPS solution)."""
    tab = tableau_float(ark436l2sa())
    g = Grid(0, 1, 0, 0.5, 4, 2, 8)
    x, y = g.coordinates()
    co = _slope_coefs(x[: g.n_int], y[: g.n_int])
    dt = 0.01
    H = HPS(g, co, tab["gamma"] * dt)
    un = H.solve(np.random.default_rng(1).standard_normal(g.n_int))
    st = ARK(H, co, tab, dt).step(un)
    sl = SlopeARK(H, co, tab, dt).step(un)
    assert np.abs(st - sl).max() <= 1e-12 * np.abs(st).max()


def test_slope_penalisation_removes_flux_jumps():
    """With every slope's flux jump set to -[[u^n]]/dt and sum_j b_j = 1, the step leaves no
    flux jump in u^{n+1} (g = 0), whatever the jumps of u^n."""
    tab = tableau_float(ark436l2sa())
    g = Grid(0, 1, 0, 0.5, 4, 2, 8)
    x, y = g.coordinates()
    co = _slope_coefs(x[: g.n_int], y[: g.n_int])
    dt = 0.01
    H = HPS(g, co, tab["gamma"] * dt)
    rng = np.random.default_rng(2)
    un = rng.standard_normal(g.N)
    un[g.boundary_indices()] = 0.0
    I = InterfaceSolver(g)
    before = np.abs(I.jump(un)).max()
    q = rng.standard_normal((tab["s"], g.n_int))
    un1 = SlopeARK(H, co, tab, dt).step(un, q_stages=q)
    assert before > 10.0
    assert np.abs(I.jump(un1)).max() <= 1e-13 * before


def test_slope_equals_stage_on_one_leaf_with_nonlinearity():
    """On one leaf (no interfaces) and fixed zero boundary data the formulations are the
    stage and slope forms of one IMEX method for the ODE u' = K u + g(u): equal maps."""
    tab = tableau_float(ark436l2sa())
    g = Grid(0, 1, 0, 1, 1, 1, 10)
    x, y = g.coordinates()
    co = _slope_coefs(x[: g.n_int], y[: g.n_int])
    dt = 0.01
    H = HPS(g, co, tab["gamma"] * dt)
    u = np.sin(math.pi * x) * np.sin(math.pi * y)
    gp = (0.2, 1.0, 0.3, -1.0)
    st = ARK(H, co, tab, dt, gp).step(u)
    sl = SlopeARK(H, co, tab, dt, gp).step(u)
    assert np.abs(st - sl).max() <= 1e-13 * np.abs(st).max()


def test_slope_fourth_order_with_time_dependent_boundary_data():
    """Heat equation with u = e^{-t} (sin(x + 2y) + x^2), whose boundary data depend on time:
    the penalised slope formulation (boundary slopes = u_t) converges at fourth order, the
    order of the tableau (error ratio 16 per halving of dt; checked >= 12)."""
    tab = tableau_float(ark436l2sa())
    g = Grid(0, 1, 0, 1, 2, 2, 16)
    x, y = g.coordinates()
    xi, yi = x[: g.n_int], y[: g.n_int]
    one, zero = np.ones(g.n_int), np.zeros(g.n_int)
    co = dict(cxx=one, cyy=one, cx=zero, cy=zero, c0=zero)
    psi = lambda X, Y: np.sin(X + 2 * Y) + X ** 2
    lap = lambda X, Y: -5.0 * np.sin(X + 2 * Y) + 2.0
    bnd = g.boundary_indices()
    T = 0.4
    errs = []
    for dt in (0.1, 0.05, 0.025):
        sl = SlopeARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt)
        u = psi(x, y)
        for m in range(int(round(T / dt))):
            t = m * dt
            q = np.array([math.exp(-(t + c * dt)) * (-psi(xi, yi) - lap(xi, yi)) for c in tab["c"]])
            fd = np.array([-math.exp(-(t + c * dt)) * psi(x[bnd], y[bnd]) for c in tab["c"]])
            u = sl.step(u, q_stages=q, fdot_stages=fd)
        errs.append(np.abs(u - math.exp(-T) * psi(x, y)).max())
    assert errs[0] / errs[1] >= 12.0 and errs[1] / errs[2] >= 12.0, errs
