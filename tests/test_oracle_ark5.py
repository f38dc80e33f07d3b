"""Pins of the fifth-order pair ARK5(4)8L[2]SA that Sec. 3 names beside ARK4(3)6L[2]SA
(Sec. 5.4 integrates the rotating flow with it).  Its coefficients are not printed in the
paper; they are checked here against what the mathematics fixes:

* every order condition of an additive Runge-Kutta pair up to order 5, i.e. one condition
  per rooted tree whose nodes carry one of two colours (ESDIRK or ERK), in exact rational
  arithmetic; the tree enumerator is pinned by the known counts of 2-coloured rooted trees
  (2, 4, 14, 52, 214) and shown to reject the fourth-order pair at order 5;
* stiff accuracy, the explicit first stage, row sums equal to c;
* L-stability from the exact stability function R(z) = det(I - zA + z 1 b^T) / det(I - zA);
* fifth-order convergence of the oracle's stage formulation with this tableau, for the
  implicit part (decaying Laplacian eigenmode) and for the explicit part (L = 0, the
  Allen-Cahn ODE u' = u - u^3 with its closed form).
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np

from oracle.ark import ARK, ark436l2sa, ark548l2sa, tableau_float
from oracle.grid import Grid
from oracle.hps import HPS


def _partitions(n, m=None):
    m = n if m is None else m
    if n == 0:
        yield []
        return
    for k in range(min(n, m), 0, -1):
        for rest in _partitions(n - k, k):
            yield [k] + rest


_TREES = {}


def coloured_trees(n):
    """All rooted trees with n nodes, each node coloured 0 (ESDIRK) or 1 (ERK), as
    (colour, sorted tuple of subtrees)."""
    if n not in _TREES:
        out = set()
        for col in (0, 1):
            if n == 1:
                out.add((col, ()))
                continue
            for parts in _partitions(n - 1):
                for kids in itertools.product(*[coloured_trees(k) for k in parts]):
                    out.add((col, tuple(sorted(kids))))
        _TREES[n] = sorted(out)
    return _TREES[n]


def _order(t):
    return 1 + sum(_order(k) for k in t[1])


def _density(t):
    return _order(t) * math.prod(_density(k) for k in t[1])


def _weights(t, mats):
    """Stage vector of the subtree: product over children of (A^{colour(child)} w_child)."""
    s = len(mats[0])
    v = [Fr(1)] * s
    for kid in t[1]:
        w = _weights(kid, mats)
        M = mats[kid[0]]
        v = [v[i] * sum(M[i][j] * w[j] for j in range(s)) for i in range(s)]
    return v


def condition_residual(tab, t):
    """b^{colour(root)} . weights(t) - 1/density(t), exactly."""
    mats = (tab["A"], tab["Ahat"])
    bs = (tab["b"], tab["bhat"])
    w = _weights(t, mats)
    return sum(x * y for x, y in zip(bs[t[0]], w)) - Fr(1, _density(t))


def test_coloured_tree_counts():
    # 2-coloured rooted trees with 1..5 nodes (OEIS A000151)
    assert [len(coloured_trees(n)) for n in range(1, 6)] == [2, 4, 14, 52, 214]
    assert all(_order(t) == n for n in range(1, 6) for t in coloured_trees(n))


def test_checker_accepts_order_four_and_rejects_order_five_for_ark436():
    t = ark436l2sa()
    tol = Fr(1, 10 ** 20)
    for n in range(1, 5):
        assert all(abs(condition_residual(t, tree)) < tol for tree in coloured_trees(n)), n
    assert max(abs(condition_residual(t, tree)) for tree in coloured_trees(5)) > Fr(1, 10 ** 4)


def test_ark548_structure():
    t = ark548l2sa()
    s, A, Ah, b, c, g = t["s"], t["A"], t["Ahat"], t["b"], t["c"], t["gamma"]
    assert s == 8 and g == Fr(41, 200)
    assert A[0] == [0] * s and all(A[i][i] == g for i in range(1, s))
    assert all(A[i][j] == 0 for i in range(s) for j in range(i + 1, s))
    assert all(Ah[i][j] == 0 for i in range(s) for j in range(i, s))
    assert A[s - 1] == b and t["bhat"] == b                    # stiffly accurate, b = bhat
    assert c[0] == 0 and c[-1] == 1
    tol = Fr(1, 10 ** 20)
    for M in (A, Ah):
        assert all(abs(sum(M[i]) - c[i]) < tol for i in range(s))


def test_ark548_order_conditions_to_five():
    t = ark548l2sa()
    tol = Fr(1, 10 ** 20)
    worst = max(abs(condition_residual(t, tree)) for n in range(1, 6) for tree in coloured_trees(n))
    assert worst < tol, float(worst)


def _det(M):
    M = [row[:] for row in M]
    n, d = len(M), Fr(1)
    for k in range(n):
        piv = next(i for i in range(k, n) if M[i][k] != 0)
        if piv != k:
            M[k], M[piv] = M[piv], M[k]
            d = -d
        d *= M[k][k]
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            for j in range(k, n):
                M[i][j] -= f * M[k][j]
    return d


def _R_exact(t, z):
    A, b, s = t["A"], t["b"], t["s"]
    D = [[Fr(int(i == j)) - z * A[i][j] for j in range(s)] for i in range(s)]
    N = [[D[i][j] + z * b[j] for j in range(s)] for i in range(s)]
    return _det(N) / _det(D)


def test_ark548_is_l_stable():
    t = ark548l2sa()
    r9, r12 = _R_exact(t, Fr(-10 ** 9)), _R_exact(t, Fr(-10 ** 12))
    assert abs(r9) < Fr(1, 10 ** 8) and abs(r12) < Fr(1, 10 ** 11)
    assert abs(r12 * 1000 / r9 - 1) < Fr(1, 1000)               # R(z) ~ C / z: R(-inf) = 0
    tf = tableau_float(t)
    Af, bf, s = tf["A"], tf["b"], tf["s"]

    def R(z):
        return 1 + z * bf @ np.linalg.solve(np.eye(s) - z * Af, np.ones(s))

    assert max(abs(R(1j * w)) for w in np.logspace(-3, 4, 200)) <= 1 + 1e-12
    assert max(abs(R(-x)) for x in np.logspace(-3, 4, 200)) <= 1 + 1e-12
    # R approximates exp to fifth order at the origin
    for z in (1e-2, -1e-2, 5e-3j):
        assert abs(R(z) - np.exp(z)) < 1e-11


def _heat_coefs(n):
    return dict(cxx=np.ones(n), cyy=np.ones(n), cx=np.zeros(n), cy=np.zeros(n), c0=np.zeros(n))


def test_ark548_temporal_order_five_on_a_decaying_mode():
    """q = g = 0, u = sin(pi x) sin(pi y) e^{-2 pi^2 t}: error ratio about 32 per halving of dt."""
    tab = tableau_float(ark548l2sa())
    g = Grid(0, 1, 0, 1, 2, 2, 12)
    x, y = g.coordinates()
    co = _heat_coefs(g.n_int)
    ex = lambda t: np.sin(np.pi * x) * np.sin(np.pi * y) * np.exp(-2 * np.pi ** 2 * t)
    errs = []
    for dt in (0.04, 0.02, 0.01):
        ark = ARK(HPS(g, co, tab["gamma"] * dt), co, tab, dt)
        u = ex(0.0)
        for _ in range(int(round(0.2 / dt))):
            u = ark.step(u)
        errs.append(np.abs(u - ex(0.2)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.6) and np.all(orders < 5.4), (errs, orders)


def test_ark548_explicit_part_order_five():
    """L = 0 and g = u - u^3: each stage solve returns its right-hand side at the interior
    nodes, so the interior values follow the ERK part for u' = u - u^3, whose solution is
    u0 e^t / sqrt(1 + u0^2 (e^{2t} - 1))."""
    tab = tableau_float(ark548l2sa())
    g = Grid(0, 1, 0, 1, 2, 2, 6)
    x, y = g.coordinates()
    n = g.n_int
    z = {k: np.zeros(n) for k in ("cxx", "cyy", "cx", "cy", "c0")}
    u0 = 0.3 + 0.5 * np.sin(3 * x) * np.cos(2 * y)
    T = 1.6
    exact = (u0 * np.exp(T) / np.sqrt(1 + u0 ** 2 * (np.exp(2 * T) - 1)))[:n]
    errs = []
    for dt in (0.2, 0.1, 0.05):
        ark = ARK(HPS(g, z, tab["gamma"] * dt), z, tab, dt, gpoly=(0.0, 1.0, 0.0, -1.0))
        u = u0.copy()
        for _ in range(int(round(T / dt))):
            u = ark.step(u)
        errs.append(np.abs(u[:n] - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.7) and np.all(orders < 5.5), (errs, orders)
