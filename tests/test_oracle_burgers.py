"""Pins of the Burgers-system oracle (oracle/burgers.py) against what the paper and the
mathematics fix: the closed-form solutions of Sec. 5.4 solve the equations (and the literal
printed traveling-wave exponent does not), the collocation advection term is exact on
polynomials, the system without advection is two scalar ARK steps, and the time stepping
converges to both closed-form solutions at the orders Sec. 5.4 reports (near 4 for the
diffusive solution, near 3 for the traveling wave, whose boundary data reduce the order)."""
import math

import numpy as np
import pytest

from oracle.ark import ARK, ark436l2sa, tableau_float
from oracle.burgers import BurgersARK, advection, grad_int
from oracle.grid import Grid
from oracle.hps import HPS
from paper_2306_02526_amd import workloads as W

TAB = tableau_float(ark436l2sa())


def d1(f, z, h):
    """Sixth-order central difference of a callable along one argument."""
    c = (1 / 60, -3 / 20, 3 / 4)
    return sum(ck * (f(z + (3 - k) * h) - f(z - (3 - k) * h)) for k, ck in enumerate(c)) / h


def d2(f, z, h):
    c0, c = -49 / 18, (1 / 90, -3 / 20, 3 / 2)
    return (c0 * f(z) + sum(ck * (f(z + (3 - k) * h) + f(z - (3 - k) * h)) for k, ck in enumerate(c))) / (h * h)


def burgers_residual(sol, t, x, y):
    """Residuals of both equations (u_t - eps Lap u + u u_x + v u_y, same for v), with
    derivatives by finite differences, relative to the largest term."""
    eps = sol.eps
    out = []
    for c in range(2):
        comp = lambda tt, xx, yy: sol.exact(tt, xx, yy)[c]
        ft = d1(lambda s: comp(s, x, y), t, 1e-3)
        fx = d1(lambda s: comp(t, s, y), x, 1e-3)
        fy = d1(lambda s: comp(t, x, s), y, 1e-3)
        lap = d2(lambda s: comp(t, s, y), x, 1e-3) + d2(lambda s: comp(t, x, s), y, 1e-3)
        u, v = sol.exact(t, x, y)
        terms = [ft, eps * lap, u * fx, v * fy]
        r = ft - eps * lap + u * fx + v * fy
        out.append(np.abs(r).max() / max(np.abs(tm).max() for tm in terms))
    return max(out)


@pytest.mark.parametrize("sol", [W.BurgersTravelingWave(0.1), W.BurgersDiffusive(0.1), W.BurgersDiffusive(0.02)],
                         ids=["traveling", "diffusive", "diffusive_eps0.02"])
def test_closed_forms_solve_the_burgers_system(sol):
    rng = np.random.default_rng(7)
    x, y = rng.uniform(0.05, 0.95, 40), rng.uniform(0.05, 0.95, 40)
    assert burgers_residual(sol, 0.3, x, y) < 1e-8


def test_literal_traveling_wave_exponent_is_not_a_solution():
    """The printed formula reads exp(4y - 4x - t) / (32 eps); it does not solve the system,
    which fixes the reading exp((4y - 4x - t) / (32 eps))."""

    class Literal:
        eps = 0.1

        def exact(self, t, x, y):
            w = 1.0 / (4.0 * (1.0 + np.exp(4.0 * y - 4.0 * x - t) / (32.0 * self.eps)))
            return 0.75 - w, 0.75 + w

    rng = np.random.default_rng(8)
    x, y = rng.uniform(0.05, 0.95, 40), rng.uniform(0.05, 0.95, 40)
    assert burgers_residual(Literal(), 0.3, x, y) > 1e-2


def test_advection_is_exact_on_polynomials():
    """u = x^2 y + 0.3, v = x y^3 - y (degree <= p - 1 on every leaf): u u_x + v u_y and
    u v_x + v v_y in closed form, at every interior node of a 3x2 grid."""
    g = Grid(-0.5, 1.0, 0.0, 1.0, 3, 2, 8)
    x, y = g.coordinates()
    u = x * x * y + 0.3
    v = x * y ** 3 - y
    ux, uy = grad_int(g, u)
    n = g.n_int
    xi, yi = x[:n], y[:n]
    assert np.allclose(ux, 2 * xi * yi, atol=1e-12, rtol=0)
    assert np.allclose(uy, xi * xi, atol=1e-12, rtol=0)
    au, av = advection(g, u, v)
    ui, vi = u[:n], v[:n]
    assert np.allclose(au, ui * 2 * xi * yi + vi * xi * xi, atol=1e-12, rtol=0)
    assert np.allclose(av, ui * yi ** 3 + vi * (3 * xi * yi * yi - 1), atol=1e-12, rtol=0)


def _setup(n1, n2, p, eps, dt):
    h = 1.0 / max(n1, n2)
    g = Grid(0.0, n1 * h, 0.0, n2 * h, n1, n2, p)
    cxx, cyy, cx, cy, c0 = W.burgers_coeffs(eps, g.n_int)
    co = dict(cxx=cxx, cyy=cyy, cx=cx, cy=cy, c0=c0)
    return g, co, HPS(g, co, TAB["gamma"] * dt)


def test_without_advection_the_system_is_two_scalar_steps():
    dt = 0.01
    g, co, hps = _setup(4, 2, 7, 0.1, dt)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(g.N), rng.standard_normal(g.N)
    nb = len(g.boundary_indices())
    fu, fv = rng.standard_normal((TAB["s"] + 1, nb)), rng.standard_normal((TAB["s"] + 1, nb))
    su, sv = BurgersARK(hps, co, TAB, dt, advect=False).step(u, v, fu, fv)
    ark = ARK(hps, co, TAB, dt)
    assert np.array_equal(su, ark.step(u, f_stages=fu))
    assert np.array_equal(sv, ark.step(v, f_stages=fv))


def boundary_stages(sol, g, t, dt):
    x, y = g.coordinates()
    b = g.boundary_indices()
    ts = [t + c * dt for c in TAB["c"]] + [t + dt]
    ex = [sol.exact(tt, x[b], y[b]) for tt in ts]
    return np.array([e[0] for e in ex]), np.array([e[1] for e in ex])


def integrate(sol, n, p, dt, T):
    g, co, hps = _setup(n, n, p, sol.eps, dt)
    orc = BurgersARK(hps, co, TAB, dt)
    x, y = g.coordinates()
    u, v = sol.exact(0.0, x, y)
    steps = int(round(T / dt))
    for k in range(steps):
        fu, fv = boundary_stages(sol, g, k * dt, dt)
        u, v = orc.step(u, v, fu, fv)
    ue, ve = sol.exact(T, x, y)
    return max(np.abs(u - ue).max(), np.abs(v - ve).max())


@pytest.mark.parametrize("sol,min_order,max_err", [(W.BurgersDiffusive(0.1), 3.5, 5e-6),
                                                   (W.BurgersTravelingWave(0.1), 2.4, 5e-7)],
                         ids=["diffusive", "traveling"])
def test_time_stepping_converges_to_closed_forms(sol, min_order, max_err):
    """4x4 leaves, p = 14, to T = 0.4 with dt = 0.1, 0.05, 0.025 (spatial error far below)."""
    errs = [integrate(sol, 4, 14, dt, 0.4) for dt in (0.1, 0.05, 0.025)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[1] < max_err, errs
    assert errs[2] < errs[1] < errs[0], errs
    assert orders[0] >= min_order, orders
    assert min(orders) >= 2.4, orders
