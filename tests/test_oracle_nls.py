"""Pins of the complex (NLS) oracle against what the mathematics fixes: the closed form of
the NLS nonlinearity's ODE, the complex HPS solve against the dense complex global system
of eq. (4), a real operator on complex data acting on the real and imaginary parts
separately, fourth-order convergence to the damped linear Schroedinger eigenmode (which
fixes the sign of i in L), and fourth-order convergence of the explicit part to the ODE's
closed form when the Laplacian is switched off (which fixes g)."""
import math

import numpy as np
import pytest

from oracle.ark import ARK, ark436l2sa, tableau_float
from oracle.dense import dense_solve
from oracle.grid import Grid
from oracle.hps import HPS
from oracle.nls import NLSARK, nls_coeffs, nls_g, ode_exact

TAB = tableau_float(ark436l2sa())


@pytest.mark.parametrize("b,c", [(0.0, 0.0), (0.0, 1.5), (0.8, 1.5), (0.8, 0.0)])
def test_ode_closed_form_solves_the_ode(b, c):
    eps = 0.3
    rng = np.random.default_rng(1)
    u0 = 0.7 * (rng.standard_normal(20) + 1j * rng.standard_normal(20))
    h, t = 1e-3, 0.7
    f = lambda s: ode_exact(u0, s, b, c, eps)
    # sixth-order central difference in t
    du = sum(ck * (f(t + (3 - k) * h) - f(t - (3 - k) * h)) for k, ck in enumerate((1 / 60, -3 / 20, 3 / 4))) / h
    rhs = nls_g(f(t), b, c, eps)
    assert np.abs(du - rhs).max() <= 1e-8 * np.abs(rhs).max()
    assert np.abs(ode_exact(u0, 0.0, b, c, eps) - u0).max() <= 1e-15 * np.abs(u0).max()


def complex_coefs(n, rng):
    return dict(cxx=np.full(n, 0.3 + 1.0j), cyy=np.full(n, 0.3 + 1.0j) + 0.05 * rng.standard_normal(n),
                cx=0.1j * np.ones(n), cy=np.zeros(n, complex), c0=np.full(n, -0.2 + 0.05j))


@pytest.mark.parametrize("n1,n2,p", [(2, 2, 6), (4, 2, 5)])
def test_complex_hps_equals_dense_global_solve(n1, n2, p):
    rng = np.random.default_rng(n1 + 10 * p)
    g = Grid(0, 1, 0, n2 / n1, n1, n2, p)
    co = complex_coefs(g.n_int, rng)
    cplx = lambda n: rng.standard_normal(n) + 1j * rng.standard_normal(n)
    body, dirichlet = cplx(g.n_int), cplx(len(g.boundary_indices()))
    jump = cplx(len(g.interface_indices()))
    u = HPS(g, co, 0.01).solve(body, dirichlet, jump)
    ref = dense_solve(g, co, 0.01, body, dirichlet, jump)
    assert u.dtype == np.complex128
    assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max()


def test_real_operator_on_complex_data_splits():
    rng = np.random.default_rng(3)
    g = Grid(0, 1, 0, 1, 2, 2, 7)
    n = g.n_int
    co = dict(cxx=np.full(n, 1.0), cyy=np.full(n, 1.2), cx=0.3 * np.ones(n), cy=np.zeros(n), c0=np.zeros(n))
    H = HPS(g, co, 0.02)
    br, bi = rng.standard_normal(n), rng.standard_normal(n)
    u = H.solve(br + 1j * bi)
    assert np.allclose(u.real, H.solve(br), rtol=0, atol=1e-13)
    assert np.allclose(u.imag, H.solve(bi), rtol=0, atol=1e-13)


def _step_errors(make, dts, T):
    errs = []
    for dt in dts:
        errs.append(make(dt, T))
    return errs


def test_damped_schroedinger_mode_converges_at_fourth_order():
    """u_t = (a eps + i) Lap u on [0,1]^2, u = 0 on the boundary: the mode sin(pi x) sin(2 pi y)
    decays as exp(-5 pi^2 (a eps + i) t)."""
    a, eps = 0.5, 0.4
    g = Grid(0, 1, 0, 1, 2, 2, 14)
    x, y = g.coordinates()
    mode = np.sin(math.pi * x) * np.sin(2 * math.pi * y)
    co = nls_coeffs(a, eps, g.n_int)

    def run(dt, T):
        ark = ARK(HPS(g, co, TAB["gamma"] * dt), co, TAB, dt)     # no explicit part
        u = mode.astype(complex)
        for _ in range(int(round(T / dt))):
            u = ark.step(u)
        return np.abs(u - np.exp(-5 * math.pi ** 2 * complex(a * eps, 1.0) * T) * mode).max()

    errs = _step_errors(run, (0.02, 0.01, 0.005), 0.2)
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 1e-5, errs
    assert min(orders) > 3.5, orders


def test_explicit_part_converges_to_the_ode_closed_form():
    """With L = 0 every stage solve returns its right-hand side at the interior nodes, so the
    interior values follow the explicit tableau for u' = g(u) and converge at fourth order to
    the closed form."""
    b, c, eps = 0.8, 1.5, 0.3
    g = Grid(0, 1, 0, 1, 2, 2, 6)
    x, y = g.coordinates()
    n = g.n_int
    co = {k: np.zeros(n, complex) for k in ("cxx", "cyy", "cx", "cy", "c0")}
    u0 = (0.8 + 0.5 * np.sin(3 * x)) * np.exp(1j * (2 * y - x))

    def run(dt, T):
        ark = NLSARK(HPS(g, co, TAB["gamma"] * dt), co, TAB, dt, b=b, c=c, eps=eps)
        u = u0.copy()
        for _ in range(int(round(T / dt))):
            u = ark.step(u)
        return np.abs(u[:n] - ode_exact(u0[:n], T, b, c, eps)).max()

    errs = _step_errors(run, (0.2, 0.1, 0.05), 1.6)
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) > 3.5, (errs, orders)


def test_real_data_with_real_operator_equals_the_real_oracle():
    """The complex-capable oracle on real data and a real operator is the real oracle."""
    g = Grid(0, 1, 0, 1, 2, 2, 6)
    n = g.n_int
    co = dict(cxx=np.ones(n), cyy=np.ones(n), cx=np.zeros(n), cy=np.zeros(n), c0=np.zeros(n))
    rng = np.random.default_rng(5)
    u = rng.standard_normal(g.N)
    ark = ARK(HPS(g, co, TAB["gamma"] * 0.01), co, TAB, 0.01)
    out = ark.step(u)
    assert out.dtype == np.float64
