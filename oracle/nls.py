"""Regularised nonlinear Schroedinger equation, stage formulation (oracle; test
infrastructure only).

Sec. 5.5 integrates
  i u_t + (1 - i a eps) Lap u + (1 + i c eps) |u|^2 u = i b eps u,
i.e. u_t = (a eps + i) Lap u + (i - c eps) |u|^2 u + b eps u, for complex u with
homogeneous Dirichlet data.  The stiff part is L u = (a eps + i) Lap u (complex
coefficients cxx = cyy = a eps + i in the operator of eq. 3), the explicit part
g(u) = (i - c eps)|u|^2 u + b eps u.  The paper does not print a, b, c or eps; the
workloads pick values and say so.  Everything else is the stage formulation of
`oracle.ark.ARK` on complex vectors: the HPS build and solve, L u by collocation and the
interface update are the real ones applied to complex data (the oracle's linear
algebra is dtype-generic).
"""
import numpy as np

from .ark import ARK


def nls_coeffs(a, eps, n):
    """Complex coefficients of L = (a eps + i) Lap at n interior nodes."""
    z = complex(a * eps, 1.0)
    c = np.full(n, z, dtype=np.complex128)
    zero = np.zeros(n, dtype=np.complex128)
    return dict(cxx=c, cyy=c.copy(), cx=zero, cy=zero.copy(), c0=zero.copy())


def nls_g(u, b, c, eps):
    """(i - c eps) |u|^2 u + b eps u."""
    return (1j - c * eps) * (np.abs(u) ** 2) * u + b * eps * u


class NLSARK(ARK):
    """One stage-formulation step of the regularised NLS on a complex HPS operator built
    with gamma_dt for L = (a eps + i) Lap (coefficients from `nls_coeffs`)."""

    def __init__(self, hps, coefs_int, tab, dt, b, c, eps):
        super().__init__(hps, coefs_int, tab, dt)
        self.b, self.c, self.eps = float(b), float(c), float(eps)

    def g_of(self, u):
        return nls_g(u, self.b, self.c, self.eps)


def ode_exact(u0, t, b, c, eps):
    """Closed-form solution of u' = (i - c eps)|u|^2 u + b eps u (no Laplacian):
    rho = |u|^2 obeys rho' = 2 eps (b rho - c rho^2) (logistic, or rho' = -2 c eps rho^2
    when b = 0), and arg u grows at the rate rho."""
    rho0 = np.abs(u0) ** 2
    if b == 0.0:
        rho = rho0 / (1.0 + 2.0 * c * eps * rho0 * t)
        phase = np.log1p(2.0 * c * eps * rho0 * t) / (2.0 * c * eps) if c != 0.0 else rho0 * t
    else:
        e = np.exp(2.0 * b * eps * t)
        den = b + c * rho0 * (e - 1.0)
        rho = b * rho0 * e / den
        phase = np.log(den / b) / (2.0 * c * eps) if c != 0.0 else rho0 * (e - 1.0) / (2.0 * b * eps)
    return np.sqrt(rho / np.where(rho0 > 0, rho0, 1.0)) * u0 * np.exp(1j * phase)


__all__ = ["nls_coeffs", "nls_g", "NLSARK", "ode_exact"]
