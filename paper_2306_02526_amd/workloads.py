"""Seeded synthetic workloads (problem data only; no arithmetic of the method).

This is the one module that both the HIP path and the CPU oracle use.  It
draws the random parameters of each workload from NumPy's PCG64 generator and
evaluates closed-form coefficient fields, initial data, exact solutions and
manufactured sources at caller-supplied coordinates.  It never computes
collocation nodes, derivative matrices or anything else of the solver.

Workloads (all on the unit square, Dirichlet data):
  heat        u_t = Lap u + q, exact u = sin(pi x) sin(pi y) e^{-t} (1 + 0.1 F(x,y)),
              F a seeded mix of 8 Fourier modes, q = e^{-t} (-phi - Lap phi)
              (the manufactured-solution setting of the paper's 2-D heat tests).
  allen_cahn  u_t = div(a grad u) + u - u^3, a = 1 + 0.5 sin(2 pi x) cos(2 pi y),
              u0 = seeded sine modes k, l <= 8 normalised to max |u0| = 1, f = 0.
  batched     a seeded mix of heat / reaction problems with smooth a in [0.5, 1.5].
  burgers     the 2-D viscous Burgers system u_t = eps Lap u - (u u_x + v u_y),
              v_t = eps Lap v - (u v_x + v v_y) with the closed-form traveling-wave and
              diffusive solutions of the paper's analytic tests (eps = 0.1) and the
              rotating-flow initial data (eps = 0.005); boundary data from the exact
              solutions, zero for the rotating flow.
  nls         the regularised NLS filamentation test, i u_t + (1 - i a eps) Lap u
              + (1 + i c eps)|u|^2 u = i b eps u on [0, 25.6]^2, u0 = 5 exp(-r^2) about the
              centre, zero boundary data; a, b, c, eps are not printed and are chosen here
              (a = b = c = 1, eps = 0.05).
"""
import math

import numpy as np

SEED_BASE = 2306025260


def rng_for(stream, offset=0):
    return np.random.default_rng(SEED_BASE + int(stream) + int(offset))


# ---------------------------------------------------------------------------------------
# heat equation with a manufactured solution
# ---------------------------------------------------------------------------------------
class HeatManufactured:
    """u(t,x,y) = e^{-t} phi(x,y), phi = sin(pi x) sin(pi y) (1 + 0.1 F),
    F = sum_m alpha_m sin(pi (k_m x + l_m y) + ph_m); L = Laplacian, g = 0."""

    def __init__(self, rng, n_modes=8, amp=0.1, kmax=4, coef=None, Lx=1.0, Ly=1.0):
        # on [0, Lx] x [0, Ly] the envelope is sin(pi x / Lx) sin(pi y / Ly)
        self.Lx, self.Ly = float(Lx), float(Ly)
        self.k = rng.integers(1, kmax + 1, size=n_modes).astype(np.float64)
        self.l = rng.integers(1, kmax + 1, size=n_modes).astype(np.float64)
        self.ph = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
        al = rng.uniform(-1.0, 1.0, size=n_modes)
        self.alpha = al / np.sum(np.abs(al))
        self.amp = amp
        # optional variable diffusivity a(x,y) (None -> a = 1): L u = div(a grad u)
        self.coef = coef

    def _F(self, x, y):
        th = math.pi * (np.multiply.outer(x, self.k) + np.multiply.outer(y, self.l)) + self.ph
        F = np.sin(th) @ self.alpha
        Fx = (np.cos(th) * (math.pi * self.k)) @ self.alpha
        Fy = (np.cos(th) * (math.pi * self.l)) @ self.alpha
        lapF = -(np.sin(th) * (math.pi ** 2) * (self.k ** 2 + self.l ** 2)) @ self.alpha
        return F, Fx, Fy, lapF

    def phi_parts(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        wx, wy = math.pi / self.Lx, math.pi / self.Ly
        s = np.sin(wx * x) * np.sin(wy * y)
        sx = wx * np.cos(wx * x) * np.sin(wy * y)
        sy = wy * np.sin(wx * x) * np.cos(wy * y)
        lap_s = -(wx * wx + wy * wy) * s
        F, Fx, Fy, lapF = self._F(x, y)
        m = 1.0 + self.amp * F
        phi = s * m
        phix = sx * m + s * self.amp * Fx
        phiy = sy * m + s * self.amp * Fy
        lap_phi = lap_s * m + 2.0 * self.amp * (sx * Fx + sy * Fy) + s * self.amp * lapF
        return phi, phix, phiy, lap_phi

    def phi(self, x, y):
        return self.phi_parts(x, y)[0]

    def exact(self, t, x, y):
        return math.exp(-t) * self.phi(x, y)

    def q_space(self, x, y):
        """q(t,x,y) = q_time(t) * q_space(x,y) with q_time(t) = e^{-t}."""
        phi, phix, phiy, lap_phi = self.phi_parts(x, y)
        if self.coef is None:
            Lphi = lap_phi
        else:
            a, ax, ay = self.coef(x, y)
            Lphi = a * lap_phi + ax * phix + ay * phiy
        return -phi - Lphi

    @staticmethod
    def q_time(t):
        return math.exp(-t)

    def L_coeffs(self, x, y):
        """Coefficients (cxx, cyy, cx, cy, c0) of L u = cxx u_xx + cyy u_yy + cx u_x + cy u_y + c0 u."""
        x = np.asarray(x, dtype=np.float64)
        if self.coef is None:
            one = np.ones_like(x)
            zero = np.zeros_like(x)
            return one, one.copy(), zero, zero.copy(), zero.copy()
        a, ax, ay = self.coef(x, y)
        return a, a.copy(), ax, ay, np.zeros_like(a)


# ---------------------------------------------------------------------------------------
# variable-coefficient Allen-Cahn
# ---------------------------------------------------------------------------------------
def allen_cahn_a(x, y):
    """a = 1 + 0.5 sin(2 pi x) cos(2 pi y) and its exact gradient."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    tp = 2.0 * math.pi
    a = 1.0 + 0.5 * np.sin(tp * x) * np.cos(tp * y)
    ax = 0.5 * tp * np.cos(tp * x) * np.cos(tp * y)
    ay = -0.5 * tp * np.sin(tp * x) * np.sin(tp * y)
    return a, ax, ay


class AllenCahn:
    """u_t = div(a grad u) + u - u^3 on [0,1]^2, u = 0 on the boundary.
    L u = a u_xx + a u_yy + a_x u_x + a_y u_y (non-divergence form of the same operator)."""

    gpoly = (0.0, 1.0, 0.0, -1.0)

    def __init__(self, rng, kmax=8, coef=None, Lx=1.0, Ly=1.0):
        # on [0, Lx] x [0, Ly] the modes are sin(k pi x / Lx) sin(l pi y / Ly); coef (None:
        # allen_cahn_a) gives a and its gradient
        self.c = rng.standard_normal((kmax, kmax))
        self.kmax = kmax
        self.coef = coef
        self.Lx, self.Ly = float(Lx), float(Ly)
        X, Y = np.meshgrid(np.linspace(0.0, self.Lx, 257), np.linspace(0.0, self.Ly, 257), indexing="ij")
        self.scale = 1.0 / np.max(np.abs(self._raw(X.ravel(), Y.ravel())))

    def _raw(self, x, y):
        k = np.arange(1, self.kmax + 1, dtype=np.float64)
        sx = np.sin(math.pi / self.Lx * np.multiply.outer(x, k))
        sy = np.sin(math.pi / self.Ly * np.multiply.outer(y, k))
        return np.einsum("nk,kl,nl->n", sx, self.c, sy)

    def u0(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return self.scale * self._raw(x.ravel(), y.ravel()).reshape(x.shape)

    def L_coeffs(self, x, y):
        a, ax, ay = (allen_cahn_a if self.coef is None else self.coef)(x, y)
        return a, a.copy(), ax, ay, np.zeros_like(a)


# ---------------------------------------------------------------------------------------
# smooth random diffusivity for the batched mix
# ---------------------------------------------------------------------------------------
class SmoothDiffusivity:
    """a = 1 + 0.5 sum_m beta_m sin(2 pi (k_m x + l_m y) + ph_m), sum |beta| = 1, so a in [0.5, 1.5]."""

    def __init__(self, rng, n_modes=4):
        kl = []
        while len(kl) < n_modes:
            k, l = rng.integers(0, 3, size=2)
            if k or l:
                kl.append((float(k), float(l)))
        self.k = np.array([v[0] for v in kl])
        self.l = np.array([v[1] for v in kl])
        self.ph = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
        be = rng.uniform(-1.0, 1.0, size=n_modes)
        self.beta = be / np.sum(np.abs(be))

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        tp = 2.0 * math.pi
        th = tp * (np.multiply.outer(x, self.k) + np.multiply.outer(y, self.l)) + self.ph
        a = 1.0 + 0.5 * (np.sin(th) @ self.beta)
        ax = 0.5 * (np.cos(th) * (tp * self.k)) @ self.beta
        ay = 0.5 * (np.cos(th) * (tp * self.l)) @ self.beta
        return a, ax, ay


def batched_mix(n_problems=256, stream=4, sides=(8, 16, 32, 64), orders=(8, 12, 16)):
    """Per-problem data of the batched workload: n1, n2 drawn from `sides`, p from `orders`,
    gamma*dt in {1e-3, 1e-2}, smooth diffusivity a in [0.5, 1.5], heat (manufactured
    solution) or Allen-Cahn type 50/50.  Leaves are squares of side 1 / max(n1, n2), so the
    domain is [0, n1 h] x [0, n2 h] (the unit square when n1 == n2)."""
    out = []
    for b in range(n_problems):
        rng = rng_for(stream, b)
        n1 = int(rng.choice(list(sides)))
        n2 = int(rng.choice(list(sides)))
        p = int(rng.choice(list(orders)))
        gdt = float(rng.choice([1e-3, 1e-2]))
        kind = "heat" if rng.uniform() < 0.5 else "allen_cahn"
        coef = SmoothDiffusivity(rng)
        h = 1.0 / max(n1, n2)
        Lx, Ly = n1 * h, n2 * h
        if kind == "heat":
            prob = HeatManufactured(rng, coef=coef, Lx=Lx, Ly=Ly)
        else:
            prob = AllenCahn(rng, coef=coef, Lx=Lx, Ly=Ly)
        out.append({"n1": n1, "n2": n2, "p": p, "gamma_dt": gdt, "kind": kind,
                    "domain": (0.0, Lx, 0.0, Ly), "problem": prob})
    return out


# ---------------------------------------------------------------------------------------
# 2-D Burgers system
# ---------------------------------------------------------------------------------------
class BurgersTravelingWave:
    """u = 3/4 - 1/(4 (1 + e^{(4y - 4x - t)/(32 eps)})), v = 3/4 + 1/(4 (1 + e^{...})).
    (The printed formula places 32 eps outside the exponential; only the exponent reading
    solves the equations.)"""

    def __init__(self, eps=0.1):
        self.eps = float(eps)

    def exact(self, t, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        w = 1.0 / (4.0 * (1.0 + np.exp((4.0 * y - 4.0 * x - t) / (32.0 * self.eps))))
        return 0.75 - w, 0.75 + w


class BurgersDiffusive:
    """u = -4 pi eps E cos(2 pi x) sin(pi y) / (2 + E sin(2 pi x) sin(pi y)),
    v = -2 pi eps E sin(2 pi x) cos(pi y) / (2 + E sin(2 pi x) sin(pi y)),
    E = e^{-5 pi^2 eps t}."""

    def __init__(self, eps=0.1):
        self.eps = float(eps)

    def exact(self, t, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        e = math.exp(-5.0 * math.pi ** 2 * self.eps * t)
        den = 2.0 + e * np.sin(2 * math.pi * x) * np.sin(math.pi * y)
        u = -4.0 * math.pi * self.eps * e * np.cos(2 * math.pi * x) * np.sin(math.pi * y) / den
        v = -2.0 * math.pi * self.eps * e * np.sin(2 * math.pi * x) * np.cos(math.pi * y) / den
        return u, v


class BurgersRotating:
    """Rotating flow on [-pi, pi]^2: u0 = -5 y e^{-3 (x^2 + y^2)}, v0 = 5 x e^{-3 (x^2 + y^2)},
    no-slip walls (u = v = 0 on the boundary), eps = 0.005."""

    domain = (-math.pi, math.pi, -math.pi, math.pi)

    def __init__(self, eps=0.005):
        self.eps = float(eps)

    def u0(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        e = np.exp(-3.0 * (x * x + y * y))
        return -5.0 * y * e, 5.0 * x * e


def burgers_coeffs(eps, n):
    """Coefficients of L = eps Lap at n nodes: cxx, cyy, cx, cy, c0."""
    e = np.full(n, float(eps))
    z = np.zeros(n)
    return e, e.copy(), z, z.copy(), z.copy()


# ---------------------------------------------------------------------------------------
# regularised nonlinear Schroedinger equation (multiple filamentation)
# ---------------------------------------------------------------------------------------
class NLSFilamentation:
    """u_t = (a eps + i) Lap u + (i - c eps)|u|^2 u + b eps u on [0, 25.6]^2, u = 0 on the
    boundary, u0 = 5 exp(-(x - 12.8)^2 - (y - 12.8)^2)."""

    domain = (0.0, 25.6, 0.0, 25.6)

    def __init__(self, a=1.0, b=1.0, c=1.0, eps=0.05):
        self.a, self.b, self.c, self.eps = float(a), float(b), float(c), float(eps)

    def u0(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return (5.0 * np.exp(-(x - 12.8) ** 2 - (y - 12.8) ** 2)).astype(np.complex128)

    def coeffs(self, n):
        """Real and imaginary parts of the coefficients of L = (a eps + i) Lap."""
        z = np.zeros(n)
        re = dict(cxx=np.full(n, self.a * self.eps), cyy=np.full(n, self.a * self.eps), cx=z, cy=z.copy(), c0=z.copy())
        im = dict(cxx=np.ones(n), cyy=np.ones(n), cx=z.copy(), cy=z.copy(), c0=z.copy())
        return re, im

    def g(self):
        """(g0, g1, g2, g3) of g(u) = (g0 + i g1) u + (g2 + i g3)|u|^2 u."""
        return (self.b * self.eps, 0.0, -self.c * self.eps, 1.0)

