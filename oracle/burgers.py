"""Two-dimensional viscous Burgers system, stage formulation (oracle; test
infrastructure only).

Sec. 5.4 solves
  u_t = eps (u_xx + u_yy) - (u u_x + v u_y),
  v_t = eps (v_xx + v_yy) - (u v_x + v v_y)
with the same discretisation and ARK4(3)6L[2]SA in the stage formulation
(eqs. 9-11).  The printed second equation repeats the Laplacian of u; it is
read as the Laplacian of v (the standard Burgers system, and the only reading
under which the printed closed-form solutions satisfy the equations).

Both components are integrated with the same tableau and the same implicit
operator (I - gamma dt L), L u = eps Lap u (any L of eq. 3 with c12 = 0 is
accepted); the explicit part of each component is the advection term, which
couples them:
  F^u_j = -(u_j (u_j)_x + v_j (u_j)_y),   F^v_j = -(u_j (v_j)_x + v_j (v_j)_y),
evaluated at interior nodes by the same leaf collocation derivatives as L
(Sec. 2.1).  Stage solves, the interior update, the boundary data f(t + c_i dt)
and the interface values from flux continuity follow `oracle.ark.ARK` (reading
R1 for the step completion) for each component.
"""
import numpy as np

from .ark import ARK, InterfaceSolver, apply_L, tableau_float
from .cheb import leaf_diff_1d


def grad_int(grid, u):
    """(u_x, u_y) at the n_int interior nodes (canonical order) by tensor-product
    collocation on each leaf (the derivative of the leaf's degree p-1 interpolant)."""
    p, q = grid.p, grid.q
    D = leaf_diff_1d(grid.h, p)
    q2 = q * q
    ux_out = np.empty(grid.n_int)
    uy_out = np.empty(grid.n_int)
    for j in range(grid.n2):
        for i in range(grid.n1):
            U = np.full((p, p), np.nan)   # U[b, a]: row b along y, column a along x
            for b in range(p):
                for a in range(p):
                    g = grid.local_to_global(i, j, a, b)
                    if g is not None:
                        U[b, a] = u[g]
            ux = U @ D.T      # ux[b, a] = sum_m D[a, m] U[b, m]
            uy = D @ U        # uy[b, a] = sum_m D[b, m] U[m, a]
            k0 = (j * grid.n1 + i) * q2
            inner = (slice(1, p - 1), slice(1, p - 1))
            ux_out[k0:k0 + q2] = ux[inner].ravel()
            uy_out[k0:k0 + q2] = uy[inner].ravel()
    return ux_out, uy_out


def advection(grid, u, v):
    """(u u_x + v u_y, u v_x + v v_y) at the interior nodes, from full vectors u, v."""
    n = grid.n_int
    ux, uy = grad_int(grid, u)
    vx, vy = grad_int(grid, v)
    ui, vi = u[:n], v[:n]
    return ui * ux + vi * uy, ui * vx + vi * vy


class BurgersARK:
    """One stage-formulation step of the Burgers system on an HPS operator built with
    gamma_dt = gamma*dt for L (L = eps Lap for eq. of Sec. 5.4).  `advect=False` drops the
    advection terms (two independent linear problems; used as a check)."""

    def __init__(self, hps, coefs_int, tab, dt, advect=True):
        self.scalar = ARK(hps, coefs_int, tab, dt)   # checks gamma*dt against the operator
        self.hps = hps
        self.grid = hps.grid
        self.coefs = coefs_int
        self.tab = self.scalar.tab
        self.dt = float(dt)
        self.advect = advect
        self.iface = InterfaceSolver(self.grid)
        self.bnd = self.grid.boundary_indices()

    def _F(self, u, v):
        if not self.advect:
            z = np.zeros(self.grid.n_int)
            return z, z.copy()
        au, av = advection(self.grid, u, v)
        return -au, -av

    def step(self, u, v, fu_stages=None, fv_stages=None):
        """u, v: full N vectors at t^n.  fu_stages, fv_stages: (s+1, n_bdry) Dirichlet data
        of each component at t^n + c_i dt and at t^n + dt (None = 0).  Returns (u, v) at
        t^n + dt."""
        g, tab, dt = self.grid, self.tab, self.dt
        s, n = tab["s"], g.n_int
        A, Ah, b, bh = tab["A"], tab["Ahat"], tab["b"], tab["bhat"]
        nb = len(self.bnd)
        f_of = lambda f, i: np.zeros(nb) if f is None else f[i]
        comps = [(u, fu_stages), (v, fv_stages)]
        Lu = [[apply_L(g, self.coefs, w)] for w, _ in comps]
        F0 = self._F(u, v)
        F = [[F0[0]], [F0[1]]]
        for i in range(1, s):
            stage = []
            for c, (w, f) in enumerate(comps):
                rhs = w[:n].copy()
                for j in range(i):
                    rhs += dt * A[i, j] * Lu[c][j] + dt * Ah[i, j] * F[c][j]
                stage.append(self.hps.solve(rhs, f_of(f, i), None))
            for c in range(2):
                Lu[c].append(apply_L(g, self.coefs, stage[c]))
            Fi = self._F(stage[0], stage[1])
            F[0].append(Fi[0])
            F[1].append(Fi[1])
        out = []
        for c, (w, f) in enumerate(comps):
            wn = np.zeros(g.N)
            wn[:n] = w[:n]
            for j in range(s):
                wn[:n] += dt * b[j] * Lu[c][j] + dt * bh[j] * F[c][j]
            wn[self.bnd] = f_of(f, s)
            self.iface.fill(wn)
            out.append(wn)
        return out[0], out[1]


__all__ = ["grad_int", "advection", "BurgersARK", "tableau_float"]
