"""IMEX additive Runge-Kutta steps, stage formulation (ARK) and slope formulation with
flux-jump penalisation (SlopeARK) (oracle; test infrastructure only).

Sec. 3.1: the stiff part L u is integrated by an ESDIRK tableau (A, b, c) with
an explicit first stage and a_ii = gamma, the non-stiff part q + g(u) by an
ERK tableau (Ahat, bhat, c); both share c.  The paper uses ARK4(3)6L[2]SA of
Kennedy & Carpenter (2003); its coefficients are not printed in the paper
and are given here from that publication (exact rationals).  Table 1 fixes
the structure: the ESDIRK last row equals b (stiffly accurate); the ERK last
row differs from bhat.

Stage formulation (eqs. 9-11):
  u_1 = u^n,
  (I - dt*gamma*L) u_i = u^n + dt sum_{j<i} a_ij L u_j
                             + dt sum_{j<i} ahat_ij (q(t^n + c_j dt) + g(u_j)),
  u_i = f(t^n + c_i dt) on the boundary,          i = 2..s.
(The source time in eq. 9 is printed with index i; it is read as c_j.)

Step completion (the paper does not print it for the stage formulation; the
reading used here is documented as R1):
  interior:  u^{n+1} = u^n + dt sum_j b_j L u_j + dt sum_j bhat_j F_j,
             F_j = q(t^n + c_j dt) + g(u_j), the standard ARK update, as in
             the slope-formulation updates of Sec. 3.1;
  boundary:  u^{n+1} = f(t^{n+1});
  interface edge nodes: the values that make the flux continuous across every
             interior edge given the interior and boundary values, i.e. the
             "explicit equation u = known RHS" solved with Dirichlet data on
             the tree (Sec. 3.1.1).
With q = g = 0 this equals u_s exactly, because the last ESDIRK row is b.

L u is evaluated by collocation at interior nodes only:
  L u = cxx u_xx + cyy u_yy + cx u_x + cy u_y + c0 u  (the operator of eq. 3
with c12 = 0, written for L instead of A).
"""
from fractions import Fraction as Fr

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cheb import leaf_diff_1d
from .dense import flux_jump_matrix


def ark436l2sa():
    """ARK4(3)6L[2]SA (Kennedy & Carpenter 2003) as exact rationals."""
    s = 6
    A = [[Fr(0)] * s for _ in range(s)]
    Ah = [[Fr(0)] * s for _ in range(s)]
    g = Fr(1, 4)
    A[1][0] = Fr(1, 4)
    A[2][0], A[2][1] = Fr(8611, 62500), Fr(-1743, 31250)
    A[3][0], A[3][1], A[3][2] = Fr(5012029, 34652500), Fr(-654441, 2922500), Fr(174375, 388108)
    A[4][0], A[4][1], A[4][2], A[4][3] = (Fr(15267082809, 155376265600), Fr(-71443401, 120774400),
                                          Fr(730878875, 902184768), Fr(2285395, 8070912))
    b = [Fr(82889, 524892), Fr(0), Fr(15625, 83664), Fr(69875, 102672), Fr(-2260, 8211), Fr(1, 4)]
    for i in range(1, s):
        A[i][i] = g
    for j in range(s - 1):
        A[5][j] = b[j]
    Ah[1][0] = Fr(1, 2)
    Ah[2][0], Ah[2][1] = Fr(13861, 62500), Fr(6889, 62500)
    Ah[3][0], Ah[3][1], Ah[3][2] = (Fr(-116923316275, 2393684061468), Fr(-2731218467317, 15368042101831),
                                    Fr(9408046702089, 11113171139209))
    Ah[4][0], Ah[4][1], Ah[4][2], Ah[4][3] = (Fr(-451086348788, 2902428689909),
                                              Fr(-2682348792572, 7519795681897),
                                              Fr(12662868775082, 11960479115383),
                                              Fr(3355817975965, 11060851509271))
    Ah[5][0], Ah[5][1], Ah[5][2], Ah[5][3], Ah[5][4] = (Fr(647845179188, 3216320057751),
                                                        Fr(73281519250, 8382639484533),
                                                        Fr(552539513391, 3454668386233),
                                                        Fr(3354512671639, 8306763924573),
                                                        Fr(4040, 17871))
    c = [Fr(0), Fr(1, 2), Fr(83, 250), Fr(31, 50), Fr(17, 20), Fr(1)]
    return {"s": s, "gamma": g, "A": A, "b": b, "Ahat": Ah, "bhat": list(b), "c": c}


def ark548l2sa():
    """ARK5(4)8L[2]SA (Kennedy & Carpenter 2003), the fifth-order pair Sec. 3 names next to
    ARK4(3)6L[2]SA and Sec. 5.4 uses for the rotating flow, as exact rationals: ESDIRK with
    an explicit first stage, a_ii = 41/200, last row equal to b; the ERK part shares c and b;
    a_i2 = 0 in both parts for i >= 4."""
    s = 8
    A = [[Fr(0)] * s for _ in range(s)]
    Ah = [[Fr(0)] * s for _ in range(s)]
    g = Fr(41, 200)
    A[1][0] = g
    A[2][:2] = [Fr(41, 400), Fr(-567603406766, 11931857230679)]
    A[3][:3] = [Fr(683785636431, 9252920307686), Fr(0), Fr(-110385047103, 1367015193373)]
    A[4][:4] = [Fr(3016520224154, 10081342136671), Fr(0), Fr(30586259806659, 12414158314087),
                Fr(-22760509404356, 11113319521817)]
    A[5][:5] = [Fr(218866479029, 1489978393911), Fr(0), Fr(638256894668, 5436446318841),
                Fr(-1179710474555, 5321154724896), Fr(-60928119172, 8023461067671)]
    A[6][:6] = [Fr(1020004230633, 5715676835656), Fr(0), Fr(25762820946817, 25263940353407),
                Fr(-2161375909145, 9755907335909), Fr(-211217309593, 5846859502534),
                Fr(-4269925059573, 7827059040749)]
    b = [Fr(-872700587467, 9133579230613), Fr(0), Fr(0), Fr(22348218063261, 9555858737531),
         Fr(-1143369518992, 8141816002931), Fr(-39379526789629, 19018526304540),
         Fr(32727382324388, 42900044865799), g]
    A[7][:7] = b[:7]
    for i in range(1, s):
        A[i][i] = g
    Ah[1][0] = Fr(41, 100)
    Ah[2][:2] = [Fr(367902744464, 2072280473677), Fr(677623207551, 8224143866563)]
    Ah[3][:3] = [Fr(1268023523408, 10340822734521), Fr(0), Fr(1029933939417, 13636558850479)]
    Ah[4][:4] = [Fr(14463281900351, 6315353703477), Fr(0), Fr(66114435211212, 5879490589093),
                 Fr(-54053170152839, 4284798021562)]
    Ah[5][:5] = [Fr(14090043504691, 34967701212078), Fr(0), Fr(15191511035443, 11219624916014),
                 Fr(-18461159152457, 12425892160975), Fr(-281667163811, 9011619295870)]
    Ah[6][:6] = [Fr(19230459214898, 13134317526959), Fr(0), Fr(21275331358303, 2942455364971),
                 Fr(-38145345988419, 4862620318723), Fr(-1, 8), Fr(-1, 8)]
    Ah[7][:7] = [Fr(-19977161125411, 11928030595625), Fr(0), Fr(-40795976796054, 6384907823539),
                 Fr(177454434618887, 12078138498510), Fr(782672205425, 8267701900261),
                 Fr(-69563011059811, 9646580694205), Fr(7356628210526, 4942186776405)]
    c = [Fr(0), Fr(41, 100), Fr(2935347310677, 11292855782101), Fr(1426016391358, 7196633302097),
         Fr(23, 25), Fr(6, 25), Fr(3, 5), Fr(1)]
    return {"s": s, "gamma": g, "A": A, "b": b, "Ahat": Ah, "bhat": list(b), "c": c}


def tableau_float(tab):
    f = lambda M: np.array([[float(x) for x in row] for row in M])
    return {"s": tab["s"], "gamma": float(tab["gamma"]), "A": f(tab["A"]), "Ahat": f(tab["Ahat"]),
            "b": np.array([float(x) for x in tab["b"]]), "bhat": np.array([float(x) for x in tab["bhat"]]),
            "c": np.array([float(x) for x in tab["c"]])}


def apply_L(grid, coefs_int, u):
    """L u at the n_int interior nodes (canonical order) from the full vector u."""
    p, q = grid.p, grid.q
    D = leaf_diff_1d(grid.h, p)
    D2 = D @ D
    dt = np.result_type(np.asarray(u), *[np.asarray(v) for v in coefs_int.values()])
    out = np.empty(grid.n_int, dtype=dt)
    q2 = q * q
    for j in range(grid.n2):
        for i in range(grid.n1):
            U = np.full((p, p), np.nan, dtype=dt)   # U[b, a]; corners stay NaN and must never be read
            for b in range(p):
                for a in range(p):
                    g = grid.local_to_global(i, j, a, b)
                    if g is not None:
                        U[b, a] = u[g]
            ux = U @ D.T      # ux[b, a] = sum_m D[a, m] U[b, m]
            uxx = U @ D2.T
            uy = D @ U        # uy[b, a] = sum_m D[b, m] U[m, a]
            uyy = D2 @ U
            k0 = (j * grid.n1 + i) * q2
            sl = slice(k0, k0 + q2)
            inner = (slice(1, p - 1), slice(1, p - 1))
            out[sl] = (coefs_int["cxx"][sl] * uxx[inner].ravel() + coefs_int["cyy"][sl] * uyy[inner].ravel()
                       + coefs_int["cx"][sl] * ux[inner].ravel() + coefs_int["cy"][sl] * uy[inner].ravel()
                       + coefs_int["c0"][sl] * U[inner].ravel())
    return out


def poly_g(gpoly, u):
    """g(u) = g0 + g1 u + g2 u^2 + g3 u^3 pointwise (None means g = 0)."""
    if gpoly is None:
        return np.zeros_like(u)
    g0, g1, g2, g3 = gpoly
    return g0 + g1 * u + g2 * u * u + g3 * u * u * u


class InterfaceSolver:
    """Interface values from flux continuity, given interior and boundary values."""

    def __init__(self, grid):
        self.grid = grid
        J = flux_jump_matrix(grid)
        self.iface = grid.interface_indices()
        rest = np.ones(grid.N, dtype=bool)
        rest[self.iface] = False
        self.rest = np.nonzero(rest)[0]
        self.Jr = sp.csr_matrix(J[self.iface])
        self.J_ii = sp.csc_matrix(self.Jr[:, self.iface])
        self.J_ir = self.Jr[:, self.rest]

    def jump(self, u):
        """flux_alpha - flux_beta of u at every interface node."""
        return self.Jr @ u

    def fill(self, u, jump=None):
        """Set the interface values of u so that its flux jump equals `jump` (None: 0)."""
        if len(self.iface) == 0:
            return u
        rhs = -(self.J_ir @ u[self.rest])
        if jump is not None:
            rhs = rhs + jump
        u[self.iface] = spla.spsolve(self.J_ii, rhs)
        return u


class ARK:
    """One stage-formulation step on an HPS operator built with gamma_dt = gamma*dt."""

    def __init__(self, hps, coefs_int, tab, dt, gpoly=None):
        self.hps = hps
        self.grid = hps.grid
        self.coefs = coefs_int
        self.tab = tableau_float(tab) if isinstance(tab["gamma"], Fr) else tab
        self.dt = float(dt)
        self.gpoly = gpoly
        if abs(self.tab["gamma"] * self.dt - hps.gamma_dt) > 1e-15 * abs(hps.gamma_dt):
            raise ValueError("operator was built for a different gamma*dt")
        self.iface = InterfaceSolver(self.grid)
        self.bnd = self.grid.boundary_indices()

    def g_of(self, u):
        """The explicit nonlinearity g at interior values u."""
        return poly_g(self.gpoly, u)

    def step(self, u, q_stages=None, f_stages=None, return_stages=False):
        """u: full N vector at t^n.  q_stages: (s, n_int) source at t^n + c_i dt (or None).
        f_stages: (s+1, n_bdry) Dirichlet data at t^n + c_i dt and at t^n + dt (or None = 0)."""
        g, tab, dt = self.grid, self.tab, self.dt
        s = tab["s"]
        n_int = g.n_int
        A, Ah, b, bh = tab["A"], tab["Ahat"], tab["b"], tab["bhat"]
        q_at = (lambda i: np.zeros(n_int)) if q_stages is None else (lambda i: q_stages[i])
        f_at = (lambda i: np.zeros(len(self.bnd))) if f_stages is None else (lambda i: f_stages[i])
        un_int = u[:n_int].copy()
        Lu = [apply_L(g, self.coefs, u)]
        F = [q_at(0) + self.g_of(un_int)]
        stages = [u.copy()]
        for i in range(1, s):
            rhs = un_int.copy()
            for j in range(i):
                rhs += dt * A[i, j] * Lu[j] + dt * Ah[i, j] * F[j]
            ui = self.hps.solve(rhs, f_at(i), None)
            stages.append(ui)
            Lu.append(apply_L(g, self.coefs, ui))
            F.append(q_at(i) + self.g_of(ui[:n_int]))
        unew = np.zeros(g.N, dtype=np.result_type(u, *Lu))
        unew[:n_int] = un_int
        for j in range(s):
            unew[:n_int] += dt * b[j] * Lu[j] + dt * bh[j] * F[j]
        unew[self.bnd] = f_at(s)
        self.iface.fill(unew)
        if return_stages:
            return unew, stages
        return unew


class SlopeARK:
    """One step of the slope formulation (Sec. 3.1, eqs. for k_i and l_i) with the
    flux-jump penalisation of Sec. 3.1 ("Penalization in the slope formulation").

      k_1 = L u^n + q(t^n),           l_1 = g(u^n),
      (I - dt gamma L) k_i = L u^n + dt sum_{j<i} a_ij L k_j + dt sum_{j<i} ahat_ij L l_j
                             + q(t^n + c_i dt),                                  i = 2..s,
      l_i = g(u^n + dt sum_{j<=i} a_ij k_j + dt sum_{j<i} ahat_ij l_j),           i = 2..s,
      u^{n+1} = u^n + dt sum_j b_j k_j + dt sum_j bhat_j l_j   (at every node).

    Readings (the paper leaves them open):
      * k_i on the boundary is u_t there (fdot_stages, the time derivative of the Dirichlet
        data at t^n + c_i dt); l_i is 0 on the boundary (the paper assigns zero slope data
        when the boundary data do not depend on time, the only case it allows with g).
      * k_1 is an explicit equation: interior values L u^n + q, boundary values as above,
        interface values from the (penalised) flux condition, i.e. the identity equation
        solved on the tree (Sec. 3.1.1).  l_i is pointwise at interior and interface nodes.
      * The penalised condition replaces zero flux jump of each slope k_i by the jump
        -[[u^n]]/dt, [[.]] = flux_alpha - flux_beta of u^n.  Since sum_j b_j = 1 this makes
        u^{n+1} flux-continuous when g = 0 (the sign that achieves what the paragraph asks).
    """

    def __init__(self, hps, coefs_int, tab, dt, gpoly=None):
        self.hps = hps
        self.grid = hps.grid
        self.coefs = coefs_int
        self.tab = tableau_float(tab) if isinstance(tab["gamma"], Fr) else tab
        self.dt = float(dt)
        self.gpoly = gpoly
        if abs(self.tab["gamma"] * self.dt - hps.gamma_dt) > 1e-15 * abs(hps.gamma_dt):
            raise ValueError("operator was built for a different gamma*dt")
        self.iface = InterfaceSolver(self.grid)
        self.bnd = self.grid.boundary_indices()

    def step(self, u, q_stages=None, fdot_stages=None):
        """u: full N vector at t^n.  q_stages: (s, n_int) source at t^n + c_i dt (or None).
        fdot_stages: (s, n_bdry) time derivative of the Dirichlet data at t^n + c_i dt
        (or None = 0)."""
        g, tab, dt = self.grid, self.tab, self.dt
        s, n_int = tab["s"], g.n_int
        A, Ah, b, bh = tab["A"], tab["Ahat"], tab["b"], tab["bhat"]
        q_at = (lambda i: np.zeros(n_int)) if q_stages is None else (lambda i: q_stages[i])
        fd_at = (lambda i: np.zeros(len(self.bnd))) if fdot_stages is None else (lambda i: fdot_stages[i])
        L = lambda v: apply_L(g, self.coefs, v)
        penalty = -self.iface.jump(u) / dt
        Lun = L(u)

        def slope_l(v):
            w = poly_g(self.gpoly, v)
            w[self.bnd] = 0.0
            return w

        k1 = np.zeros(g.N)
        k1[:n_int] = Lun + q_at(0)
        k1[self.bnd] = fd_at(0)
        self.iface.fill(k1, penalty)
        k, l = [k1], [slope_l(u.copy())]
        Lk, Ll = [L(k1)], [L(l[0])]
        for i in range(1, s):
            rhs = Lun + q_at(i)
            for j in range(i):
                rhs = rhs + dt * A[i, j] * Lk[j] + dt * Ah[i, j] * Ll[j]
            ki = self.hps.solve(rhs, fd_at(i), penalty if len(self.iface.iface) else None)
            k.append(ki)
            Lk.append(L(ki))
            ui = u.copy()
            for j in range(i + 1):
                ui += dt * A[i, j] * k[j]
            for j in range(i):
                ui += dt * Ah[i, j] * l[j]
            l.append(slope_l(ui))
            Ll.append(L(l[i]))
        unew = u.copy()
        for j in range(s):
            unew += dt * b[j] * k[j] + dt * bh[j] * l[j]
        return unew
