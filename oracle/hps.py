"""HPS build and solve, written from the paper (oracle; test infrastructure only).

Problem (Sec. 2, eqs. 2-3): A u = g in Omega, u = f on the boundary, with
  A u = -c11 u_xx - c22 u_yy + c1 u_x + c2 u_y + c u      (c12 = 0).
For an implicit ESDIRK stage the operator is A = I - gamma*dt*L (eq. 10),
where L u = cxx u_xx + cyy u_yy + cx u_x + cy u_y + c0 u, so that
  c11 = gdt*cxx, c22 = gdt*cyy, c1 = -gdt*cx, c2 = -gdt*cy, c = 1 - gdt*c0.

Leaf (eqs. 5-6): A_ii u_i + A_ib u_b = g_i, S = -A_ii^{-1} A_ib, and the DtN
map T gives the coordinate-direction flux (d/dx on vertical edges, d/dy on
horizontal edges) on the leaf boundary.  The printed "T = D S" is read as the
flux rows applied to the whole tile [S u_b ; u_b].

Merge (eqs. 7-8 and the formulas after them):
  S_tau = (T^a_33 - T^b_33)^{-1} [ -T^a_31 | T^b_32 ],
  T_tau = diag(T^a_11, T^b_22) + [T^a_13 ; T^b_23] S_tau.
The beta blocks printed with an alpha superscript in eq. (7) are read as beta.

Body load and interface jump (not printed; the paper defers to a book).  They
follow from the same flux-continuity condition the merge uses: each child
obeys v = T u_b + h with h the flux of its particular solution (zero boundary
data), and on J3 the condition flux_alpha - flux_beta = r3 gives
  u_3 = S_tau u_12 + w_3,   w_3 = (T^a_33 - T^b_33)^{-1} (h^b_3 - h^a_3 + r3),
  h_tau = [ h^a_1 + T^a_13 w_3 ; h^b_2 + T^b_23 w_3 ].
r3 = 0 for the plain elliptic solve.  The downward sweep is Algorithm 1 with
the particular parts added: root boundary <- f, u_3 = S u_12 + w_3 at every
node, and u_i = S_leaf u_b + w on every leaf.

Linear systems are solved with LU factorisations kept from the build (the
build-once / solve-many structure of Sec. 3.1); nothing is inverted
explicitly.
"""
import numpy as np
import scipy.linalg as sla

from .cheb import leaf_diff_1d


# ---------------------------------------------------------------------------------------
# leaf
# ---------------------------------------------------------------------------------------
def leaf_index_sets(p):
    """Local flat index f = b*p + a of the interior nodes (row-major, x fastest) and of
    the leaf boundary in the order [left (y asc), right (y asc), bottom (x asc), top (x asc)]."""
    q = p - 2
    Ji = [b * p + a for b in range(1, q + 1) for a in range(1, q + 1)]
    left = [b * p + 0 for b in range(1, q + 1)]
    right = [b * p + (p - 1) for b in range(1, q + 1)]
    bottom = [0 * p + a for a in range(1, q + 1)]
    top = [(p - 1) * p + a for a in range(1, q + 1)]
    return np.array(Ji), np.array(left + right + bottom + top)


def tile_operators(h, p):
    """Full-tile x- and y-derivative matrices for the flat index b*p + a."""
    D = leaf_diff_1d(h, p)
    I = np.eye(p)
    Dx = np.kron(I, D)   # (Dx u)[b*p+a] = sum_m D[a,m] u[b*p+m]
    Dy = np.kron(D, I)   # (Dy u)[b*p+a] = sum_m D[b,m] u[m*p+a]
    return Dx, Dy


def leaf_matrix(h, p, coefs, gamma_dt):
    """Rows of A = I - gdt*L at the leaf's interior nodes, over all p*p tile nodes.

    coefs: dict with arrays cxx, cyy, cx, cy, c0 of length q*q (interior order).
    """
    Dx, Dy = tile_operators(h, p)
    Dxx = Dx @ Dx
    Dyy = Dy @ Dy
    Ji, _ = leaf_index_sets(p)
    c11 = gamma_dt * coefs["cxx"]
    c22 = gamma_dt * coefs["cyy"]
    c1 = -gamma_dt * coefs["cx"]
    c2 = -gamma_dt * coefs["cy"]
    c = 1.0 - gamma_dt * coefs["c0"]
    E = np.eye(p * p)[Ji]
    A = (c[:, None] * E - c11[:, None] * Dxx[Ji] - c22[:, None] * Dyy[Ji]
         + c1[:, None] * Dx[Ji] + c2[:, None] * Dy[Ji])
    return A


def flux_rows(h, p):
    """Rows giving the coordinate-direction flux on the leaf boundary (order as Jb)."""
    Dx, Dy = tile_operators(h, p)
    q = p - 2
    rows = [Dx[b * p + 0] for b in range(1, q + 1)]
    rows += [Dx[b * p + (p - 1)] for b in range(1, q + 1)]
    rows += [Dy[0 * p + a] for a in range(1, q + 1)]
    rows += [Dy[(p - 1) * p + a] for a in range(1, q + 1)]
    return np.array(rows)


class Leaf:
    def __init__(self, grid, i, j, coefs, gamma_dt):
        p = grid.p
        self.i, self.j = i, j
        self.is_leaf = True
        Ji, Jb = leaf_index_sets(p)
        A = leaf_matrix(grid.h, p, coefs, gamma_dt)
        self.A_ii = A[:, Ji]
        self.A_ib = A[:, Jb]
        self.lu = sla.lu_factor(self.A_ii)
        self.S = -sla.lu_solve(self.lu, self.A_ib)
        F = flux_rows(grid.h, p)
        self.F_i = F[:, Ji]
        self.F_b = F[:, Jb]
        self.T = self.F_i @ self.S + self.F_b
        # global indices of the interior nodes and of the boundary, in the leaf's order
        self.int_glob = np.array([grid.local_to_global(i, j, f % p, f // p) for f in Ji])
        self.bnd = np.array([grid.local_to_global(i, j, f % p, f // p) for f in Jb])
        self.box = (i, i + 1, j, j + 1)


# ---------------------------------------------------------------------------------------
# tree and merge
# ---------------------------------------------------------------------------------------
class Node:
    """Internal node tau with children alpha (left/bottom) and beta (right/top)."""

    def __init__(self, alpha, beta, is_root):
        self.is_leaf = False
        self.alpha, self.beta = alpha, beta
        a_pos = {g: k for k, g in enumerate(alpha.bnd)}
        b_pos = {g: k for k, g in enumerate(beta.bnd)}
        shared = set(alpha.bnd) & set(beta.bnd)
        self.J3 = np.array([g for g in alpha.bnd if g in shared])
        self.J1 = np.array([g for g in alpha.bnd if g not in shared])
        self.J2 = np.array([g for g in beta.bnd if g not in shared])
        self.a1 = np.array([a_pos[g] for g in self.J1], dtype=int)
        self.a3 = np.array([a_pos[g] for g in self.J3], dtype=int)
        self.b2 = np.array([b_pos[g] for g in self.J2], dtype=int)
        self.b3 = np.array([b_pos[g] for g in self.J3], dtype=int)
        self.bnd = np.concatenate([self.J1, self.J2])
        Ta, Tb = alpha.T, beta.T
        Ta11 = Ta[np.ix_(self.a1, self.a1)]
        Ta13 = Ta[np.ix_(self.a1, self.a3)]
        Ta31 = Ta[np.ix_(self.a3, self.a1)]
        Ta33 = Ta[np.ix_(self.a3, self.a3)]
        Tb22 = Tb[np.ix_(self.b2, self.b2)]
        Tb23 = Tb[np.ix_(self.b2, self.b3)]
        Tb32 = Tb[np.ix_(self.b3, self.b2)]
        Tb33 = Tb[np.ix_(self.b3, self.b3)]
        self.Ta13, self.Tb23 = Ta13, Tb23
        self.lu = sla.lu_factor(Ta33 - Tb33)
        self.S = sla.lu_solve(self.lu, np.hstack([-Ta31, Tb32]))
        if is_root:
            self.T = None
        else:
            n1, n2 = len(self.J1), len(self.J2)
            Td = np.zeros((n1 + n2, n1 + n2), dtype=np.result_type(Ta11, Tb22))
            Td[:n1, :n1] = Ta11
            Td[n1:, n1:] = Tb22
            self.T = Td + np.vstack([Ta13, Tb23]) @ self.S
        ai0, ai1, aj0, aj1 = alpha.box
        bi0, bi1, bj0, bj1 = beta.box
        self.box = (min(ai0, bi0), max(ai1, bi1), min(aj0, bj0), max(aj1, bj1))
        # the children's DtN maps are not needed once the parent is merged
        alpha.T = None
        beta.T = None


def _split(i0, i1, j0, j1):
    """Halve the longer side of a box of leaves; ties are cut vertically (Sec. 2.1)."""
    if (i1 - i0) >= (j1 - j0):
        im = (i0 + i1) // 2
        return (i0, im, j0, j1), (im, i1, j0, j1)
    jm = (j0 + j1) // 2
    return (i0, i1, j0, jm), (i0, i1, jm, j1)


class HPS:
    """Build (once) and solve (many times) for A = I - gamma_dt * L on a Grid."""

    def __init__(self, grid, coefs_int, gamma_dt):
        """coefs_int: dict of arrays cxx, cyy, cx, cy, c0 over the n_int interior nodes
        in canonical order."""
        n1, n2 = grid.n1, grid.n2
        if n1 & (n1 - 1) or n2 & (n2 - 1):
            raise ValueError("n1 and n2 must be powers of two")
        self.grid = grid
        self.gamma_dt = float(gamma_dt)
        # complex coefficients (Sec. 5.5) give complex operators; real ones stay FP64
        self.dtype = np.result_type(np.float64, *[np.asarray(v) for v in coefs_int.values()])
        q2 = grid.q * grid.q
        self.leaves = {}

        def build(box, is_root):
            i0, i1, j0, j1 = box
            if i1 - i0 == 1 and j1 - j0 == 1:
                k = j0 * n1 + i0
                c = {name: np.asarray(v, dtype=np.result_type(v, np.float64))[k * q2:(k + 1) * q2]
                     for name, v in coefs_int.items()}
                leaf = Leaf(grid, i0, j0, c, gamma_dt)
                self.leaves[(i0, j0)] = leaf
                return leaf
            ba, bb = _split(*box)
            alpha = build(ba, False)
            beta = build(bb, False)
            return Node(alpha, beta, is_root)

        self.root = build((0, n1, 0, n2), True)
        self.bnd_idx = grid.boundary_indices()
        self.iface_idx = grid.interface_indices()

    def solve(self, body, dirichlet=None, jump=None):
        """Solve A u = body (interior), u = dirichlet on the outer boundary, and
        flux_alpha - flux_beta = jump on interface edge nodes.  Returns u over all N
        nodes in canonical order."""
        g = self.grid
        dt = np.result_type(self.dtype, *[np.asarray(v) for v in (body, dirichlet, jump) if v is not None])
        body = np.asarray(body, dtype=dt)
        r3 = np.zeros(g.N, dtype=dt)
        if jump is not None:
            r3[self.iface_idx] = jump
        u = np.zeros(g.N, dtype=dt)
        if dirichlet is not None:
            u[self.bnd_idx] = dirichlet
        if isinstance(self.root, Leaf):
            leaf = self.root
            w = sla.lu_solve(leaf.lu, body[leaf.int_glob])
            u[leaf.int_glob] = leaf.S @ u[leaf.bnd] + w
            return u
        w_store = {}

        def up(node):
            if node.is_leaf:
                w = sla.lu_solve(node.lu, body[node.int_glob])
                w_store[id(node)] = w
                return node.F_i @ w
            ha = up(node.alpha)
            hb = up(node.beta)
            d = hb[node.b3] - ha[node.a3] + r3[node.J3]
            w3 = sla.lu_solve(node.lu, d)
            w_store[id(node)] = w3
            return np.concatenate([ha[node.a1] + node.Ta13 @ w3,
                                   hb[node.b2] + node.Tb23 @ w3])

        def down(node):
            if node.is_leaf:
                u[node.int_glob] = node.S @ u[node.bnd] + w_store[id(node)]
                return
            u[node.J3] = node.S @ u[node.bnd] + w_store[id(node)]
            down(node.alpha)
            down(node.beta)

        up(self.root)
        down(self.root)
        return u
