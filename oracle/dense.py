"""The global collocation system of eq. (4), assembled node by node (oracle; test infrastructure only).

Sec. 2.1, eq. (4): one row per grid node.
  * interior node:          (A u)(x_i) = g_i, the PDE collocated with the
                            leaf's spectral derivatives;
  * edge node inside Omega: flux continuity across the edge, here written as
                            flux_alpha - flux_beta = r3 (r3 = 0 for the PDE),
                            with alpha the left/bottom leaf and the flux taken
                            in the coordinate direction (Sec. 2.1);
  * edge node on the boundary: u = f (Dirichlet data).
The HPS solver never forms this matrix; here it is formed and factorised to
give an independent route to the same discrete solution (Sec. 3.1.1 reports
the two agree to machine precision).  Entries are written out from the
one-dimensional derivative matrix with explicit loops, not through the leaf
operators of the HPS code.
"""
import numpy as np
import scipy.sparse as sp

from .cheb import leaf_diff_1d


def _add_pde_rows(grid, coefs_int, gamma_dt, rows, cols, vals):
    p, q = grid.p, grid.q
    D = leaf_diff_1d(grid.h, p)
    D2 = D @ D
    for j in range(grid.n2):
        for i in range(grid.n1):
            for b in range(1, q + 1):
                for a in range(1, q + 1):
                    r = grid.interior_index(i, j, a, b)
                    k = r  # coefficient arrays are indexed like the interior nodes
                    c11 = gamma_dt * coefs_int["cxx"][k]
                    c22 = gamma_dt * coefs_int["cyy"][k]
                    c1 = -gamma_dt * coefs_int["cx"][k]
                    c2 = -gamma_dt * coefs_int["cy"][k]
                    c = 1.0 - gamma_dt * coefs_int["c0"][k]
                    rows.append(r); cols.append(r); vals.append(c)
                    for m in range(p):
                        gx = grid.local_to_global(i, j, m, b)   # along x through (a, b)
                        gy = grid.local_to_global(i, j, a, m)   # along y through (a, b)
                        rows.append(r); cols.append(gx)
                        vals.append(-c11 * D2[a, m] + c1 * D[a, m])
                        rows.append(r); cols.append(gy)
                        vals.append(-c22 * D2[b, m] + c2 * D[b, m])


def flux_jump_matrix(grid):
    """Sparse (N x N) matrix whose row at an interface edge node gives
    flux_alpha(u) - flux_beta(u) there; zero rows elsewhere."""
    p, q = grid.p, grid.q
    D = leaf_diff_1d(grid.h, p)
    rows, cols, vals = [], [], []
    # vertical interface lines: alpha = leaf (k-1, j) on the left, beta = leaf (k, j)
    for k in range(1, grid.n1):
        for j in range(grid.n2):
            for b in range(1, q + 1):
                r = grid.vert_index(k, j, b)
                for m in range(p):
                    rows.append(r); cols.append(grid.local_to_global(k - 1, j, m, b))
                    vals.append(D[p - 1, m])
                    rows.append(r); cols.append(grid.local_to_global(k, j, m, b))
                    vals.append(-D[0, m])
    # horizontal interface lines: alpha = leaf (i, k-1) below, beta = leaf (i, k) above
    for k in range(1, grid.n2):
        for i in range(grid.n1):
            for a in range(1, q + 1):
                r = grid.horz_index(k, i, a)
                for m in range(p):
                    rows.append(r); cols.append(grid.local_to_global(i, k - 1, a, m))
                    vals.append(D[p - 1, m])
                    rows.append(r); cols.append(grid.local_to_global(i, k, a, m))
                    vals.append(-D[0, m])
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.N, grid.N))


def global_matrix(grid, coefs_int, gamma_dt):
    """Dense N x N matrix of eq. (4) for A = I - gamma_dt L with Dirichlet rows."""
    rows, cols, vals = [], [], []
    _add_pde_rows(grid, coefs_int, gamma_dt, rows, cols, vals)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(grid.N, grid.N)).toarray()
    A += flux_jump_matrix(grid).toarray()
    for g in grid.boundary_indices():
        A[g, g] = 1.0
    return A


def dense_solve(grid, coefs_int, gamma_dt, body, dirichlet=None, jump=None):
    """Solve the global system by dense LU (tiny grids only)."""
    if grid.N > 6000:
        raise ValueError("dense reference is for tiny grids")
    A = global_matrix(grid, coefs_int, gamma_dt)
    rhs = np.zeros(grid.N, dtype=np.result_type(A, np.asarray(body)))
    rhs[: grid.n_int] = body
    if dirichlet is not None:
        rhs[grid.boundary_indices()] = dirichlet
    if jump is not None:
        rhs[grid.interface_indices()] = jump
    return np.linalg.solve(A, rhs)
