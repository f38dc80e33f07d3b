"""Chebyshev-Lobatto collocation on one leaf (oracle; test infrastructure only).

Sec. 2.1 discretises every leaf square with p x p Chebyshev nodes and builds
"spectral differentiation operators" on them; Sec. 4.1 states the node
formula x_j = cos(j pi / (p - 1)) on [-1, 1].  The derivative matrix here is
the textbook Chebyshev-Gauss-Lobatto collocation derivative (the exact
derivative of the degree p-1 interpolant), written out entry by entry.
"""
import numpy as np


def cheb_points(p):
    """Reference nodes xi_m = cos(m pi / (p-1)), m = 0..p-1 (Sec. 4.1)."""
    if p < 2:
        raise ValueError("p must be >= 2")
    m = np.arange(p, dtype=np.float64)
    return np.cos(np.pi * m / (p - 1))


def cheb_diff_ref(p):
    """Derivative matrix on the reference nodes xi_m (descending order).

    Off-diagonal: D[i, j] = (k_i / k_j) (-1)^(i+j) / (xi_i - xi_j) with
    k_0 = k_{p-1} = 2 and k_m = 1 otherwise.  Diagonal: the negative row sum,
    so that the derivative of a constant is exactly zero.
    """
    xi = cheb_points(p)
    kap = np.ones(p)
    kap[0] = 2.0
    kap[-1] = 2.0
    D = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            if i != j:
                D[i, j] = (kap[i] / kap[j]) * (-1.0) ** (i + j) / (xi[i] - xi[j])
    for i in range(p):
        D[i, i] = -np.sum(D[i, :i]) - np.sum(D[i, i + 1:])
    return D


def leaf_points_1d(a, h, p):
    """Physical nodes on [a, a+h]: x_m = a + h (1 - xi_m) / 2, ascending in m."""
    return a + h * (1.0 - cheb_points(p)) / 2.0


def leaf_diff_1d(h, p):
    """d/dx on the physical nodes of a leaf of side h.

    x = a + h (1 - xi) / 2 gives dxi/dx = -2/h, so D_x = (-2/h) D_xi with the
    same node indexing m.
    """
    return (-2.0 / h) * cheb_diff_ref(p)
