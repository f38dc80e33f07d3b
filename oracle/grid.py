"""Corner-free collocation grid and canonical numbering (oracle; test infrastructure only).

Sec. 2.1: the rectangle is split into n1 x n2 equal squares, each carrying
p x p Chebyshev nodes; corner nodes of every square are dropped because no
collocation row references them when c12 = 0.  The node count is
N = (p-2)(p n1 n2 + n1 + n2).

Canonical order (shared with the library's external interface):
  1. leaf interiors: leaf (i, j) in row-major order (index j*n1 + i), then the
     (p-2)^2 interior nodes of the leaf row-major with x fastest;
  2. vertical edges: grid line k = 0..n1, then leaf row j, then node
     ascending in y;
  3. horizontal edges: grid line k = 0..n2, then leaf column i, then node
     ascending in x.
Local node (a, b) on a leaf means the a-th node in x and b-th node in y,
a, b in 0..p-1 ascending.
"""
import numpy as np

from .cheb import leaf_points_1d


class Grid:
    def __init__(self, x0, x1, y0, y1, n1, n2, p):
        self.x0, self.x1, self.y0, self.y1 = float(x0), float(x1), float(y0), float(y1)
        self.n1, self.n2, self.p = int(n1), int(n2), int(p)
        if self.p < 3:
            raise ValueError("p must be >= 3")
        self.h = (self.x1 - self.x0) / self.n1
        hy = (self.y1 - self.y0) / self.n2
        if abs(self.h - hy) > 1e-14 * max(1.0, abs(self.h)):
            raise ValueError("leaves must be square")
        self.q = self.p - 2
        q = self.q
        self.n_int = self.n1 * self.n2 * q * q
        self.n_vert = (self.n1 + 1) * self.n2 * q
        self.n_horz = (self.n2 + 1) * self.n1 * q
        self.n_edge = self.n_vert + self.n_horz
        self.N = self.n_int + self.n_edge

    # ---- global index of a local node -------------------------------------------------
    def interior_index(self, i, j, a, b):
        q = self.q
        return ((j * self.n1 + i) * q + (b - 1)) * q + (a - 1)

    def vert_index(self, k, j, b):
        """Vertical grid line k, leaf row j, local y index b in 1..q."""
        return self.n_int + (k * self.n2 + j) * self.q + (b - 1)

    def horz_index(self, k, i, a):
        """Horizontal grid line k, leaf column i, local x index a in 1..q."""
        return self.n_int + self.n_vert + (k * self.n1 + i) * self.q + (a - 1)

    def local_to_global(self, i, j, a, b):
        """Global index of local node (a, b) of leaf (i, j); None for a corner."""
        p = self.p
        on_x = a in (0, p - 1)
        on_y = b in (0, p - 1)
        if on_x and on_y:
            return None
        if not on_x and not on_y:
            return self.interior_index(i, j, a, b)
        if on_x:
            return self.vert_index(i if a == 0 else i + 1, j, b)
        return self.horz_index(j if b == 0 else j + 1, i, a)

    # ---- node classes ----------------------------------------------------------------
    def boundary_mask(self):
        """True for edge nodes on the outer boundary, over all N nodes."""
        m = np.zeros(self.N, dtype=bool)
        q = self.q
        for k in (0, self.n1):
            for j in range(self.n2):
                for b in range(1, q + 1):
                    m[self.vert_index(k, j, b)] = True
        for k in (0, self.n2):
            for i in range(self.n1):
                for a in range(1, q + 1):
                    m[self.horz_index(k, i, a)] = True
        return m

    def boundary_indices(self):
        """Global indices of the outer-boundary nodes, in canonical order."""
        return np.nonzero(self.boundary_mask())[0]

    def interface_indices(self):
        """Global indices of the edge nodes not on the outer boundary, canonical order."""
        m = self.boundary_mask()
        m[: self.n_int] = True
        return np.nonzero(~m)[0]

    # ---- coordinates -----------------------------------------------------------------
    def coordinates(self):
        x = np.full(self.N, np.nan)
        y = np.full(self.N, np.nan)
        p = self.p
        for j in range(self.n2):
            for i in range(self.n1):
                xs = leaf_points_1d(self.x0 + i * self.h, self.h, p)
                ys = leaf_points_1d(self.y0 + j * self.h, self.h, p)
                for b in range(p):
                    for a in range(p):
                        g = self.local_to_global(i, j, a, b)
                        if g is not None:
                            x[g] = xs[a]
                            y[g] = ys[b]
        return x, y
