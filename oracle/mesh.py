"""Structured hexahedral meshes of a cube and their degree-k node sets.

Section 2: elements are images of the reference cube under a polynomial map of
degree k whose support points are the Gauss-Lobatto nodes, placed by a manifold
description.  Here the manifold is the box [0,1]^3 deformed by

    Phi(X) = X + a * sin(pi X) sin(pi Y) sin(pi Z) * (1, 1, 1),

the same scalar added to each coordinate (a = 0: Cartesian mesh).  The map is the
identity on the boundary of the cube, so the physical domain stays [0,1]^3.  A
Cartesian box may also cover [lo, lo + length]^3 (the paper's smooth-solution example
uses (-1, 1)^3).

Boundary conditions are described per face by a mask: bit 0 set means the three
lower faces (x_e = lo) carry Dirichlet conditions, bit 1 the three upper faces
(x_e = lo + length); faces without Dirichlet conditions carry Neumann conditions.
'dirichlet' = 3, 'neumann' = 0, 'mixed' = 2 (the smooth-solution example: Neumann at
x_e = -1, Dirichlet at x_e = +1).

Numbering (shared with nothing; stated so that tests can compare layouts):
* cells lexicographic, x fastest: c = cx + Nc (cy + Nc cz);
* continuous DoFs lexicographic on the (k Nc + 1)^3 grid of per-cell GLL
  positions, x fastest;
* local cell DoFs lexicographic i + n j + n^2 l (n = k + 1), x fastest.
"""
import numpy as np

from .basis import gauss_lobatto


BC_MASKS = {"dirichlet": 3, "neumann": 0, "mixed": 2}


def bc_mask(bc):
    return BC_MASKS[bc] if isinstance(bc, str) else int(bc)


class Box:
    """N_c^3 cells of a cube carrying the continuous Q_k space."""

    def __init__(self, cells_per_dim, degree, curve_amp=0.0, lo=0.0, length=1.0):
        if cells_per_dim < 1 or degree < 1:
            raise ValueError("need at least one cell and degree >= 1")
        if curve_amp != 0.0 and (lo != 0.0 or length != 1.0):
            raise ValueError("the curved map is defined on the unit cube only")
        self.Nc = int(cells_per_dim)
        self.k = int(degree)
        self.n = self.k + 1
        self.N1 = self.k * self.Nc + 1
        self.lo = float(lo)
        self.length = float(length)
        self.h = self.length / self.Nc
        self.a = float(curve_amp)
        self.n_cells = self.Nc ** 3
        self.n_dofs = self.N1 ** 3
        self.gll, self.gll_w = gauss_lobatto(self.n)

    # ---- numbering ------------------------------------------------------
    def cell_coords(self, cells=None):
        c = np.arange(self.n_cells) if cells is None else np.asarray(cells)
        return c % self.Nc, (c // self.Nc) % self.Nc, c // (self.Nc * self.Nc)

    def cell_dofs(self, cells=None):
        """(len(cells), n^3) global DoF indices, local order i + n j + n^2 l."""
        cx, cy, cz = self.cell_coords(cells)
        n, k, N1 = self.n, self.k, self.N1
        i = np.arange(n)
        loc_x = np.tile(i, n * n)
        loc_y = np.tile(np.repeat(i, n), n)
        loc_z = np.repeat(i, n * n)
        gx = cx[:, None] * k + loc_x[None, :]
        gy = cy[:, None] * k + loc_y[None, :]
        gz = cz[:, None] * k + loc_z[None, :]
        return gx + N1 * (gy + N1 * gz)

    def boundary_mask(self, bc="dirichlet"):
        """DoFs on faces with Dirichlet conditions (bc: name or face mask)."""
        m = bc_mask(bc)
        g = np.arange(self.N1)
        b1 = ((g == 0) & bool(m & 1)) | ((g == self.N1 - 1) & bool(m & 2))
        bz, by, bx = np.meshgrid(b1, b1, b1, indexing="ij")
        return (bx | by | bz).ravel()

    def node_coords_1d(self):
        """Reference (undeformed) coordinate of each of the N1 grid lines."""
        g = np.arange(self.N1)
        c = np.minimum(g // self.k, self.Nc - 1)
        return self.lo + (c + self.gll[g - c * self.k]) * self.h

    # ---- geometry -------------------------------------------------------
    def deform(self, X):
        """Phi applied to points X[..., 3]."""
        X = np.asarray(X, dtype=np.float64)
        s = np.sin(np.pi * X[..., 0]) * np.sin(np.pi * X[..., 1]) * np.sin(np.pi * X[..., 2])
        return X + self.a * s[..., None]

    def dof_points(self):
        """Physical position of every continuous DoF, (N1^3, 3)."""
        x1 = self.node_coords_1d()
        Z, Y, X = np.meshgrid(x1, x1, x1, indexing="ij")
        P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
        return self.deform(P)

    def cell_node_coords(self, cells=None):
        """(len(cells), n^3, 3): the isoparametric support points of each cell."""
        cx, cy, cz = self.cell_coords(cells)
        n = self.n
        lx = np.tile(self.gll, n * n)
        ly = np.tile(np.repeat(self.gll, n), n)
        lz = np.repeat(self.gll, n * n)
        X = np.stack([self.lo + (cx[:, None] + lx[None, :]) * self.h,
                      self.lo + (cy[:, None] + ly[None, :]) * self.h,
                      self.lo + (cz[:, None] + lz[None, :]) * self.h], axis=-1)
        return self.deform(X)
