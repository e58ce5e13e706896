"""Symmetric interior penalty DG Laplacian on Cartesian meshes of a cube.

Section 2.2, eq. (poisson_dgsip): with kappa = 1,

    (grad v, grad u)_T - <v n, (grad u^- + grad u^+)/2>_dT
                       - <grad v / 2, n (u^- - u^+)>_dT + <v, sigma (u^- - u^+)>_dT,

where <.,.>_dT runs over all faces of every cell, so each interior face is seen
from both sides with the outward normal n of the cell whose test function v is
used.  Eq. (bc_dgsip) gives the exterior values on the boundary:
Dirichlet u^+ = -u^- + 2 g_D, grad u^+ = grad u^-;
Neumann u^+ = u^-, grad u^+ . n = -grad u^- . n - 2 g_N (kappa = 1), with the paper's
g_N = -n . grad u the outward flux.  The operator holds the terms in the unknowns; the
data terms go to the right-hand side (boundary_data_load): on a Dirichlet face
int (2 sigma g_D v - g_D n . grad v), on a Neumann face int (n . grad u) v.
Which faces are Dirichlet is given as in mesh.Box: 'dirichlet' (all), 'neumann' (none),
'mixed' (the upper faces x_e = lo + length) or a face mask.

The penalty is sigma = c_pen (k+1)^2 / h; the paper's choice (k+1)^2 d / h is
c_pen = d = 3.  The basis is the Lagrange basis in the k+1 Gauss-Legendre points of
each direction; face integrals use the (k+1)^2-point Gauss rule on the face.

Layout: cell-major DG vector, DoF index = cell * n^3 + (i + n j + n^2 l), cells
lexicographic with x fastest.

The oracle transcribes the weak form face by face and cell by cell into dense
blocks (one block per (cell, face) pair) and assembles them into CSR.
"""
import numpy as np
import scipy.sparse as sp

from .basis import gauss_legendre, lagrange_derivatives, lagrange_values
from .cg import reference_tables, tensor_weights


class DGBox:
    """N_c^3 Cartesian cells of [lo, lo + length]^3 carrying the DG Q_k space."""

    def __init__(self, cells_per_dim, degree, c_pen=1.0, lo=0.0, length=1.0):
        self.Nc = int(cells_per_dim)
        self.k = int(degree)
        self.n = self.k + 1
        self.lo = float(lo)
        self.length = float(length)
        self.h = self.length / self.Nc
        self.c_pen = float(c_pen)
        self.sigma = self.c_pen * (self.k + 1) ** 2 / self.h
        self.n_cells = self.Nc ** 3
        self.n_dofs = self.n_cells * self.n ** 3
        self.nodes, self.weights = gauss_legendre(self.n)

    def neighbor(self, cell, d, s):
        """Cell across face (axis d, side s: 0 = low, 1 = high), or -1 on the boundary."""
        c = [cell % self.Nc, (cell // self.Nc) % self.Nc, cell // (self.Nc * self.Nc)]
        c[d] += 1 if s == 1 else -1
        if c[d] < 0 or c[d] >= self.Nc:
            return -1
        return c[0] + self.Nc * (c[1] + self.Nc * c[2])


def face_tables(nodes, points, d, xi_d):
    """Basis values and d/dxi_d derivatives at the tensor face points of the face
    xi_d = const; point index t1 + m t2 over the two other axes in increasing order."""
    n, m = len(nodes), len(points)
    V = lagrange_values(nodes, points)
    Vn = lagrange_values(nodes, [xi_d])[0]
    Dn = lagrange_derivatives(nodes, [xi_d])[0]
    tang = [a for a in range(3) if a != d]
    val = np.zeros((m * m, n ** 3))
    der = np.zeros((m * m, n ** 3))
    for i3 in range(n):
        for i2 in range(n):
            for i1 in range(n):
                idx = (i1, i2, i3)
                col = i1 + n * i2 + n * n * i3
                for t2 in range(m):
                    for t1 in range(m):
                        tv = V[t1, idx[tang[0]]] * V[t2, idx[tang[1]]]
                        val[t1 + m * t2, col] = tv * Vn[idx[d]]
                        der[t1 + m * t2, col] = tv * Dn[idx[d]]
    return val, der


def cell_matrix(dg):
    """(grad v, grad u) on one Cartesian cell of size h, Gauss quadrature k+1."""
    _, grad = reference_tables(dg.nodes, dg.nodes)
    w3 = tensor_weights(dg.weights)
    # J = h I: det J = h^3, physical gradient = grad_xi / h
    return dg.h * np.einsum("q,bqi,bqj->ij", w3, grad, grad)


def face_blocks(dg):
    """For each face (d, s): the block acting on the own cell's values (interior
    face), the block acting on the neighbour's values, and the own-cell block of a
    Dirichlet boundary face.  Rows are the own cell's test functions."""
    W = np.kron(dg.weights, dg.weights) * dg.h ** 2
    blocks = {}
    for d in range(3):
        for s in (0, 1):
            sign = 1.0 if s == 1 else -1.0            # outward normal = sign * e_d
            Vm, Gm = face_tables(dg.nodes, dg.nodes, d, float(s))
            Vp, Gp = face_tables(dg.nodes, dg.nodes, d, float(1 - s))
            Dm = sign * Gm / dg.h                       # n . grad phi^-
            Dp = sign * Gp / dg.h                       # n . grad phi^+ (same n)
            WV = W[:, None] * Vm
            WD = W[:, None] * Dm
            # -<v n, ({grad u})> - <grad v/2, n [u]> + <v, sigma [u]>
            own = -0.5 * WV.T @ Dm - 0.5 * WD.T @ Vm + dg.sigma * WV.T @ Vm
            nbr = -0.5 * WV.T @ Dp + 0.5 * WD.T @ Vp - dg.sigma * WV.T @ Vp
            # Dirichlet: u^+ = -u^-, n.grad u^+ = n.grad u^-
            dirichlet = -WV.T @ Dm - WD.T @ Vm + 2.0 * dg.sigma * WV.T @ Vm
            blocks[(d, s)] = (own, nbr, dirichlet)
    return blocks


def assemble(dg, bc="dirichlet"):
    """CSR matrix of the SIPG operator (bc: name or face mask of the Dirichlet faces)."""
    from .mesh import bc_mask
    m = bc_mask(bc)
    n3 = dg.n ** 3
    Ac = cell_matrix(dg)
    blocks = face_blocks(dg)
    rows, cols, vals = [], [], []
    loc = np.arange(n3)
    R = np.repeat(loc, n3)
    Cc = np.tile(loc, n3)
    for e in range(dg.n_cells):
        acc_own = Ac.copy()
        for (d, s), (own, nbr, dirichlet) in blocks.items():
            f = dg.neighbor(e, d, s)
            if f >= 0:
                acc_own += own
                rows.append(e * n3 + R)
                cols.append(f * n3 + Cc)
                vals.append(nbr.ravel())
            elif m & (1 << s):
                acc_own += dirichlet
        rows.append(e * n3 + R)
        cols.append(e * n3 + Cc)
        vals.append(acc_own.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dg.n_dofs, dg.n_dofs)).tocsr()
    A.sum_duplicates()
    return A


def apply_rows(dg, u, rows, bc="dirichlet"):
    """(A u)[rows], computed from the cell's own block and its six face blocks."""
    from .mesh import bc_mask
    m = bc_mask(bc)
    n3 = dg.n ** 3
    Ac = cell_matrix(dg)
    blocks = face_blocks(dg)
    y = np.zeros(len(rows))
    for t, r in enumerate(np.asarray(rows)):
        e, i = int(r) // n3, int(r) % n3
        ue = u[e * n3:(e + 1) * n3]
        acc = Ac[i] @ ue
        for (d, s), (own, nbr, dirichlet) in blocks.items():
            f = dg.neighbor(e, d, s)
            if f >= 0:
                acc += own[i] @ ue + nbr[i] @ u[f * n3:(f + 1) * n3]
            elif m & (1 << s):
                acc += dirichlet[i] @ ue
        y[t] = acc
    return y


def cell_points(dg):
    """Physical coordinates (n_cells, n^3, 3) of the Gauss points of every cell."""
    n = dg.n
    c = np.arange(dg.n_cells)
    cx, cy, cz = c % dg.Nc, (c // dg.Nc) % dg.Nc, c // (dg.Nc * dg.Nc)
    lx = np.tile(dg.nodes, n * n)
    ly = np.tile(np.repeat(dg.nodes, n), n)
    lz = np.repeat(dg.nodes, n * n)
    return dg.lo + np.stack([(cx[:, None] + lx) * dg.h, (cy[:, None] + ly) * dg.h,
                             (cz[:, None] + lz) * dg.h], axis=-1)


def rhs(dg, f):
    """b_i = (phi_i, f) with the (k+1)^3-point Gauss rule (homogeneous Dirichlet data)."""
    val, _ = reference_tables(dg.nodes, dg.nodes)
    w3 = tensor_weights(dg.weights) * dg.h ** 3
    fx = f(cell_points(dg))                       # (cells, Q)
    return np.einsum("eq,qi->ei", w3[None, :] * fx, val).ravel()


def l2_error(dg, u, exact, extra_points=2):
    """|| u_h - exact ||_{L2} with k+1+extra_points Gauss points per direction."""
    xq, wq = gauss_legendre(dg.n + extra_points)
    val, _ = reference_tables(dg.nodes, xq)
    w3 = tensor_weights(wq) * dg.h ** 3
    n = dg.n + extra_points
    c = np.arange(dg.n_cells)
    cx, cy, cz = c % dg.Nc, (c // dg.Nc) % dg.Nc, c // (dg.Nc * dg.Nc)
    P = dg.lo + np.stack([(cx[:, None] + np.tile(xq, n * n)) * dg.h,
                          (cy[:, None] + np.tile(np.repeat(xq, n), n)) * dg.h,
                          (cz[:, None] + np.repeat(xq, n * n)) * dg.h], axis=-1)
    uh = u.reshape(dg.n_cells, -1) @ val.T
    return float(np.sqrt(np.sum(w3[None, :] * (uh - exact(P)) ** 2)))


def boundary_data_load(dg, g_dirichlet, flux, bc="mixed"):
    """Right-hand side terms of the boundary data: on the Dirichlet faces of `bc`
    int (2 sigma g_D v - g_D n . grad v), on the other boundary faces int flux v, where
    g_dirichlet(x) and flux(x, normal) = n . grad u are evaluated at the (k+1)^2 Gauss
    points of each boundary face."""
    from .mesh import bc_mask
    m = bc_mask(bc)
    n3 = dg.n ** 3
    W = np.kron(dg.weights, dg.weights) * dg.h ** 2
    b = np.zeros(dg.n_dofs)
    Nc = dg.Nc
    c = np.arange(dg.n_cells)
    cc = [c % Nc, (c // Nc) % Nc, c // (Nc * Nc)]
    for d in range(3):
        tang = [a for a in range(3) if a != d]
        for s in (0, 1):
            sign = 1.0 if s == 1 else -1.0
            V, G = face_tables(dg.nodes, dg.nodes, d, float(s))
            Dn = sign * G / dg.h
            cells = c[cc[d] == (Nc - 1 if s else 0)]
            # face points: normal coordinate on the face, tangential at the Gauss points
            t1 = np.tile(dg.nodes, dg.n)
            t2 = np.repeat(dg.nodes, dg.n)
            X = np.zeros((len(cells), dg.n * dg.n, 3))
            X[:, :, d] = dg.lo + (cc[d][cells][:, None] + s) * dg.h
            X[:, :, tang[0]] = dg.lo + (cc[tang[0]][cells][:, None] + t1[None, :]) * dg.h
            X[:, :, tang[1]] = dg.lo + (cc[tang[1]][cells][:, None] + t2[None, :]) * dg.h
            normal = np.zeros(3)
            normal[d] = sign
            if m & (1 << s):
                g = g_dirichlet(X)
                be = (2.0 * dg.sigma * (W[None, :] * g)) @ V - (W[None, :] * g) @ Dn
            else:
                be = (W[None, :] * flux(X, normal)) @ V
            for j, e in enumerate(cells):
                b[e * n3:(e + 1) * n3] += be[j]
    return b
