"""Continuous Q_k Laplacian: element matrices, assembly, right-hand side, errors.

Section 2.1, eq. (poisson_fem): the element stiffness matrix of (grad v, kappa grad u)
is assembled into the global matrix with Dirichlet rows and columns eliminated.
Section 3, eq. (mf_eval): the integral is evaluated with Gauss-Legendre quadrature,
k+1 points per direction, as

    A^e_ij = sum_q w_q det(J_q) kappa_e (J_q^{-T} grad_xi phi_i) . (J_q^{-T} grad_xi phi_j),

with J_q the Jacobian of the isoparametric map of the cell at quadrature point q.
The oracle forms every A^e as a dense matrix from all basis gradients at all
quadrature points (no sum factorization) and assembles it into CSR.

Dirichlet convention on the full-length vector: rows and columns of boundary DoFs
are removed and a unit diagonal put back, so the operator is the identity on
boundary DoFs and symmetric positive definite on the whole space.
"""
import numpy as np
import scipy.sparse as sp

from .basis import gauss_legendre, lagrange_derivatives, lagrange_values


def reference_tables(nodes, points):
    """Tensor-product basis values and reference gradients at tensor points.

    Returns (val[Q, n^3], grad[3, Q, n^3]) with point index q1 + m q2 + m^2 q3 and
    basis index i1 + n i2 + n^2 i3 (x fastest in both).
    """
    V = lagrange_values(nodes, points)
    D = lagrange_derivatives(nodes, points)
    val = np.kron(V, np.kron(V, V))
    gx = np.kron(V, np.kron(V, D))
    gy = np.kron(V, np.kron(D, V))
    gz = np.kron(D, np.kron(V, V))
    return val, np.stack([gx, gy, gz])


def tensor_weights(w):
    return np.kron(w, np.kron(w, w))


def cell_geometry(node_xyz, grad):
    """J[e, q, a, b] = d x_a / d xi_b = sum_i x_i[a] d phi_i / d xi_b at each point."""
    return np.einsum("eia,bqi->eqab", node_xyz, grad, optimize=True)


def element_matrices(box, kappa=None, cells=None, n_quad=None, kappa_fn=None):
    """Dense element stiffness matrices (len(cells), n^3, n^3), eq. (mf_eval).

    kappa: per-cell diffusion coefficient (None: 1).  kappa_fn: an optional coefficient
    of the position, evaluated at the physical image of every quadrature point and
    multiplied into the cell's kappa (the variable-coefficient case of Sec. 4.3).
    n_quad: Gauss points per direction (default k+1, the paper's choice).
    """
    cells = np.arange(box.n_cells) if cells is None else np.asarray(cells)
    m = box.n if n_quad is None else int(n_quad)
    xq, wq = gauss_legendre(m)
    val, grad = reference_tables(box.gll, xq)
    w3 = tensor_weights(wq)
    kap = np.ones(box.n_cells) if kappa is None else np.asarray(kappa, dtype=np.float64)
    n3 = box.n ** 3
    out = np.empty((len(cells), n3, n3))
    per_cell = 8 * len(w3) * n3 * 3 * 3
    chunk = max(1, int(2e8 // per_cell))
    for s in range(0, len(cells), chunk):
        cs = cells[s:s + chunk]
        X = box.cell_node_coords(cs)
        J = cell_geometry(X, grad)
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("inverted cell: det J <= 0")
        Jinv = np.linalg.inv(J)
        # physical gradients J^{-T} grad_xi phi_i: g[e,q,i,a] = sum_b Jinv[e,q,b,a] grad[b,q,i]
        g = np.einsum("eqba,bqi->eqia", Jinv, grad, optimize=True)
        wdet = w3[None, :] * det * kap[cs][:, None]
        if kappa_fn is not None:
            wdet = wdet * kappa_fn(np.einsum("qi,eia->eqa", val, X))
        # A^e_ij = sum_q sum_a wdet[e,q] g[e,q,i,a] g[e,q,j,a], formed as one batched matrix
        # product over the combined index (q, a)
        E, Q = g.shape[0], g.shape[1]
        left = (g * wdet[:, :, None, None]).transpose(0, 2, 1, 3).reshape(E, n3, Q * 3)
        right = g.transpose(0, 1, 3, 2).reshape(E, Q * 3, n3)
        out[s:s + len(cs)] = np.matmul(left, right)
    return out


def assemble(box, kappa=None, bc="dirichlet", n_quad=None, kappa_fn=None):
    """Global CSR matrix.  Identity rows/columns on the DoFs of the Dirichlet faces of
    `bc` ('dirichlet': all faces, 'mixed': the upper faces, or a face mask); 'neumann':
    the plain assembled matrix (natural conditions everywhere)."""
    Ae = element_matrices(box, kappa, n_quad=n_quad, kappa_fn=kappa_fn)
    dofs = box.cell_dofs()
    n3 = box.n ** 3
    rows = np.repeat(dofs, n3, axis=1).ravel()
    cols = np.tile(dofs, (1, n3)).ravel()
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(box.n_dofs, box.n_dofs)).tocsr()
    A.sum_duplicates()
    dmask = box.boundary_mask(bc)
    if not dmask.any():
        return A
    keep = sp.diags((~dmask).astype(np.float64))
    bnd = sp.diags(dmask.astype(np.float64))
    return (keep @ A @ keep + bnd).tocsr()


def cells_of_dof(box, dof):
    """Cells whose closure contains the continuous DoF `dof`."""
    N1, k, Nc = box.N1, box.k, box.Nc
    g = (dof % N1, (dof // N1) % N1, dof // (N1 * N1))
    ranges = []
    for gi in g:
        c = {min(gi // k, Nc - 1)}
        if gi % k == 0 and 0 < gi < N1 - 1:
            c.add(gi // k - 1)
        ranges.append(sorted(c))
    return [cx + Nc * (cy + Nc * cz) for cz in ranges[2] for cy in ranges[1] for cx in ranges[0]]


def apply_rows(box, u, rows, kappa=None, bc="dirichlet", kappa_fn=None):
    """(A u)[rows] with the operator of `assemble` (same bc), element by element.

    Used at sizes where the CSR matrix does not fit: each requested row is the
    sum over the cells containing that DoF of the corresponding row of A^e times
    the cell's (Dirichlet-zeroed) values.
    """
    rows = np.asarray(rows)
    bmask = box.boundary_mask(bc)
    cell_lists = [cells_of_dof(box, int(r)) for r in rows]
    uniq = np.unique(np.concatenate([np.asarray(c) for c in cell_lists]))
    Ae = element_matrices(box, kappa, cells=uniq, kappa_fn=kappa_fn)
    dofs = box.cell_dofs(uniq)
    where = {int(c): i for i, c in enumerate(uniq)}
    uz = np.where(bmask, 0.0, u)
    y = np.zeros(len(rows))
    for t, r in enumerate(rows):
        if bmask[r]:
            y[t] = u[r]
            continue
        for c in cell_lists[t]:
            e = where[c]
            loc = int(np.nonzero(dofs[e] == r)[0][0])
            y[t] += Ae[e, loc] @ uz[dofs[e]]
    return y


def cosine_coefficient(amp=1e6):
    """The strongly varying coefficient of Sec. 4.3, eq. (diffusivity_shell), read with
    each cosine factor squared so that it is positive (as printed, 1 + 10^6 times the
    product of the cosines changes sign, which no diffusion coefficient may):
        kappa(x) = 1 + amp * prod_{e=1..3} cos^2(2 pi x_e + 0.1 e).
    Returns the function of positions x[..., 3]."""
    def kappa(x):
        p = np.ones(x.shape[:-1])
        for e in range(3):
            p = p * np.cos(2.0 * np.pi * x[..., e] + 0.1 * (e + 1)) ** 2
        return 1.0 + amp * p
    return kappa


def sine_solution(x):
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])


def sine_forcing(x):
    """f = -Laplace(u) for u = sin(pi x) sin(pi y) sin(pi z)."""
    return 3.0 * np.pi ** 2 * sine_solution(x)


def rhs(box, f=sine_forcing, n_quad=None, zero_boundary=True):
    """b_i = sum_e sum_q w_q det J_q f(x_q) phi_i(xi_q), zero on the Dirichlet boundary
    (homogeneous Dirichlet data) unless zero_boundary is False.

    x_q is the isoparametric image of the Gauss point; k+1 points by default.
    """
    m = box.n if n_quad is None else int(n_quad)
    xq, wq = gauss_legendre(m)
    val, grad = reference_tables(box.gll, xq)
    w3 = tensor_weights(wq)
    b = np.zeros(box.n_dofs)
    chunk = 4096
    for s in range(0, box.n_cells, chunk):
        cs = np.arange(s, min(s + chunk, box.n_cells))
        X = box.cell_node_coords(cs)
        det = np.linalg.det(cell_geometry(X, grad))
        xphys = np.einsum("qi,eia->eqa", val, X)
        be = np.einsum("eq,qi->ei", w3[None, :] * det * f(xphys), val)
        np.add.at(b, box.cell_dofs(cs).ravel(), be.ravel())
    if zero_boundary:
        b[box.boundary_mask()] = 0.0
    return b


def interpolate(box, fn):
    """Nodal interpolant: u_i = fn(x_i) at the physical DoF positions."""
    return fn(box.dof_points())


def l2_norm(box, fn, extra_points=2):
    """|| fn ||_{L2} over the mesh with k+1+extra_points Gauss points per direction."""
    xq, wq = gauss_legendre(box.n + extra_points)
    val, grad = reference_tables(box.gll, xq)
    w3 = tensor_weights(wq)
    s2 = 0.0
    chunk = 2048
    for s in range(0, box.n_cells, chunk):
        cs = np.arange(s, min(s + chunk, box.n_cells))
        X = box.cell_node_coords(cs)
        det = np.linalg.det(cell_geometry(X, grad))
        xphys = np.einsum("qi,eia->eqa", val, X)
        s2 += np.sum(w3[None, :] * det * fn(xphys) ** 2)
    return float(np.sqrt(s2))


def l2_error(box, u, exact=sine_solution, extra_points=2):
    """|| u_h - exact ||_{L2} with k+1+extra_points Gauss points per direction."""
    xq, wq = gauss_legendre(box.n + extra_points)
    val, grad = reference_tables(box.gll, xq)
    w3 = tensor_weights(wq)
    err2 = 0.0
    chunk = 2048
    for s in range(0, box.n_cells, chunk):
        cs = np.arange(s, min(s + chunk, box.n_cells))
        X = box.cell_node_coords(cs)
        det = np.linalg.det(cell_geometry(X, grad))
        xphys = np.einsum("qi,eia->eqa", val, X)
        uh = u[box.cell_dofs(cs)] @ val.T
        err2 += np.sum(w3[None, :] * det * (uh - exact(xphys)) ** 2)
    return float(np.sqrt(err2))
