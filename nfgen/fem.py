"""Bilinear (Q1) and trilinear (Q1 hex) finite elements on structured boxes.

Only what the synthetic workloads need: shape functions and their gradients
at 2x2 / 2x2x2 Gauss points, constant-coefficient element matrices, and a
COO-based assembler that keeps the full element pattern (explicit zeros that
come out of assembly are kept, so the sparsity pattern is a function of the
mesh alone).
"""
import numpy as np
import scipy.sparse as sp

_G = 1.0 / np.sqrt(3.0)


def q1_2d(hx, hy):
    """Gauss data of a Q1 quad of size hx*hy.

    Local node order: (0,0), (1,0), (1,1), (0,1).
    Returns N[q,a], dN[q,a,dim], w[q] (weights times Jacobian).
    """
    xa = np.array([-1, 1, 1, -1], float)
    ya = np.array([-1, -1, 1, 1], float)
    pts = [(-_G, -_G), (_G, -_G), (_G, _G), (-_G, _G)]
    N = np.zeros((4, 4))
    dN = np.zeros((4, 4, 2))
    for q, (xi, eta) in enumerate(pts):
        N[q] = 0.25 * (1 + xa * xi) * (1 + ya * eta)
        dN[q, :, 0] = 0.25 * xa * (1 + ya * eta) * (2.0 / hx)
        dN[q, :, 1] = 0.25 * ya * (1 + xa * xi) * (2.0 / hy)
    w = np.full(4, hx * hy / 4.0)
    return N, dN, w


def q1_3d(hx, hy, hz):
    """Gauss data of a trilinear hex of size hx*hy*hz.

    Local node order: bottom face (z=0) counter-clockwise from the origin,
    then the top face in the same order.
    """
    xa = np.array([-1, 1, 1, -1, -1, 1, 1, -1], float)
    ya = np.array([-1, -1, 1, 1, -1, -1, 1, 1], float)
    za = np.array([-1, -1, -1, -1, 1, 1, 1, 1], float)
    pts = [(xa[i] * _G, ya[i] * _G, za[i] * _G) for i in range(8)]
    N = np.zeros((8, 8))
    dN = np.zeros((8, 8, 3))
    for q, (xi, eta, zeta) in enumerate(pts):
        N[q] = 0.125 * (1 + xa * xi) * (1 + ya * eta) * (1 + za * zeta)
        dN[q, :, 0] = 0.125 * xa * (1 + ya * eta) * (1 + za * zeta) * (2.0 / hx)
        dN[q, :, 1] = 0.125 * ya * (1 + xa * xi) * (1 + za * zeta) * (2.0 / hy)
        dN[q, :, 2] = 0.125 * za * (1 + xa * xi) * (1 + ya * eta) * (2.0 / hz)
    w = np.full(8, hx * hy * hz / 8.0)
    return N, dN, w


def elasticity_matrix(dim, E, nu, plane_strain=True):
    """Isotropic constitutive matrix in Voigt order (xx, yy[, zz], xy[, yz, zx])."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    if dim == 2:
        return np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] = lam + 2 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    return D


def strain_matrix(dNq):
    """B (nvoigt x nen*dim) at one Gauss point, dofs interleaved per node."""
    nen, dim = dNq.shape
    if dim == 2:
        B = np.zeros((3, 2 * nen))
        B[0, 0::2] = dNq[:, 0]
        B[1, 1::2] = dNq[:, 1]
        B[2, 0::2] = dNq[:, 1]
        B[2, 1::2] = dNq[:, 0]
        return B
    B = np.zeros((6, 3 * nen))
    B[0, 0::3] = dNq[:, 0]
    B[1, 1::3] = dNq[:, 1]
    B[2, 2::3] = dNq[:, 2]
    B[3, 0::3] = dNq[:, 1]
    B[3, 1::3] = dNq[:, 0]
    B[4, 1::3] = dNq[:, 2]
    B[4, 2::3] = dNq[:, 1]
    B[5, 0::3] = dNq[:, 2]
    B[5, 2::3] = dNq[:, 0]
    return B


def ke_elastic(gauss, E, nu):
    N, dN, w = gauss
    dim = dN.shape[2]
    D = elasticity_matrix(dim, E, nu)
    K = 0.0
    for q in range(len(w)):
        B = strain_matrix(dN[q])
        K = K + w[q] * B.T @ D @ B
    return K


def ke_laplace(gauss, kappa=1.0):
    N, dN, w = gauss
    return kappa * np.einsum("q,qad,qbd->ab", w, dN, dN)


def ke_mass(gauss):
    N, dN, w = gauss
    return np.einsum("q,qa,qb->ab", w, N, N)


def ke_grad_shape(gauss):
    """G[(a,c), b] = int dN_a/dx_c N_b  (vector dofs interleaved per node)."""
    N, dN, w = gauss
    nen, dim = dN.shape[1], dN.shape[2]
    G = np.einsum("q,qac,qb->acb", w, dN, N)
    return G.reshape(nen * dim, nen)


def grid_conn_2d(nx, ny):
    """Element -> node connectivity of an nx*ny quad grid, node id = j*(nx+1)+i."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    n0 = j * (nx + 1) + i
    return np.stack([n0, n0 + 1, n0 + nx + 2, n0 + nx + 1], axis=1)


def grid_conn_3d(nx, ny, nz):
    """Hex grid connectivity, node id = (k*(ny+1)+j)*(nx+1)+i."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    sx = 1
    sy = nx + 1
    sz = (nx + 1) * (ny + 1)
    n0 = k * sz + j * sy + i
    bot = [n0, n0 + sx, n0 + sx + sy, n0 + sy]
    top = [b + sz for b in bot]
    return np.stack(bot + top, axis=1)


def element_dofs(conn, ncomp):
    """Interleaved dof ids per element: dof = node*ncomp + comp."""
    nel, nen = conn.shape
    return (conn[:, :, None] * ncomp + np.arange(ncomp)[None, None, :]).reshape(nel, nen * ncomp)


def assemble(rows_e, cols_e, Ke, nrows, ncols, row_map=None, col_map=None):
    """Sum element matrices into CSR.

    rows_e (nel, a), cols_e (nel, b) are global ids; Ke is (a, b) (same for all
    elements) or (nel, a, b).  row_map/col_map renumber ids (-1 = eliminated).
    Explicit zeros are kept; columns are sorted.
    """
    nel = rows_e.shape[0]
    R = np.broadcast_to(rows_e[:, :, None], (nel, rows_e.shape[1], cols_e.shape[1]))
    C = np.broadcast_to(cols_e[:, None, :], R.shape)
    V = np.broadcast_to(Ke, R.shape) if Ke.ndim == 2 else Ke
    R = R.ravel()
    C = C.ravel()
    V = np.ascontiguousarray(V).ravel()
    if row_map is not None:
        R = row_map[R]
    if col_map is not None:
        C = col_map[C]
    keep = (R >= 0) & (C >= 0)
    M = sp.coo_matrix((V[keep], (R[keep], C[keep])), shape=(nrows, ncols)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return M


def renumber(keep_mask):
    """Map old ids -> new consecutive ids (-1 where dropped)."""
    m = np.full(keep_mask.shape[0], -1, dtype=np.int64)
    m[keep_mask] = np.arange(int(keep_mask.sum()))
    return m
