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


# --------------------------------------------------------------------------
# Structured hex grids: assembly straight into a 27-point node stencil
# --------------------------------------------------------------------------
_LOCAL3 = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                    [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])


def grid_nodes(dims):
    """(i, j, k) of every node of an (nx+1, ny+1, nz+1) grid, id = (k*ny1+j)*nx1+i."""
    nx1, ny1, nz1 = dims
    k, j, i = np.meshgrid(np.arange(nz1), np.arange(ny1), np.arange(nx1), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def stencil_assemble(nel_dims, ncomp, pair_block):
    """Sum hex element matrices into st[node, slot, c, d] (slot = 27-point
    neighbour offset, lexicographic in (dz, dy, dx)).

    pair_block(a, b) returns the (nel, ncomp, ncomp) block of every element
    matrix coupling local node a (rows) to local node b (columns), elements
    in the order of grid_conn_3d.
    """
    nx, ny, nz = nel_dims
    dims = (nx + 1, ny + 1, nz + 1)
    nn = dims[0] * dims[1] * dims[2]
    conn = grid_conn_3d(nx, ny, nz)
    st = np.zeros((nn, 27, ncomp, ncomp))
    for a in range(8):
        rows = conn[:, a]                       # distinct for a fixed a
        for b in range(8):
            d = _LOCAL3[b] - _LOCAL3[a]
            slot = (d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)
            st[rows, slot] += pair_block(a, b)
    return st, dims


def stencil_to_csr(st, dims, row_map, col_map, nrows, ncols, comp_pairs=None, dirichlet=None):
    """CSR from a node stencil.

    row_map / col_map: old dof (node*ncomp + comp) -> new index or -1; both
    must be increasing on the kept dofs so that rows and columns come out
    sorted.  comp_pairs (ncomp, ncomp) bool: component couplings to store.
    dirichlet: bool per old dof; such rows and columns keep only their
    diagonal, set to 1.
    """
    nn, _, nc, _ = st.shape
    nx1, ny1, nz1 = dims
    ijk = grid_nodes(dims)
    offs = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    nb_ijk = ijk[:, None, :] + offs[None, :, :]
    inside = np.all((nb_ijk >= 0) & (nb_ijk < np.array(dims)), axis=2)
    nb = (nb_ijk[..., 2] * ny1 + nb_ijk[..., 1]) * nx1 + nb_ijk[..., 0]
    nb = np.where(inside, nb, 0)
    if comp_pairs is None:
        comp_pairs = np.ones((nc, nc), bool)
    u = np.arange(nn)
    rdof = u[:, None] * nc + np.arange(nc)[None, :]                 # (nn, c)
    cdof = nb[:, :, None] * nc + np.arange(nc)[None, None, :]       # (nn, s, d)
    R = np.broadcast_to(rdof[:, :, None, None], (nn, nc, 27, nc))
    Cd = np.broadcast_to(cdof[:, None, :, :], (nn, nc, 27, nc))
    keep = (np.broadcast_to(inside[:, None, :, None], R.shape)
            & np.broadcast_to(comp_pairs[None, :, None, :], R.shape))
    V = np.ascontiguousarray(np.transpose(st, (0, 2, 1, 3)))      # (nn, c, s, d)
    if dirichlet is not None:
        dr = dirichlet[R]
        dc = dirichlet[Cd]
        diag = (R == Cd)
        keep &= (~dr & ~dc) | diag
        V = np.where(diag & dr, 1.0, V)
    rows = row_map[R]
    cols = col_map[Cd]
    keep &= (rows >= 0) & (cols >= 0)
    rows = rows[keep]
    cols = cols[keep].astype(np.int32)
    vals = V[keep]
    ptr = np.zeros(nrows + 1, np.int64)
    ptr[1:] = np.bincount(rows, minlength=nrows)
    np.cumsum(ptr, out=ptr)
    M = sp.csr_matrix((vals, cols, ptr), shape=(nrows, ncols))
    M.has_sorted_indices = True
    return M


def gauss_tensors_3d(h):
    """Constant per-element tensors of a cube of side h (2x2x2 Gauss):
    L[a,b] = int grad N_a . grad N_b,  C[d,a,b] = int N_a dN_b/dx_d,
    G[c,a,b] = int dN_a/dx_c N_b,  D[c,d,a,b] = int dN_a/dx_c dN_b/dx_d,
    M[a,b] = int N_a N_b."""
    N, dN, w = q1_3d(h, h, h)
    L = np.einsum("q,qad,qbd->ab", w, dN, dN)
    Cm = np.einsum("q,qa,qbd->dab", w, N, dN)
    G = np.einsum("q,qac,qb->cab", w, dN, N)
    D = np.einsum("q,qac,qbd->cdab", w, dN, dN)
    M = np.einsum("q,qa,qb->ab", w, N, N)
    return L, Cm, G, D, M
