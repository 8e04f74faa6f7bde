"""Seeded N x N block systems that stand in for the paper's coupled problems.

Each builder returns a :class:`BlockSystem`: per-field sizes, block sizes and
near-nullspace vectors, the N x N grid of CSR blocks (``None`` = zero block)
and seeded right-hand sides.  The block shapes follow the paper's coupled
systems: the 2x2 thermo-structure Jacobian (Section 6, TSI monolithic system),
the 3x3 solid / grid / fluid FSI system (Section 6, FSI block system) and the
lung's FSI-plus-constraint saddle point (Section 6, lung block system).  The
physics is synthetic; only the structure and scales are meant to match.
"""
from dataclasses import dataclass, field as dfield
import numpy as np
import scipy.sparse as sp

from . import fem


@dataclass
class Field:
    name: str
    ndof: int
    block_size: int
    nullspace: np.ndarray          # (nns, ndof), row c = near-nullspace vector c

    @property
    def nns(self):
        return self.nullspace.shape[0]


@dataclass
class BlockSystem:
    fields: list
    blocks: list                   # blocks[i][j]: scipy CSR (float64) or None
    rhs: np.ndarray                # (nrhs, n): row c = right-hand side c
    meta: dict = dfield(default_factory=dict)

    @property
    def nfields(self):
        return len(self.fields)

    @property
    def n(self):
        return sum(f.ndof for f in self.fields)

    def offsets(self):
        o = [0]
        for f in self.fields:
            o.append(o[-1] + f.ndof)
        return o

    def nnz(self):
        return sum(b.nnz for row in self.blocks for b in row if b is not None)

    def assembled(self):
        """The whole matrix as one CSR (for dense/LU comparisons in tests)."""
        rows = []
        for i, fi in enumerate(self.fields):
            rows.append([self.blocks[i][j] if self.blocks[i][j] is not None
                         else sp.csr_matrix((fi.ndof, fj.ndof)) for j, fj in enumerate(self.fields)])
        M = sp.bmat(rows, format="csr")
        M.sort_indices()
        return M


def uniform_rhs(n, nrhs, seed):
    """iid uniform[-1, 1] right-hand sides, (nrhs, n)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x5EED]))
    return rng.uniform(-1.0, 1.0, size=(nrhs, n))


def rigid_modes_2d(xy, center):
    """Planar rigid-body modes (2 translations + rotation), interleaved dofs."""
    n = xy.shape[0]
    B = np.zeros((3, 2 * n))
    B[0, 0::2] = 1.0
    B[1, 1::2] = 1.0
    B[2, 0::2] = -(xy[:, 1] - center[1])
    B[2, 1::2] = xy[:, 0] - center[0]
    return B


def rigid_modes_3d(xyz, center):
    """3 translations + 3 infinitesimal rotations, interleaved dofs."""
    n = xyz.shape[0]
    d = xyz - np.asarray(center)[None, :]
    B = np.zeros((6, 3 * n))
    for c in range(3):
        B[c, c::3] = 1.0
    # rotation about z: (-y, x, 0); about x: (0, -z, y); about y: (z, 0, -x)
    B[3, 0::3] = -d[:, 1]
    B[3, 1::3] = d[:, 0]
    B[4, 1::3] = -d[:, 2]
    B[4, 2::3] = d[:, 1]
    B[5, 0::3] = d[:, 2]
    B[5, 2::3] = -d[:, 0]
    return B


# --------------------------------------------------------------------------
# 2-field thermo-structure-like system (the TSI 2x2 block Jacobian)
# --------------------------------------------------------------------------
def tsi2d(nel=32, E=1.0, nu=0.3, kappa=1.0, dt=0.1, alpha=1e-2, cba=1e-3,
          cba_sign=+1.0, seed=0, nrhs=1, clamp=True, heat_mass=True,
          coupling=True):
    """Plane-strain elasticity (field A, 2 dof/node) + transient heat (field B).

    Unit square, nel x nel bilinear elements.  A is clamped at x = 0 (those
    dofs are removed).  B = M/dt + kappa*K on all nodes.
    C_AB = alpha * int B^T m N  with m = (1, 1, 0) (thermal stress),
    C_BA = cba_sign * cba * int N div(N_u)  (mass-weighted divergence).
    clamp=False / heat_mass=False give the singular Neumann operators whose
    kernels are the rigid-body / constant modes (used to test prolongators).
    """
    h = 1.0 / nel
    nn1 = nel + 1
    nnodes = nn1 * nn1
    ii, jj = np.meshgrid(np.arange(nn1), np.arange(nn1), indexing="xy")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1)
    conn = fem.grid_conn_2d(nel, nel)
    g = fem.q1_2d(h, h)

    free_node = np.ones(nnodes, bool)
    if clamp:
        free_node[ii.ravel() == 0] = False
    free_dof = np.repeat(free_node, 2)
    umap = fem.renumber(free_dof)
    nA = int(free_dof.sum())
    nB = nnodes

    edofs = fem.element_dofs(conn, 2)
    Ke = fem.ke_elastic(g, E, nu)
    AAA = fem.assemble(edofs, edofs, Ke, nA, nA, umap, umap)

    Kt = fem.ke_laplace(g, kappa)
    Mt = fem.ke_mass(g)
    Bt = kappa * Kt + (Mt / dt if heat_mass else 0.0 * Mt)
    ABB = fem.assemble(conn, conn, Bt, nB, nB)

    blocks = [[AAA, None], [None, ABB]]
    if coupling:
        G = fem.ke_grad_shape(g)                        # (8, 4)
        CAB = fem.assemble(edofs, conn, alpha * G, nA, nB, umap, None)
        CBA = fem.assemble(conn, edofs, cba_sign * cba * G.T, nB, nA, None, umap)
        blocks = [[AAA, CAB], [CBA, ABB]]

    nsA = rigid_modes_2d(xy[free_node], (0.5, 0.5))
    nsB = np.ones((1, nB))
    fields = [Field("structure", nA, 2, nsA), Field("thermo", nB, 1, nsB)]
    sys_ = BlockSystem(fields, blocks, uniform_rhs(nA + nB, nrhs, seed),
                       meta=dict(kind="tsi2d", nel=nel, seed=seed))
    return sys_


def _not_yet(*a, **k):
    raise NotImplementedError


fsi3d = _not_yet
lung3d = _not_yet
request_trace = _not_yet
