"""Lung-like saddle system: the generator's physics and the oracle's SIMPLE /
AMG(SIMPLE) paths, pinned against closed forms, dense library solves and
structural invariants of the monolithic hierarchy."""
import numpy as np
import pytest
import scipy.sparse as sp

import nfgen
from oracle import Oracle

SPLIT = dict(split=[0, 0, 1])


@pytest.fixture(scope="module")
def lung_tiny():
    return nfgen.lung3d(n=4, depth=3, acinus=2, seed=3)


@pytest.fixture(scope="module")
def lung_small():
    return nfgen.lung3d(n=8, depth=4, acinus=2, seed=0)


# ------------------------------------------------------------- generator
def test_airway_block_is_spd_and_encodes_poiseuille_and_conservation(lung_small):
    s = lung_small
    W = s.blocks[1][1]
    assert abs(W - W.T).max() == 0.0
    assert np.linalg.eigvalsh(W.toarray()).min() > 0.0
    AWL = s.blocks[1][2]
    lam = np.random.default_rng(1).uniform(-1, 1, AWL.shape[1])
    x = sp.linalg.spsolve(W.tocsc(), -(AWL @ lam))
    p, q = x[0::2], x[1::2]
    nseg = p.size
    first = nseg - lam.size
    Wd = W.diagonal()
    for sgm in range(nseg):
        pp = p[(sgm - 1) // 2] if sgm > 0 else 0.0
        if sgm < first:
            # Poiseuille: R q = pressure drop; mass conservation at the node
            assert abs(Wd[2 * sgm + 1] * q[sgm] - (pp - p[sgm])) < 1e-10
            assert abs(q[sgm] - q[2 * sgm + 1] - q[2 * sgm + 2]) < 1e-10
        else:
            # segment and acinus in series down to the acinus pressure
            assert abs(Wd[2 * sgm + 1] * q[sgm] - (pp - lam[sgm - first])) < 1e-10


def test_constraint_rows_measure_acinus_volume_change(lung_small):
    """B_k applied to the dilation u(x) = x - x0 gives div u * |acinus| = 3 (m h)^3
    for acini away from the clamped face (closed form of the surface integral)."""
    n, m = 8, 2
    s = lung_small
    B = s.blocks[2][0].toarray()
    h = 1.0 / n
    dims = n + 1
    kk, jj, ii = np.meshgrid(np.arange(dims), np.arange(dims), np.arange(dims), indexing="ij")
    xyz = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1) * h
    free = kk.ravel() > 0
    u = (xyz[free] - 0.3).ravel()           # interleaved (x, y, z) dofs of free nodes
    vol = B @ u
    # rows whose acinus touches z = 0 lose the clamped face's contribution
    touches = np.array([np.any(np.abs(B[k].reshape(-1, 3)[:, 2]) > 0) and
                        np.count_nonzero(B[k]) < 6 * (m + 1) ** 2 for k in range(B.shape[0])])
    full = vol[~touches]
    assert full.size > 0
    assert np.allclose(full, 3.0 * (m * h) ** 3, rtol=1e-12)


def test_coupling_blocks_are_antisymmetric_pair(lung_small):
    s = lung_small
    assert abs(s.blocks[0][2] + s.blocks[2][0].T).max() == 0.0
    assert s.blocks[2][2] is None


# ------------------------------------------------------------ oracle pins
def test_simple_exact_blocks_solves_to_dense(lung_tiny):
    s = lung_tiny
    A = s.assembled().toarray()
    xd = np.linalg.solve(A, s.rhs[0])
    o = Oracle(s.fields, s.blocks, "SIMPLE(LU;LU)", **SPLIT)
    x, st = o.gmres(s.rhs[0], rtol=1e-12, maxit=200)
    assert st["status"] == 0
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_simple_precond_is_the_paper_block_factorisation(lung_tiny):
    """With exact predictor and Schur solves, SIMPLE applies M^-1 for
    M = [A11 0; A21 S~] [I D~^-1 A12; 0 I] (Sec. 3.2 matrix form), built here
    densely with numpy."""
    s = lung_tiny
    A = s.assembled().toarray()
    n1 = s.fields[0].ndof + s.fields[1].ndof
    A11, A12, A21, A22 = A[:n1, :n1], A[:n1, n1:], A[n1:, :n1], A[n1:, n1:]
    dt = np.abs(A11).sum(axis=1)
    St = A22 - A21 @ (A12 / dt[:, None])
    L = np.block([[A11, np.zeros_like(A12)], [A21, St]])
    U = np.block([[np.eye(n1), A12 / dt[:, None]], [np.zeros_like(A21), np.eye(A.shape[0] - n1)]])
    r = np.random.default_rng(5).standard_normal(A.shape[0])
    z_ref = np.linalg.solve(L @ U, r)
    o = Oracle(s.fields, s.blocks, "SIMPLE(LU;LU)", **SPLIT)
    z = o.precond_apply(r)
    assert np.linalg.norm(z - z_ref) <= 1e-10 * np.linalg.norm(z_ref)


def test_amg_simple_single_level_is_dense_solve(lung_tiny):
    s = lung_tiny
    o = Oracle(s.fields, s.blocks, "AMG(SIMPLE)", coarse_max=10 ** 6, **SPLIT)
    assert o.nlevels(0) == 1
    r = np.random.default_rng(2).standard_normal(s.n)
    z = o.precond_apply(r)
    zd = np.linalg.solve(s.assembled().toarray(), r)
    assert np.linalg.norm(z - zd) <= 1e-9 * np.linalg.norm(zd)


def test_amg_simple_hierarchy_structure(lung_small):
    """Multipliers are not coarsened (P = I on every level), their block stays
    zero, every coarse block is the Galerkin product R_i A_ij P_j, and the
    coupling pair keeps A^c_13 = -(A^c_31)^T."""
    s = lung_small
    o = Oracle(s.fields, s.blocks, "AMG(SIMPLE)", coarse_max=200, **SPLIT)
    nl = o.nlevels(0)
    assert nl >= 2
    for l in range(nl - 1):
        P2 = o.matrix(0, l, "P", 2, 0)
        assert P2.shape[0] == P2.shape[1] == s.fields[2].ndof
        assert abs(P2 - sp.identity(P2.shape[0])).max() == 0.0
        assert o.matrix(0, l + 1, "A", 2, 2) is None
        for i in range(3):
            for j in range(3):
                Aij = o.matrix(0, l, "A", i, j)
                Ac = o.matrix(0, l + 1, "A", i, j)
                if Aij is None:
                    assert Ac is None
                    continue
                ref = (o.matrix(0, l, "R", i, 0) @ Aij @ o.matrix(0, l, "P", j, 0)).toarray()
                got = Ac.toarray()
                if i == j and i < 2:
                    # dead tentative columns get a unit diagonal on the coarse level
                    keep = np.abs(ref).sum(1) > 0
                    got, ref = got[keep][:, keep], ref[keep][:, keep]
                assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        A13 = o.matrix(0, l + 1, "A", 0, 2).toarray()
        A31 = o.matrix(0, l + 1, "A", 2, 0).toarray()
        assert np.abs(A13 + A31.T).max() <= 1e-12 * np.abs(A31).max()


@pytest.mark.parametrize("spec", ["AMG(SIMPLE)", "SIMPLE(AMG(BGS);LU)", "SIMPLE(BGS(AMG);LU)"])
def test_lung_methods_converge_to_dense_solution(lung_small, spec):
    s = lung_small
    xd = np.linalg.solve(s.assembled().toarray(), s.rhs[0])
    o = Oracle(s.fields, s.blocks, spec, **SPLIT)
    x, st = o.gmres(s.rhs[0], rtol=1e-10, maxit=400)
    assert st["status"] == 0
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)


def test_amg_simple_schur_chebyshev_branch(lung_small):
    """Above schur_direct_max the level Schur solve is Chebyshev on S~; the
    preconditioner stays a convergent GMRES preconditioner."""
    s = lung_small
    xd = np.linalg.solve(s.assembled().toarray(), s.rhs[0])
    o = Oracle(s.fields, s.blocks, "AMG(SIMPLE)", schur_direct_max=4, **SPLIT)
    x, st = o.gmres(s.rhs[0], rtol=1e-10, maxit=600)
    assert st["status"] == 0
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
