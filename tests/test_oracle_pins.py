"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own code: each compares it with a
closed form, an invariant, a brute-force check on a tiny input, a dense
library factorisation, or the paper's matrix form of a method.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import nfgen
import oracle
from oracle import Oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_tsi(nel=6, **kw):
    return nfgen.tsi2d(nel=nel, **kw)


# --------------------------------------------------------------- splitmix64
def test_splitmix64_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    for k, hexval in rows:
        assert oracle.splitmix64((int(k) * gamma) % 2**64) == int(hexval, 16)


# ------------------------------------------------------------- block SpMV
def test_block_matvec_matches_dense():
    s = small_tsi(8)
    o = Oracle(s.fields, s.blocks, "BGS(LU)")
    x = np.random.default_rng(1).standard_normal(s.n)
    A = s.assembled().toarray()
    y = o.matvec(x)
    ref = A @ x
    bound = 1e-14 * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)


# ------------------------------------------------------------ node graph
@pytest.mark.parametrize("field,b,cut", [(0, 2, False), (1, 1, False), (0, 2, True), (1, 1, True)])
def test_node_graph_brute_force(field, b, cut):
    """u ~ v iff some dof of u and some dof of v are coupled by a stored entry
    in either direction (the pattern of A + A^T), u != v."""
    s = small_tsi(5)
    A = s.blocks[field][field]
    if cut:
        A = nfgen.one_sided_pattern(A, 3)
        assert (A != A.T).nnz > 0
    gp, ga = oracle.node_graph(A, b)
    D = A.toarray() != 0
    D = D | D.T
    nn = A.shape[0] // b
    for u in range(nn):
        blk = D[b * u:b * u + b].reshape(b, nn, b).any(axis=(0, 2))
        blk[u] = False
        assert list(ga[gp[u]:gp[u + 1]]) == list(np.nonzero(blk)[0])


# ---------------------------------------------------------------- MIS-2
def _dist2(gp, ga, n):
    adj = np.zeros((n, n), bool)
    for u in range(n):
        adj[u, ga[gp[u]:gp[u + 1]]] = True
    a2 = adj | (adj.astype(int) @ adj.astype(int) > 0)
    np.fill_diagonal(a2, False)
    return adj, a2


def _random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    M = rng.random((n, n)) < p
    M = M | M.T
    np.fill_diagonal(M, False)
    gp = np.zeros(n + 1, np.int64)
    adj = []
    for u in range(n):
        nb = np.nonzero(M[u])[0]
        adj.extend(nb)
        gp[u + 1] = len(adj)
    return gp, np.array(adj, np.int32)


GRAPHS = [("tsi-structure", lambda: oracle.node_graph(small_tsi(9).blocks[0][0], 2)),
          ("tsi-thermo", lambda: oracle.node_graph(small_tsi(9).blocks[1][1], 1)),
          ("random-sparse", lambda: _random_graph(150, 0.02, 3)),
          ("random-dense", lambda: _random_graph(120, 0.1, 4)),
          ("isolated", lambda: _random_graph(60, 0.0, 5))]


@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("seed", [0, 7])
def test_mis2_independent_maximal_partition(name, make, seed):
    gp, ga = make()
    n = len(gp) - 1
    st, agg, na = oracle.mis2_aggregate(gp, ga, seed)
    adj, a2 = _dist2(gp, ga, n)
    roots = np.nonzero(st == 1)[0]
    assert set(np.unique(st)) <= {1, 2}
    # independence: roots pairwise at distance >= 3
    assert not a2[np.ix_(roots, roots)].any()
    # maximality: every non-root within distance 2 of a root
    others = np.nonzero(st != 1)[0]
    assert a2[np.ix_(others, roots)].any(axis=1).all()
    # partition with one root per aggregate; roots numbered in node order
    assert na == len(roots)
    assert np.all(agg >= 0) and np.all(agg < na)
    assert list(agg[roots]) == list(range(na))
    # every node is at most 2 steps from its own root, inside its aggregate
    for u in others:
        r = roots[agg[u]]
        assert adj[u, r] or (adj[u] & adj[:, r] & (agg == agg[u])).any()


def test_mis2_deterministic_and_seeded():
    gp, ga = oracle.node_graph(small_tsi(12).blocks[1][1], 1)
    a = oracle.mis2_aggregate(gp, ga, 3)
    b = oracle.mis2_aggregate(gp, ga, 3)
    c = oracle.mis2_aggregate(gp, ga, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])


def test_mis2_matches_definition_bruteforce():
    """Synchronous rounds re-derived by brute force over (key, id) tuples."""
    gp, ga = _random_graph(80, 0.05, 11)
    n = 80
    _, a2 = _dist2(gp, ga, n)
    seed = 5
    key = [oracle.splitmix64(seed ^ oracle.splitmix64(u)) for u in range(n)]
    st = np.zeros(n, int)
    while (st == 0).any():
        und = st == 0
        new = [u for u in range(n) if und[u] and all(
            (key[w], w) < (key[u], u) for w in np.nonzero(a2[u] & und)[0])]
        st[new] = 1
        near = a2[:, st == 1].any(axis=1)
        st[und & near & (st == 0)] = 2
    got, _, _ = oracle.mis2_aggregate(gp, ga, seed)
    assert np.array_equal(got, st)


def _aggregates_by_definition(gp, ga, st):
    """Aggregates from the MIS-2 states, written out from the definition on a
    dense adjacency: roots numbered in ascending node order; a non-root
    adjacent to a root joins it (that root is unique); every other node joins
    the adjacent phase-2 node's aggregate with the smallest number."""
    n = len(gp) - 1
    adj = np.zeros((n, n), bool)
    for u in range(n):
        adj[u, ga[gp[u]:gp[u + 1]]] = True
    roots = np.nonzero(st == 1)[0]
    agg = np.full(n, -1)
    agg[roots] = np.arange(len(roots))
    phase2 = np.zeros(n, bool)
    for u in range(n):
        if st[u] == 1:
            continue
        near = [r for r in roots if adj[u, r]]
        assert len(near) <= 1                 # roots are at least 3 apart
        if near:
            agg[u] = agg[near[0]]
            phase2[u] = True
    ties = 0
    for u in range(n):
        if agg[u] >= 0:
            continue
        cand = sorted({agg[v] for v in np.nonzero(adj[u] & phase2)[0]})
        assert cand, u
        ties += len(cand) > 1
        agg[u] = cand[0]
    return agg, ties


@pytest.mark.parametrize("name,make", GRAPHS + [("tsi-structure-13", lambda: oracle.node_graph(small_tsi(13).blocks[0][0], 2)),
                                                ("fsi-grid", lambda: oracle.node_graph(nfgen.fsi3d(n=6, layers=2).blocks[1][1], 3))])
@pytest.mark.parametrize("seed", [0, 7, 12])
def test_aggregation_phase3_smallest_number(name, make, seed):
    """The oracle's aggregates equal the definition; and the graphs used here
    contain nodes whose phase-2 neighbours lie in different aggregates, so a
    largest-number or first-found join would fail this test."""
    gp, ga = make()
    st, agg, na = oracle.mis2_aggregate(gp, ga, seed)
    ref, ties = _aggregates_by_definition(gp, ga, st)
    assert np.array_equal(agg, ref)


def test_aggregation_phase3_ties_occur():
    """The graphs of the phase-3 test include real ties (see above)."""
    total = 0
    for _, make in GRAPHS:
        gp, ga = make()
        for seed in (0, 7, 12):
            st, _, _ = oracle.mis2_aggregate(gp, ga, seed)
            total += _aggregates_by_definition(gp, ga, st)[1]
    assert total >= 5, total


# ------------------------------------------------------ tentative prolongator
def test_tentative_orthonormal_and_reproduces_nullspace():
    s = small_tsi(10)
    A = s.blocks[0][0]
    gp, ga = oracle.node_graph(A, 2)
    _, agg, na = oracle.mis2_aggregate(gp, ga, 0)
    B = s.fields[0].nullspace
    P, Bc, ndead = oracle.tentative(agg, na, 2, B)
    assert ndead == 0
    PtP = (P.T @ P).toarray()
    assert np.allclose(PtP, np.eye(P.shape[1]), atol=1e-14)
    assert np.max(np.abs(P @ Bc.T - B.T)) < 1e-14
    # R factors upper triangular with positive diagonal
    for a in range(na):
        R = Bc[:, 3 * a:3 * a + 3].T
        assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)


def test_tentative_dead_column():
    # one aggregate of a single 2-dof node with 3 rigid modes -> rank 2
    B = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, -3.0]])   # third = 2 e1 - 3 e2
    P, Bc, ndead = oracle.tentative(np.array([0]), 1, 2, B)
    assert ndead == 1
    assert np.allclose(P.toarray()[:, 2], 0.0)
    assert np.max(np.abs(P @ Bc.T - B.T)) < 1e-14


# ---------------------------------------------------------- hierarchy pins
@pytest.fixture(scope="module")
def tsi_ctx():
    s = nfgen.tsi2d(nel=16)
    return s, Oracle(s.fields, s.blocks, "BGS(AMG)", sweeps=2, coarse_max=40)


def test_power_lambda_close_to_eig(tsi_ctx):
    s, o = tsi_ctx
    A = s.blocks[1][1]
    d = A.diagonal()
    ev = np.max(np.abs(np.linalg.eigvals(A.toarray() / d[:, None])))
    lam = o.lam(1, 0)
    assert lam == oracle.power_lambda(A, 0, 10)
    assert 0.5 * ev < lam <= ev * (1 + 1e-12)


def _check_P_reproduces_nullspace(o, h, A, B):
    P = o.matrix(h, 0, "P")
    Bc = o.nullspace(h, 1)
    AB = np.abs(A @ B.T).max(axis=1)
    free = AB < 1e-12                     # rows where A B = 0
    assert free.sum() > 0.5 * A.shape[0]
    err = np.abs(P @ Bc.T - B.T).max(axis=1)
    assert err[free].max() < 1e-12
    # and the tentative part alone reproduces B exactly on every row
    assert o.nlevels(h) >= 2


def test_smoothed_P_reproduces_rigid_modes(tsi_ctx):
    s, o = tsi_ctx
    _check_P_reproduces_nullspace(o, 0, s.blocks[0][0], s.fields[0].nullspace)


def test_smoothed_P_reproduces_constant_mode():
    """Pure Laplacian grounded at one node: constants are in the kernel of every
    row that does not touch the grounded node."""
    s = nfgen.tsi2d(nel=16, heat_mass=False, coupling=False)
    K = s.blocks[1][1][1:, 1:].tocsr()
    f = nfgen.Field("heat", K.shape[0], 1, np.ones((1, K.shape[0])))
    o = Oracle([f], [[K]], "AMG", coarse_max=40)
    _check_P_reproduces_nullspace(o, 0, K, f.nullspace)


def test_galerkin_rap_and_transpose(tsi_ctx):
    s, o = tsi_ctx
    for h in range(o.hier_count()):
        for l in range(o.nlevels(h) - 1):
            A = o.matrix(h, l, "A")
            P = o.matrix(h, l, "P")
            R = o.matrix(h, l, "R")
            Ac = o.matrix(h, l + 1, "A")
            # R == P^T bitwise (pattern and values)
            PT = sp.csr_matrix(P.T)
            PT.sort_indices()
            assert np.array_equal(R.indptr, PT.indptr) and np.array_equal(R.indices, PT.indices)
            assert np.array_equal(R.data, PT.data)
            dense = P.toarray().T @ A.toarray() @ P.toarray()
            scale = np.abs(dense).max()
            assert np.abs(Ac.toarray() - dense).max() < 1e-13 * scale
            sym = np.abs(Ac - Ac.T).max() / scale
            assert sym < 1e-14


def test_one_level_is_exact():
    s = nfgen.tsi2d(nel=4)
    o = Oracle(s.fields, s.blocks, "BGS[sweeps=1,order=fwd](AMG)", coarse_max=1000)
    assert [o.nlevels(h) for h in range(o.hier_count())] == [1, 1]
    r = np.random.default_rng(0).standard_normal(s.n)
    z = o.precond_apply(r)
    n0 = s.fields[0].ndof
    # forward BGS with exact block solves: field 0 solve, then field 1
    z0 = np.linalg.solve(s.blocks[0][0].toarray(), r[:n0])
    z1 = np.linalg.solve(s.blocks[1][1].toarray(), r[n0:] - s.blocks[1][0] @ z0)
    assert np.allclose(z, np.concatenate([z0, z1]), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- Chebyshev
@pytest.mark.parametrize("degree,ratio,boost", [(1, 30.0, 1.1), (2, 30.0, 1.1), (3, 30.0, 1.1), (1, 4.0, 1.1),
                                                (2, 4.0, 1.0)])
def test_chebyshev_closed_form(degree, ratio, boost):
    n, c = 40, 0.3
    A = sp.diags([np.full(n - 1, c), np.ones(n), np.full(n - 1, c)], [-1, 0, 1], format="csr")
    k = np.arange(1, n + 1)
    lam_k = 1 + 2 * c * np.cos(k * np.pi / (n + 1))
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(np.arange(1, n + 1), k) * np.pi / (n + 1))
    lam = lam_k.max()
    lo, hi = lam / ratio, boost * lam
    th, de = (hi + lo) / 2, (hi - lo) / 2
    T = lambda m, t: np.cos(m * np.arccos(t)) if abs(t) <= 1 else np.cosh(m * np.arccosh(abs(t))) * (np.sign(t) ** m)
    for j in range(n):
        v = V[:, j]
        x = oracle.chebyshev(A, lam, A @ v, degree=degree, ratio=ratio, boost=boost)
        p = T(degree, (th - lam_k[j]) / de) / T(degree, th / de)
        assert np.abs(x - (1 - p) * v).max() < 1e-14


# ---------------------------------------------------------------- V-cycle
@pytest.mark.parametrize("spec", ["AMG", "AMG[smoother=sgs,omega=0.9]", "AMG[smoother=sgs,omega=0.9,half=1]",
                                  "AMG[smoother=sgs,omega=1.1,half=1,steps=2]", "AMG[smoother=ddgs,omega=0.9,ddmin=1]",
                                  "AMG[smoother=ddgs,omega=0.8,half=1,ddmin=1]"])
def test_vcycle_symmetric_contraction(spec):
    """With R = P^T, an exact coarse solve and a post-smoother that is the
    adjoint of the pre-smoother (the same Chebyshev polynomial, or the
    backward colour sweep after the forward one), the V-cycle is a symmetric
    operator and an A-norm contraction (Sec. 3.1)."""
    s = nfgen.tsi2d(nel=10)
    sub = [s.fields[1]]
    blocks = [[s.blocks[1][1]]]
    o = Oracle(sub, blocks, spec, coarse_max=20)
    assert o.nlevels(0) >= 2
    n = s.fields[1].ndof
    M = o.precond_apply(np.eye(n))          # row i = M e_i  (M symmetric)
    A = blocks[0][0].toarray()
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    ev = sla.eigvals(np.eye(n) - M.T @ A).real
    assert ev.min() > -1e-10 and ev.max() < 1.0


def test_vcycle_half_sweeps_differ_by_phase():
    """Half sweeps taken in the same direction before and after the coarse
    correction would make the V-cycle non-symmetric: the symmetric result
    above depends on the post-smoother sweeping backward."""
    s = nfgen.tsi2d(nel=10)
    A = s.blocks[1][1]
    n = A.shape[0]
    E = np.eye(n)
    fwd = np.array([oracle.sgs(A, 1, E[i], omega=0.9, half=1) for i in range(n)])       # forward only
    bwd = np.array([oracle.sgs(A, 1, E[i], omega=0.9, x0=np.zeros(n), half=1) for i in range(n)])
    assert np.abs(fwd - bwd.T).max() < 1e-12 * np.abs(fwd).max()   # adjoint pair
    assert np.abs(fwd - fwd.T).max() > 1e-3 * np.abs(fwd).max()    # not symmetric alone


# -------------------------------------------------------------------- BGS
def _bgs_dense_formula(s, r, sweeps, order):
    A = s.assembled().toarray()
    n0 = s.fields[0].ndof
    M = np.zeros_like(A)
    M[:n0, :n0] = A[:n0, :n0]
    M[n0:, n0:] = A[n0:, n0:]
    if order == "fwd":
        M[n0:, :n0] = A[n0:, :n0]
    else:
        M[:n0, n0:] = A[:n0, n0:]
    E = np.eye(len(A)) - np.linalg.solve(M, A)
    return (np.eye(len(A)) - np.linalg.matrix_power(E, sweeps)) @ np.linalg.solve(A, r)


@pytest.mark.parametrize("order", ["fwd", "bwd"])
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_bgs_exact_blocks_stationary_iteration(order, sweeps):
    s = nfgen.tsi2d(nel=5, alpha=0.3, cba=0.2)
    o = Oracle(s.fields, s.blocks, f"BGS[sweeps={sweeps},order={order}](LU)")
    r = np.random.default_rng(2).standard_normal(s.n)
    z = o.precond_apply(r)
    ref = _bgs_dense_formula(s, r, sweeps, order)
    assert np.abs(z - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("order,drop", [("fwd", (0, 1)), ("bwd", (1, 0))])
def test_bgs_block_triangular_one_iteration(order, drop):
    s = nfgen.tsi2d(nel=5)
    s.blocks[drop[0]][drop[1]] = None
    o = Oracle(s.fields, s.blocks, f"BGS[sweeps=1,order={order}](LU)")
    x, st = o.gmres(s.rhs[0], rtol=1e-12)
    assert st["iters"] == 1 and st["status"] == 0
    xd = np.linalg.solve(s.assembled().toarray(), s.rhs[0])
    assert np.abs(x - xd).max() < 1e-10 * np.abs(xd).max()


# ------------------------------------------------------------------- SIMPLE
def _simple_dense(A11, A12, A21, A22, dt):
    S = A22 - A21 @ np.diag(1 / dt) @ A12
    n1 = len(A11)
    L = np.block([[A11, np.zeros_like(A12)], [A21, S]])
    U = np.block([[np.eye(n1), np.diag(1 / dt) @ A12], [np.zeros_like(A21), np.eye(len(A22))]])
    return L @ U


def heat_first_tsi(nel, **kw):
    """The TSI-like system with its fields swapped: the transient heat block
    M/dt + K (row sums = the lumped mass / dt, all positive) is the SIMPLE
    predictor and the elastic block the Schur field."""
    return nfgen.permute_fields(nfgen.tsi2d(nel=nel, **kw), [1, 0])


# the literal SIMPLEC diagonal |sum_j a_ij| needs a predictor whose row sums
# do not vanish: it is pinned on the heat-first system, where it differs from
# the other two choices (K has off-diagonal entries of both signs' effect)
@pytest.mark.parametrize("heat_first,mode", [(False, 0), (False, 2), (True, 0), (True, 1), (True, 2)])
def test_simple_matches_matrix_form(heat_first, mode):
    s = heat_first_tsi(5, alpha=0.2, cba=0.1) if heat_first else nfgen.tsi2d(nel=5, alpha=0.2, cba=0.1)
    A = s.assembled().toarray()
    n0 = s.fields[0].ndof
    A11, A12, A21, A22 = A[:n0, :n0], A[:n0, n0:], A[n0:, :n0], A[n0:, n0:]
    B11 = s.blocks[0][0].toarray()
    dt = {0: np.abs(B11).sum(1), 1: np.abs(B11.sum(1)), 2: np.diag(B11)}[mode]
    assert dt.min() > 1e-3 * dt.max()
    if mode == 1:
        # the three diagonals are different here, so this pins mode 1 itself
        assert np.abs(dt - np.abs(B11).sum(1)).max() > 0.1 * dt.max()
        assert np.abs(dt - np.diag(B11)).max() > 0.1 * dt.max()
    o = Oracle(s.fields, s.blocks, "SIMPLE(LU;LU)", simplec_mode=mode)
    r = np.random.default_rng(3).standard_normal(s.n)
    z = o.precond_apply(r)
    M = _simple_dense(A11, A12, A21, A22, dt)
    ref = np.linalg.solve(M, r)
    assert np.abs(z - ref).max() < 1e-10 * np.abs(ref).max()


def test_simplec_literal_gmres_reaches_dense_solution():
    """GMRES with SIMPLE(AMG;AMG) and the literal SIMPLEC diagonal on the
    heat-first system converges to the dense solution."""
    s = heat_first_tsi(16)
    o = Oracle(s.fields, s.blocks, "SIMPLE(AMG;AMG)", simplec_mode=1, coarse_max=40)
    x, st = o.gmres(s.rhs[0], rtol=1e-10)
    xd = np.linalg.solve(s.assembled().toarray(), s.rhs[0])
    assert st["status"] == 0
    assert np.linalg.norm(x - xd) < 1e-7 * np.linalg.norm(xd)


def test_simple_exact_when_A11_diagonal():
    """A11 diagonal and positive: the SIMPLEC diagonal equals A11, so M_SIMPLE = A."""
    rng = np.random.default_rng(4)
    n1, n2 = 30, 12
    A11 = sp.diags(rng.uniform(1, 2, n1), format="csr")
    A12 = sp.random(n1, n2, 0.3, random_state=1, format="csr")
    A21 = sp.random(n2, n1, 0.3, random_state=2, format="csr")
    fields = [nfgen.Field("a", n1, 1, np.ones((1, n1))), nfgen.Field("b", n2, 1, np.ones((1, n2)))]
    o = Oracle(fields, [[A11, A12], [A21, None]], "SIMPLE(LU;LU)")
    b = rng.standard_normal(n1 + n2)
    x, st = o.gmres(b, rtol=1e-12)
    assert st["iters"] == 1
    A = sp.bmat([[A11, A12], [A21, None]]).toarray()
    assert np.abs(A @ x - b).max() < 1e-10


# ------------------------------------------------------------ monolithic AMG
def test_mono_amg_one_field_is_single_field_amg():
    s = nfgen.tsi2d(nel=12)
    f = [s.fields[0]]
    b = [[s.blocks[0][0]]]
    o1 = Oracle(f, b, "AMG", coarse_max=30)
    o2 = Oracle(f, b, "AMG(BGS)", coarse_max=30)
    r = np.random.default_rng(5).standard_normal(f[0].ndof)
    z1, z2 = o1.precond_apply(r), o2.precond_apply(r)
    assert np.abs(z1 - z2).max() < 1e-13 * np.abs(z1).max()


def test_mono_amg_decoupled_is_per_field_amg():
    s = nfgen.tsi2d(nel=16, coupling=False)
    o1 = Oracle(s.fields, s.blocks, "BGS[sweeps=1](AMG)", coarse_max=200)
    o2 = Oracle(s.fields, s.blocks, "AMG(BGS)", coarse_max=200)
    assert o2.nlevels(0) == o1.nlevels(0) == o1.nlevels(1)
    r = np.random.default_rng(6).standard_normal(s.n)
    z1, z2 = o1.precond_apply(r), o2.precond_apply(r)
    assert np.abs(z1 - z2).max() < 1e-12 * np.abs(z1).max()


def test_mono_amg_coarse_blocks_are_RiAijPj():
    s = nfgen.tsi2d(nel=16)
    o = Oracle(s.fields, s.blocks, "AMG(BGS)", coarse_max=100)
    assert o.nlevels(0) >= 2
    for l in range(o.nlevels(0) - 1):
        for i in range(2):
            for j in range(2):
                Aij = o.matrix(0, l, "A", i, j).toarray()
                Ri = o.matrix(0, l, "R", i).toarray()
                Pj = o.matrix(0, l, "P", j).toarray()
                Ac = o.matrix(0, l + 1, "A", i, j).toarray()
                ref = Ri @ Aij @ Pj
                assert np.abs(Ac - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1e-300)
    # whole-matrix form: R A P with block-diagonal R, P
    A = sp.bmat([[o.matrix(0, 0, "A", i, j) for j in range(2)] for i in range(2)]).toarray()
    P = sla.block_diag(*[o.matrix(0, 0, "P", i).toarray() for i in range(2)])
    Ac = sp.bmat([[o.matrix(0, 1, "A", i, j) for j in range(2)] for i in range(2)]).toarray()
    assert np.abs(Ac - P.T @ A @ P).max() < 1e-13 * np.abs(Ac).max()


# -------------------------------------------------------------------- GMRES
@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_gmres_minimal_residual_over_krylov_space(k):
    s = nfgen.tsi2d(nel=4)
    o = Oracle(s.fields, s.blocks, "BGS(AMG)", coarse_max=10)
    A = s.assembled().toarray()
    b = s.rhs[0]
    x, st = o.gmres(b, restart=50, maxit=k, rtol=1e-30)
    assert st["iters"] == k
    # x must minimise ||b - A x|| over x in M K_k(A M, b)
    cols = []
    v = b.copy()
    for _ in range(k):
        mv = o.precond_apply(v)
        cols.append(mv)
        v = A @ mv
    K = np.array(cols).T
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    best = np.linalg.norm(b - A @ Q @ c)
    got = np.linalg.norm(b - A @ x)
    assert abs(got - best) <= 1e-9 * np.linalg.norm(b)


def test_gmres_restart_and_flexible_reach_tolerance():
    s = nfgen.tsi2d(nel=8)
    o = Oracle(s.fields, s.blocks, "BGS(AMG)", sweeps=2, coarse_max=30)
    A = s.assembled()
    xd = spla.spsolve(A.tocsc(), s.rhs[0])
    for restart, flexible in [(50, 0), (3, 0), (50, 1), (4, 1)]:
        x, st = o.gmres(s.rhs[0], restart=restart, flexible=flexible, rtol=1e-10)
        rel = np.linalg.norm(s.rhs[0] - A @ x) / np.linalg.norm(s.rhs[0])
        assert st["status"] == 0 and rel < 1e-10 and abs(rel - st["relres"]) < 1e-12
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-7


def test_end_to_end_tsi_full_size_vs_sparse_lu():
    s = nfgen.tsi2d()
    o = Oracle(s.fields, s.blocks, "BGS(AMG)", sweeps=2, order="bwd")
    x, st = o.gmres(s.rhs[0], restart=50, rtol=1e-8)
    A = s.assembled()
    xd = spla.spsolve(A.tocsc(), s.rhs[0])
    assert st["status"] == 0
    assert np.linalg.norm(s.rhs[0] - A @ x) / np.linalg.norm(s.rhs[0]) < 1e-8
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-6


# -------------------------------------------------------------- error paths
def test_errors():
    s = nfgen.tsi2d(nel=4)
    for spec in ["BGS(AMG", "BGS(AMG[smoother=sgs,half=2])", "BGS(AMG[smoother=sgs,omega=0])",
                 "BGS(AMG[smoother=sgs,cheb_from=0])"]:
        with pytest.raises(oracle.OracleError) as e:
            Oracle(s.fields, s.blocks, spec, sweeps=2)
        assert e.value.code == -1, spec
    bad = [[s.blocks[0][0], s.blocks[0][1]], [s.blocks[1][0], None]]
    with pytest.raises(oracle.OracleError) as e:
        Oracle(s.fields, bad, "BGS(AMG)")
    assert e.value.code == -3
    o = Oracle(s.fields, s.blocks, "BGS(AMG)", coarse_max=10)
    b = s.rhs[0].copy()
    b[3] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        o.gmres(b)
    assert e.value.code == -5
    x, st = o.gmres(s.rhs[0], maxit=1, rtol=1e-14)
    assert st["status"] == 1 and st["iters"] == 1


# --------------------------------------------------- multicolour Gauss-Seidel
def _crown_graph(k):
    """K_{k,k} minus a perfect matching, numbered u_0 v_0 u_1 v_1 ...: greedy
    in node order needs k colours, the graph is 2-colourable."""
    n = 2 * k
    M = np.zeros((n, n), bool)
    for i in range(k):
        for j in range(k):
            if i != j:
                M[2 * i, 2 * j + 1] = M[2 * j + 1, 2 * i] = True
    gp = np.concatenate([[0], np.cumsum(M.sum(1))]).astype(np.int64)
    ga = np.concatenate([np.nonzero(M[u])[0] for u in range(n)]).astype(np.int32)
    return gp, ga


def _natural_greedy(adj):
    n = adj.shape[0]
    col = -np.ones(n, int)
    for u in range(n):
        used = {col[v] for v in np.nonzero(adj[u])[0] if v < u}
        col[u] = next(c for c in range(n + 1) if c not in used)
    return col


def _degeneracy(adj):
    """max over the removal sequence of the least remaining degree (the same
    for every tie-breaking)"""
    alive = np.ones(adj.shape[0], bool)
    deg = adj.sum(1).astype(int)
    worst = 0
    while alive.any():
        cand = np.nonzero(alive)[0]
        u = cand[np.argmin(deg[cand])]
        worst = max(worst, deg[u])
        alive[u] = False
        deg -= adj[u].astype(int)
    return worst


@pytest.mark.parametrize("name,make", GRAPHS + [("crown-40", lambda: _crown_graph(20))])
def test_coloring_valid_and_greedy(name, make):
    """Valid (no coupled pair shares a colour); greedy in some order (every
    node sees every smaller colour among its neighbours); at most as many
    colours as the node-order greedy colouring and at most degeneracy + 1
    (the smallest-last bound); the node-order colouring itself when that is
    not beaten."""
    gp, ga = make()
    n = len(gp) - 1
    col, nc = oracle.color_nodes(gp, ga, 3)
    adj, _ = _dist2(gp, ga, n)
    np.fill_diagonal(adj, False)
    assert col.min() == 0 and col.max() == nc - 1
    i, j = np.nonzero(adj)
    assert np.all(col[i] != col[j])
    for u in range(n):
        seen = {col[v] for v in np.nonzero(adj[u])[0]}
        assert all(c in seen for c in range(col[u]))
    nat = _natural_greedy(adj)
    assert nc <= min(nat.max() + 1, _degeneracy(adj) + 1)
    if nc == nat.max() + 1:
        assert np.array_equal(col, nat)
    if name == "crown-40":
        assert nat.max() + 1 == 20 and nc == 2


@pytest.mark.parametrize("b", [1, 2])
def test_coloring_one_sided_coupling(b):
    """A pattern in which row u couples to v but row v not to u: u and v still
    get different colours (the colouring sees the coupling from both ends)."""
    s = small_tsi(7)
    A = nfgen.one_sided_pattern(s.blocks[2 - b][2 - b], 5, frac=0.5)
    gp, ga = oracle.node_graph(A, b)
    col, nc = oracle.color_nodes(gp, ga, 0)
    coo = sp.coo_matrix(A)
    nu, nv = coo.row // b, coo.col // b
    off = nu != nv
    assert off.sum() > 0
    assert np.all(col[nu[off]] != col[nv[off]])


def test_coloring_structured_stencil_uses_eight_colours():
    s = nfgen.fsi3d(n=6, layers=2)
    gp, ga = oracle.node_graph(s.blocks[1][1], 3)   # 27-point stencil on a 5^3 node grid
    col, nc = oracle.color_nodes(gp, ga, 0)
    assert nc == 8


@pytest.mark.parametrize("field,b,omega", [(0, 2, 0.69), (1, 1, 1.0), (0, 2, 1.3)])
def test_sgs_equals_colour_splitting(field, b, omega):
    """One symmetric sweep = the forward then backward SOR splittings in which
    'earlier' means an earlier colour and a node's own dofs count as not yet
    updated."""
    s = nfgen.tsi2d(nel=5, seed=1)
    A = s.blocks[field][field]
    gp, ga = oracle.node_graph(A, b)
    col, nc = oracle.color_nodes(gp, ga, 0)
    Ad = A.toarray()
    n = Ad.shape[0]
    cr = np.repeat(col, b)
    D = np.diag(np.diag(Ad))
    Lf = np.where(cr[None, :] < cr[:, None], Ad, 0.0)
    Lb = np.where(cr[None, :] > cr[:, None], Ad, 0.0)
    rng = np.random.default_rng(2)
    rhs, x0 = rng.standard_normal(n), rng.standard_normal(n)
    Uf = Ad - D - Lf
    Ub = Ad - D - Lb
    x1 = np.linalg.solve(D / omega + Lf, rhs + (D / omega - D - Uf) @ x0)
    x2 = np.linalg.solve(D / omega + Lb, rhs + (D / omega - D - Ub) @ x1)
    got = oracle.sgs(A, b, rhs, omega=omega, steps=1, seed=0, x0=x0)
    assert np.abs(got - x2).max() < 1e-11 * np.abs(x2).max()
    # zero initial guess
    y1 = np.linalg.solve(D / omega + Lf, rhs)
    y2 = np.linalg.solve(D / omega + Lb, rhs + (D / omega - D - Ub) @ y1)
    assert np.abs(oracle.sgs(A, b, rhs, omega=omega) - y2).max() < 1e-11 * np.abs(y2).max()
    # half sweeps: forward only from a zero guess, backward only otherwise
    assert np.abs(oracle.sgs(A, b, rhs, omega=omega, half=1) - y1).max() < 1e-11 * np.abs(y1).max()
    z1 = np.linalg.solve(D / omega + Lb, rhs + (D / omega - D - Ub) @ x0)
    got = oracle.sgs(A, b, rhs, omega=omega, x0=x0, half=1)
    assert np.abs(got - z1).max() < 1e-11 * np.abs(z1).max()


# ------------------------------------------------------- Krylov breakdown
def test_gmres_breakdown_statuses():
    """Forward BGS with exact block solves on the singular A = [[I, I], [I, I]]
    makes A M^-1 = [[0, I], [0, I]]: for b = [e_1; 0] the first Arnoldi
    vector maps to zero and the iterate cannot improve (EBREAKDOWN, x = 0);
    for b = [e_1; e_1] = A [e_1; 0] the breakdown gives the exact solution."""
    n = 3
    I = sp.identity(n, format="csr")
    f = [nfgen.Field(f"f{k}", n, 1, np.ones((1, n))) for k in range(2)]
    o = Oracle(f, [[I, I], [I, I]], "BGS[sweeps=1,order=fwd](LU)")
    b = np.zeros(2 * n)
    b[0] = 1.0
    with pytest.raises(oracle.OracleError) as e:
        o.gmres(b)
    assert e.value.code == -4
    b[n] = 1.0
    x, st = o.gmres(b)
    assert st["status"] == 0 and st["iters"] == 1
    assert np.abs(sp.bmat([[I, I], [I, I]]) @ x - b).max() < 1e-14


# -------------------------------------------------------------------- DD(GS)
def _dd_splittings(A, b, col, sub):
    """D, and the lower / upper parts of the DD(GS) splitting: entry (r, p) of
    a node u coupled to node v of the same subdomain with an earlier (later)
    colour."""
    Ad = A.toarray()
    cr, sr = np.repeat(col, b), np.repeat(sub, b)
    same = sr[None, :] == sr[:, None]
    Lf = np.where(same & (cr[None, :] < cr[:, None]), Ad, 0.0)
    Lb = np.where(same & (cr[None, :] > cr[:, None]), Ad, 0.0)
    return Ad, np.diag(np.diag(Ad)), Lf, Lb


@pytest.mark.parametrize("field,b,omega", [(0, 2, 0.79), (1, 1, 0.69), (0, 2, 1.2)])
def test_ddgs_equals_subdomain_splitting(field, b, omega):
    """One DD(GS) sweep: (D/omega + L_s)(x1 - x0) = rhs - A x0, where L_s keeps
    the couplings to nodes of the same subdomain (the level's MIS-2
    aggregates) with an earlier colour; the backward sweep uses the later
    colours; half sweeps take one of the two."""
    s = nfgen.tsi2d(nel=9, seed=2)
    A = s.blocks[field][field]
    gp, ga = oracle.node_graph(A, b)
    col, nc = oracle.color_nodes(gp, ga, 0)
    _, agg, na = oracle.mis2_aggregate(gp, ga, 0)
    assert 1 < na < len(agg)
    Ad, D, Lf, Lb = _dd_splittings(A, b, col, agg)
    rng = np.random.default_rng(4)
    n = Ad.shape[0]
    rhs, x0 = rng.standard_normal(n), rng.standard_normal(n)
    x1 = x0 + np.linalg.solve(D / omega + Lf, rhs - Ad @ x0)
    x2 = x1 + np.linalg.solve(D / omega + Lb, rhs - Ad @ x1)
    got = oracle.sgs(A, b, rhs, omega=omega, x0=x0, dd=True)
    assert np.abs(got - x2).max() < 1e-11 * np.abs(x2).max()
    y1 = np.linalg.solve(D / omega + Lf, rhs)
    assert np.abs(oracle.sgs(A, b, rhs, omega=omega, half=1, dd=True) - y1).max() < 1e-11 * np.abs(y1).max()
    z1 = x0 + np.linalg.solve(D / omega + Lb, rhs - Ad @ x0)
    assert np.abs(oracle.sgs(A, b, rhs, omega=omega, x0=x0, half=1, dd=True) - z1).max() < 1e-11 * np.abs(z1).max()
    # the subdomain coupling is real here: it differs from the global colour sweep
    glob = oracle.sgs(A, b, rhs, omega=omega, x0=x0)
    assert np.abs(glob - got).max() > 1e-6 * np.abs(got).max()


def test_ddgs_limits_sgs_and_jacobi():
    """One subdomain: DD(GS) is the multicolour SGS.  One node per subdomain:
    every sweep is damped Jacobi, x1 = x0 + omega D^-1 (rhs - A x0)."""
    s = nfgen.tsi2d(nel=7, seed=5)
    A = s.blocks[0][0]
    nn = A.shape[0] // 2
    rng = np.random.default_rng(6)
    rhs, x0 = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    one = oracle.sgs(A, 2, rhs, omega=0.8, x0=x0, dd=True, sub=np.zeros(nn, np.int32))
    assert np.array_equal(one, oracle.sgs(A, 2, rhs, omega=0.8, x0=x0))
    dinv = 1.0 / A.diagonal()
    x1 = x0 + 0.8 * dinv * (rhs - A @ x0)
    x2 = x1 + 0.8 * dinv * (rhs - A @ x1)
    got = oracle.sgs(A, 2, rhs, omega=0.8, x0=x0, dd=True, sub=np.arange(nn, dtype=np.int32))
    assert np.abs(got - x2).max() < 1e-12 * np.abs(x2).max()


# ------------------------------------------------ Petrov-Galerkin transfers
def _fluid_only(n=8, seed=3):
    s = nfgen.fsi3d(n=n, layers=2, seed=seed)
    return [s.fields[2]], [[s.blocks[2][2]]]


def test_pg_dampings_minimise_column_residuals():
    """Petrov-Galerkin prolongator on the nonsymmetric fluid block:
    P - P_tent = -Q diag(omega) with Q = D^-1 A P_tent, and each column's
    damping minimises ||A P e_j||_2 over omega_j >= 0, i.e. A P e_j is
    orthogonal to A Q e_j where omega_j > 0 and the derivative at 0 is
    non-negative where omega_j = 0."""
    f, b = _fluid_only()
    A = b[0][0]
    o = Oracle(f, b, "AMG[pg=1]", coarse_max=100)
    assert o.nlevels(0) >= 2
    P = o.matrix(0, 0, "P").toarray()
    agg = o.aggregates(0, 0)
    na = agg.max() + 1
    Pt, _, _ = oracle.tentative(agg, na, f[0].block_size, f[0].nullspace)
    Pt = Pt.toarray()
    Ad = A.toarray()
    Q = (Ad / np.diag(Ad)[:, None]) @ Pt
    Dlt = Pt - P
    nq = np.linalg.norm(Q, axis=0)
    om = np.array([Dlt[:, j] @ Q[:, j] / nq[j] ** 2 if nq[j] > 0 else 0.0 for j in range(P.shape[1])])
    assert np.abs(Dlt - Q * om[None, :]).max() < 1e-13 * np.abs(P).max()
    assert om.min() >= 0.0 and (om > 0).sum() > P.shape[1] // 2
    AP, AQ = Ad @ P, Ad @ Q
    for j in range(P.shape[1]):
        g = AP[:, j] @ AQ[:, j]
        scale = np.linalg.norm(AP[:, j]) * np.linalg.norm(AQ[:, j]) + 1e-300
        if om[j] > 0:
            assert abs(g) < 1e-10 * scale, j
        else:
            assert g >= -1e-10 * scale, j


def test_pg_restriction_and_galerkin():
    """R comes from the same construction on A^T (so R != P^T on the fluid),
    A_c = R A P; on a symmetric block the Petrov-Galerkin restriction is P^T
    and the hierarchy that of the same dampings on both sides."""
    f, b = _fluid_only()
    A = b[0][0].toarray()
    o = Oracle(f, b, "AMG[pg=1]", coarse_max=100)
    P, R = o.matrix(0, 0, "P").toarray(), o.matrix(0, 0, "R").toarray()
    assert np.abs(R - P.T).max() > 1e-6 * np.abs(P).max()
    Ac = o.matrix(0, 1, "A").toarray()
    assert np.abs(Ac - R @ A @ P).max() < 1e-13 * np.abs(Ac).max()
    # the restriction is the transposed prolongator of A^T
    ot = Oracle(f, [[b[0][0].T.tocsr()]], "AMG[pg=1]", coarse_max=100)
    if np.array_equal(ot.aggregates(0, 0), o.aggregates(0, 0)):
        assert np.abs(ot.matrix(0, 0, "P").toarray() - R.T).max() < 1e-12 * np.abs(R).max()
    s = nfgen.tsi2d(nel=10)
    fs, bs = [s.fields[1]], [[s.blocks[1][1]]]
    osym = Oracle(fs, bs, "AMG[pg=1]", coarse_max=30)
    Ps, Rs = osym.matrix(0, 0, "P").toarray(), osym.matrix(0, 0, "R").toarray()
    assert np.abs(Rs - Ps.T).max() < 1e-13 * np.abs(Ps).max()


def test_pg_amg_gmres_reaches_dense_solution():
    f, b = _fluid_only(n=8, seed=5)
    A = b[0][0]
    rhs = np.random.default_rng(3).standard_normal(A.shape[0])
    o = Oracle(f, b, "AMG[smoother=sgs,omega=0.85,half=1,pg=1]", coarse_max=100)
    x, st = o.gmres(rhs, rtol=1e-10, maxit=300)
    xd = np.linalg.solve(A.toarray(), rhs)
    assert st["status"] == 0 and np.linalg.norm(x - xd) < 1e-7 * np.linalg.norm(xd)


def test_ddgs_few_aggregates_is_one_subdomain():
    """A level with fewer aggregates than ddmin (default 256) is one
    subdomain: the DD(GS) hierarchy then applies exactly the multicolour SGS;
    with ddmin = 1 the subdomains are the aggregates and the result differs."""
    s = nfgen.tsi2d(nel=16)
    f, b = [s.fields[1]], [[s.blocks[1][1]]]
    r = np.random.default_rng(8).standard_normal(f[0].ndof)
    z_sgs = Oracle(f, b, "AMG[smoother=sgs,omega=0.9,half=1]", coarse_max=30).precond_apply(r)
    z_dd = Oracle(f, b, "AMG[smoother=ddgs,omega=0.9,half=1]", coarse_max=30).precond_apply(r)
    z_dd1 = Oracle(f, b, "AMG[smoother=ddgs,omega=0.9,half=1,ddmin=1]", coarse_max=30).precond_apply(r)
    assert np.array_equal(z_sgs, z_dd)
    assert np.abs(z_dd1 - z_sgs).max() > 1e-8 * np.abs(z_sgs).max()


@pytest.mark.parametrize("half,degree", [(0, 2), (1, 3)])
def test_cheb_from_vcycle_dense_composition(half, degree):
    """cheb_from=1: multicolour Gauss-Seidel on the finest level, Chebyshev on
    the coarser ones.  The preconditioner equals the V(1,1) cycle (Sec. 3.1)
    composed from dense matrices of the oracle's hierarchy: the colour SOR
    splittings on level 0, the Chebyshev error polynomial
    T_k((theta - D^-1 A) / delta) / T_k(theta / delta) of the matrix D^-1 A
    on level 1 (matrix recurrence), an exact solve on level 2."""
    s = nfgen.tsi2d(nel=16)
    omega, ratio, boost = 0.9, 8.0, 1.1
    spec = f"AMG[smoother=sgs,omega={omega},half={half},cheb_from=1,degree={degree}]"
    o = Oracle([s.fields[0]], [[s.blocks[0][0]]], spec, coarse_max=20, cheb_ratio=ratio)
    assert o.nlevels(0) == 3
    A = [o.matrix(0, l, "A").toarray() for l in range(3)]
    P = [o.matrix(0, l, "P").toarray() for l in range(2)]
    R = [o.matrix(0, l, "R").toarray() for l in range(2)]
    # level 0: forward / backward colour splittings
    b0 = o.block_size(0, 0)
    gp, ga = oracle.node_graph(o.matrix(0, 0, "A"), b0)
    col, _ = oracle.color_nodes(gp, ga, 0)
    cr = np.repeat(col, b0)
    D = np.diag(np.diag(A[0]))
    Lf = np.where(cr[None, :] < cr[:, None], A[0], 0.0)
    Lb = np.where(cr[None, :] > cr[:, None], A[0], 0.0)

    def fwd(x, b):
        return np.linalg.solve(D / omega + Lf, b + (D / omega - A[0] + Lf) @ x)

    def bwd(x, b):
        return np.linalg.solve(D / omega + Lb, b + (D / omega - A[0] + Lb) @ x)

    # level 1: Chebyshev error polynomial of D^-1 A
    lam = o.lam(0, 1)
    hi, lo = boost * lam, lam / ratio
    th, de = (hi + lo) / 2, (hi - lo) / 2
    M1 = np.diag(1.0 / np.diag(A[1])) @ A[1]
    Y = (th * np.eye(len(M1)) - M1) / de
    Tm, T = np.eye(len(M1)), Y
    for _ in range(degree - 1):
        Tm, T = T, 2 * Y @ T - Tm
    E1 = T / np.cosh(degree * np.arccosh(th / de))

    def cheb(x, b):
        xs = np.linalg.solve(A[1], b)
        return xs - E1 @ (xs - x)

    def vcycle(l, b):
        if l == 2:
            return np.linalg.solve(A[2], b)
        z = np.zeros_like(b)
        if l == 0:
            x = fwd(z, b) if half else bwd(fwd(z, b), b)
        else:
            x = cheb(z, b)
        x = x + P[l] @ vcycle(l + 1, R[l] @ (b - A[l] @ x))
        if l == 0:
            return bwd(x, b) if half else bwd(fwd(x, b), b)
        return cheb(x, b)

    n = A[0].shape[0]
    want = np.stack([vcycle(0, e) for e in np.eye(n)])
    got = o.precond_apply(np.eye(n))
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    # Chebyshev on level 1 does change the result
    plain = Oracle([s.fields[0]], [[s.blocks[0][0]]], f"AMG[smoother=sgs,omega={omega},half={half}]",
                   coarse_max=20, cheb_ratio=ratio).precond_apply(np.eye(n))
    assert np.abs(plain - got).max() > 1e-6 * np.abs(got).max()
