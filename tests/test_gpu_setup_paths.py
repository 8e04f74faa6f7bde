"""Setup paths that the physics workloads at test size do not reach, against
the oracle: block products whose output rows overflow the LDS passes (up to
the register-owned fallback beyond all of them), and the greedy colouring with its
counters in global memory (more nodes than the LDS variant holds, or a node
with more than 255 smaller neighbours)."""
import numpy as np
import pytest
import scipy.sparse as sp

import nfgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


def _grid_plus_random(n, b, extra, seed):
    """Node graph: 27-point stencil on an n^3 grid plus `extra` random
    long-range neighbours per node (symmetrised); b dofs per node with dense
    blocks, symmetric and strictly diagonally dominant (SPD)."""
    rng = np.random.default_rng(seed)
    N = n ** 3
    ijk = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    rows, cols = [], []
    for d in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij")).reshape(3, -1).T:
        if not d.any():
            continue
        nb = ijk + d
        ok = np.all((nb >= 0) & (nb < n), axis=1)
        rows.append(np.nonzero(ok)[0])
        cols.append(np.ravel_multi_index(nb[ok].T, (n, n, n)))
    r = np.repeat(np.arange(N), extra)
    c = rng.integers(0, N, N * extra)
    keep = r != c
    rows.append(r[keep])
    cols.append(c[keep])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    G = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(N, N)).tocsr()
    G = ((G + G.T) > 0).astype(np.float64).tocoo()
    # dense b x b blocks with small random entries on every edge
    bi = np.repeat(G.row * b, b * b) + np.tile(np.repeat(np.arange(b), b), G.nnz)
    bj = np.repeat(G.col * b, b * b) + np.tile(np.tile(np.arange(b), b), G.nnz)
    v = -rng.uniform(0.0, 1.0, bi.size)
    A = sp.coo_matrix((v, (bi, bj)), shape=(N * b, N * b)).tocsr()
    A = (A + A.T) * 0.5
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = A.tocsr()
    A.sort_indices()
    ns = np.zeros((b, N * b))
    for c_ in range(b):
        ns[c_, c_::b] = 1.0
    return A, ns


def _lap2d(m):
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m, m))
    I = sp.identity(m)
    A = (sp.kron(T, I) + sp.kron(I, T)).tocsr()
    A.sort_indices()
    return A


def _system(A, b, ns):
    f = nfgen.Field("f", A.shape[0], b, ns)
    rhs = np.random.default_rng(1).uniform(-1, 1, (1, A.shape[0]))
    return nfgen.BlockSystem([f], [[A]], rhs)


def _compare(s, spec, tol=1e-10, **opts):
    from paper_1605_01522_amd import NField
    dev = torch.device("cuda:0")
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = NField(s.fields, s.blocks, spec, **opts)
    assert g.nlevels(0) == o.nlevels(0)
    for l in range(o.nlevels(0)):
        assert g.level_size(0, l, 0) == o.level_size(0, l, 0)
    r = np.random.default_rng(7).standard_normal((2, s.n))
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    for k in range(2):
        assert np.linalg.norm(zg[k] - zo[k]) <= tol * np.linalg.norm(zo[k]), k
    return g


@pytest.mark.parametrize("n,b", [(21, 4), (15, 8)])
def test_block_products_long_rows(n, b):
    """n^3 nodes of b dofs with random long-range couplings.  b = 4: 9,261
    fine A P rows, all beyond the 512-value pass, within the 2,048-value one;
    b = 8: almost every A P and every R (A P) row beyond 2,048 values."""
    _say(f"case block products, long rows, n={n} b={b}")
    from paper_1605_01522_amd import NField
    A, ns = _grid_plus_random(n, b, 3, seed=5)
    s = _system(A, b, ns)
    g = _compare(s, "AMG", coarse_max=64)
    sca = NField(s.fields, s.blocks, "AMG", coarse_max=64, block_products=0)
    r = torch.tensor(np.random.default_rng(9).standard_normal((1, s.n)), device=torch.device("cuda:0"))
    assert np.array_equal(g.precond_apply(r).cpu().numpy(), sca.precond_apply(r).cpu().numpy())
    g.close()
    sca.close()


def test_block_products_beyond_lds():
    """Monolithic AMG over a coarsened scalar field and a dense field of 150
    nodes x 8 dofs that is not coarsened (P = I): its Galerkin block keeps
    rows of 150 blocks of 8 x 8 (9,600 values), beyond every LDS pass."""
    _say("case block products beyond LDS (dense uncoarsened field)")
    from paper_1605_01522_amd import NField
    rng = np.random.default_rng(11)
    m = 20
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(m, m))
    I = sp.identity(m)
    A0 = (sp.kron(sp.kron(T, I), I) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(I, I), T)).tocsr()
    A0.sort_indices()
    n1 = 150 * 8
    M = rng.uniform(-1.0, 1.0, (n1, n1))
    M = (M + M.T) * 0.5
    M += np.diag(np.abs(M).sum(axis=1) + 1.0)
    A1 = sp.csr_matrix(M)
    A1.sort_indices()
    ns1 = np.zeros((8, n1))
    for c in range(8):
        ns1[c, c::8] = 1.0
    f0 = nfgen.Field("a", A0.shape[0], 1, np.ones((1, A0.shape[0])))
    f1 = nfgen.Field("b", n1, 8, ns1)
    rhs = rng.uniform(-1, 1, (1, A0.shape[0] + n1))
    s = nfgen.BlockSystem([f0, f1], [[A0, None], [None, A1]], rhs)
    opts = dict(coarse_max=1500)
    dev = torch.device("cuda:0")
    o = oracle.Oracle(s.fields, s.blocks, "AMG(BGS)", **opts)
    g = NField(s.fields, s.blocks, "AMG(BGS)", **opts)
    sca = NField(s.fields, s.blocks, "AMG(BGS)", block_products=0, **opts)
    assert g.nlevels(0) == o.nlevels(0) >= 2
    r = np.random.default_rng(7).standard_normal((2, s.n))
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    zs = sca.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    assert np.array_equal(zg, zs)
    for k in range(2):
        assert np.linalg.norm(zg[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k]), k
    g.close()
    sca.close()


def test_coloring_many_nodes():
    """84,100 nodes: the colouring keeps its counters in global memory."""
    _say("case colouring, 84,100 nodes")
    A = _lap2d(290)
    s = _system(A, 1, np.ones((1, A.shape[0])))
    _compare(s, "AMG[smoother=sgs]").close()


def test_coloring_wide_node():
    """A node coupled to 300 smaller nodes: more than a byte counter holds."""
    _say("case colouring, node with 300 smaller neighbours")
    m = 40
    L = _lap2d(m).tolil()
    n = m * m + 1
    A = sp.lil_matrix((n, n))
    A[: n - 1, : n - 1] = L
    idx = np.random.default_rng(3).choice(n - 1, 300, replace=False)
    for i in idx:
        A[n - 1, i] = A[i, n - 1] = -0.01
        A[i, i] += 0.01
    A[n - 1, n - 1] = 300 * 0.01 + 1.0
    A = A.tocsr()
    A.sort_indices()
    s = _system(A, 1, np.ones((1, n)))
    _compare(s, "AMG[smoother=sgs]", coarse_max=50).close()


@pytest.mark.parametrize("n", [600, 2100])
def test_node_graph_rows_differ(n):
    """Two dofs per node on a chain; dof 0 of node 0 is coupled to dof 0 of
    every node.  The two rows of each node then reach different nodes, so
    the node graph and the block columns cannot take the first row's set:
    they sort the node's entries (n = 600), and for node 0 at n = 2,100 its
    2,100-entry row is beyond the sort's capacity and is merged serially."""
    _say(f"case node graph with differing rows, n={n}")
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(n, n))
    A = sp.kron(T, sp.identity(2)).tolil()
    for j in range(1, n):
        A[0, 2 * j] = A[2 * j, 0] = -0.01
        A[2 * j, 2 * j] += 0.01
    A[0, 0] += 0.01 * (n - 1) + 1.0
    A = A.tocsr()
    A.sort_indices()
    ns = np.zeros((2, 2 * n))
    ns[0, 0::2] = 1.0
    ns[1, 1::2] = 1.0
    s = _system(A, 2, ns)
    _compare(s, "AMG[smoother=sgs]", coarse_max=40).close()
    _compare(s, "AMG", coarse_max=40).close()
