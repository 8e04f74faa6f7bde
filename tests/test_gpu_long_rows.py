"""Sparse products and transposes with rows beyond the LDS tables (more than
4096 entries): a field whose matrix has one dense row and column, so that
A P_tent, R = P^T and R A P all have such rows.  GPU hierarchy and
preconditioner against the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import nfgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bordered(n, seed):
    rng = np.random.default_rng(seed)
    main = np.full(n, 4.0)
    off = np.full(n - 1, -1.0)
    A = sp.diags([off, main, off], [-1, 0, 1], format="lil")
    border = 1e-3 * rng.uniform(0.5, 1.0, n)
    A[0, 1:] = border[1:]
    A[1:, 0] = border[1:, None]
    A[0, 0] = 4.0 + border.sum()
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


@pytest.mark.parametrize("n", [6000, 9000])
def test_long_row_products_parity(n):
    assert torch.cuda.is_available()
    from paper_1605_01522_amd import NField
    print(f"case long rows n={n}", flush=True)
    A = _bordered(n, n)
    f = nfgen.Field("f", n, 1, np.ones((1, n)))
    o = oracle.Oracle([f], [[A]], "AMG", coarse_max=50)
    g = NField([f], [[A]], "AMG", coarse_max=50)
    assert g.nlevels(0) == o.nlevels(0) >= 2
    for l in range(o.nlevels(0)):
        assert g.level_size(0, l) == o.level_size(0, l)
        for which in ("A", "P", "R"):
            if which != "A" and l + 1 == o.nlevels(0):
                continue
            Mo, Mg = o.matrix(0, l, which), g.matrix(0, l, which)
            assert np.array_equal(Mo.indptr, Mg.indptr) and np.array_equal(Mo.indices, Mg.indices), (l, which)
            assert np.abs(Mo.data - Mg.data).max() <= 1e-12 * np.abs(Mo.data).max(), (l, which)
    # the dense row really went through the long-row paths
    assert o.matrix(0, 0, "R").getnnz(axis=1).max() > 4096
    r = np.random.default_rng(1).standard_normal(n)
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)


def test_long_row_schur_product_parity():
    """SIMPLE's S~ = A22 - A21 D~^-1 A12 with one dense row of A21: that row
    of the product has every column of the Schur field (> 4096)."""
    assert torch.cuda.is_available()
    from paper_1605_01522_amd import NField
    print("case long-row Schur product", flush=True)
    n1, n2 = 6000, 5000
    rng = np.random.default_rng(3)
    A11 = sp.diags([np.full(n1 - 1, -1.0), np.full(n1, 4.0), np.full(n1 - 1, -1.0)], [-1, 0, 1], format="csr")
    A22 = sp.diags([np.full(n2 - 1, -1.0), np.full(n2, 4.0), np.full(n2 - 1, -1.0)], [-1, 0, 1], format="csr")
    A21 = sp.lil_matrix((n2, n1))
    A21[0, :] = 1e-3 * rng.uniform(0.5, 1.0, n1)
    for i in range(1, n2):
        A21[i, i] = 0.1
    A21 = sp.csr_matrix(A21)
    A12 = sp.csr_matrix(A21.T)
    blocks = [[A11, A12], [A21, A22]]
    for row in blocks:
        for b in row:
            b.sort_indices()
    fields = [nfgen.Field("a", n1, 1, np.ones((1, n1))), nfgen.Field("b", n2, 1, np.ones((1, n2)))]
    spec = "SIMPLE(AMG;AMG)"
    o = oracle.Oracle(fields, blocks, spec, coarse_max=50)
    g = NField(fields, blocks, spec, coarse_max=50)
    r = np.random.default_rng(4).standard_normal(n1 + n2)
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)
    # the Schur hierarchy's fine matrix is S~; its first row is full
    S = o.matrix(1, 0, "A")
    assert S.getnnz(axis=1).max() == n2
    Sg = g.matrix(1, 0, "A")
    assert np.array_equal(S.indices, Sg.indices) and np.abs(S.data - Sg.data).max() <= 1e-12 * np.abs(S.data).max()
