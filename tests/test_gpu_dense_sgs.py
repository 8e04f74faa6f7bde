"""Levels with many Gauss-Seidel colours apply their symmetric sweep as a
precomputed dense affine map; the preconditioner stays the oracle's (same
sweep, other summation order), and the dense kernel is really the one used."""
import numpy as np
import pytest

import nfgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPEC = "SIMPLE(BGS(AMG);AMG[smoother=sgs,omega=0.69])"


@pytest.mark.parametrize("n,layers,steps", [(20, 4, 1), (20, 4, 2)])
def test_dense_sweep_matches_oracle(n, layers, steps):
    assert torch.cuda.is_available()
    from paper_1605_01522_amd import NField, nfield
    print(f"case dense sgs fsi3d n={n} steps={steps}", flush=True)
    s = nfgen.fsi3d(n=n, layers=layers, seed=0)
    spec = SPEC.replace("omega=0.69", f"omega=0.69,steps={steps}")
    o = oracle.Oracle(s.fields, s.blocks, spec, split=[0, 0, 1])
    nfield.nfield_prof_enable(1)
    g = NField(s.fields, s.blocks, spec, split=[0, 0, 1])
    r = np.random.default_rng(5).standard_normal((2, s.n))
    zg = g.precond_apply(torch.tensor(r, device="cuda")).cpu().numpy()
    torch.cuda.synchronize()
    prof = nfield.nfield_prof_read()
    nfield.nfield_prof_enable(0)
    assert any(p["mode"] == "sgs_dense" for p in prof), [p["mode"] for p in prof]
    zo = o.precond_apply(r)
    for k in range(2):
        assert np.linalg.norm(zg[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k])
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device="cuda"), rtol=1e-8, maxit=500)
    xo, so = o.gmres(s.rhs[0], rtol=1e-8, maxit=500)
    x = x.cpu().numpy()
    assert st[0]["status"] == 0 and np.linalg.norm(s.rhs[0] - A @ x) < 1e-8 * np.linalg.norm(s.rhs[0])
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    assert abs(st[0]["iters"] - so["iters"]) <= 2
    g.close()
