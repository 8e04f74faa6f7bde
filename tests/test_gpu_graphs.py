"""Preconditioner replayed from a captured HIP graph against the same
preconditioner launched kernel by kernel: every replay, with the program's
own eager work and synchronisations between replays, and after a rebuild,
gives the same bits."""
import numpy as np
import pytest

import nfgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    ("tsi", lambda: nfgen.tsi2d(nel=24, seed=3), "BGS(AMG)", dict(sweeps=2, order="bwd")),
    ("fsi", lambda: nfgen.fsi3d(n=10, layers=2, seed=0), "SIMPLE(BGS(AMG);AMG[smoother=sgs,omega=0.69])",
     dict(split=[0, 0, 1])),
    ("lung", lambda: nfgen.lung3d(n=8, depth=4, acinus=2, seed=0), "SIMPLE(AMG[smoother=sgs,omega=0.79](BGS);LU)",
     dict(split=[0, 0, 1])),
    ("tsi-fp32", lambda: nfgen.tsi2d(nel=24, seed=3), "BGS(AMG)", dict(sweeps=2, order="bwd", hier_fp32=1)),
    ("lung-cheb-coarse", lambda: nfgen.lung3d(n=16, depth=7, acinus=4, seed=2),
     "SIMPLE(AMG[smoother=sgs,omega=0.79,cheb_from=1,degree=3](BGS);LU)",
     dict(split=[0, 0, 1], simplec_mode=2, coarse_max=200, cheb_ratio=8.0)),
]


@pytest.mark.parametrize("name,make,spec,opts", CASES, ids=[c[0] for c in CASES])
def test_graph_replay_matches_eager(name, make, spec, opts):
    assert torch.cuda.is_available()
    from paper_1605_01522_amd import NField
    print(f"case graphs {name}", flush=True)
    s = make()
    dev = torch.device("cuda:0")
    eager = NField(s.fields, s.blocks, spec, graphs=0, **opts)
    graph = NField(s.fields, s.blocks, spec, graphs=1, **opts)
    rng = np.random.default_rng(11)
    for nrhs in (1, 3):
        r = torch.tensor(rng.standard_normal((nrhs, s.n)), device=dev)
        ref = eager.precond_apply(r).cpu().numpy()
        for rep in range(4):
            z = graph.precond_apply(r).cpu().numpy()
            assert np.array_equal(z, ref), (name, nrhs, rep)
            # eager work of the program between replays
            y = graph.matvec(r)
            _ = (y * 2.0 - r).sum().item()
            torch.cuda.synchronize()
    # after a rebuild the graph is captured again from the new hierarchy
    graph.rebuild()
    eager.rebuild()
    r = torch.tensor(rng.standard_normal((2, s.n)), device=dev)
    assert np.array_equal(graph.precond_apply(r).cpu().numpy(), eager.precond_apply(r).cpu().numpy())
    flex = 1 if opts.get("hier_fp32") else 0
    b = torch.tensor(s.rhs[0], device=dev)
    xg, sg = graph.gmres_solve(b, rtol=1e-8, maxit=500, flexible=flex)
    xe, se = eager.gmres_solve(b, rtol=1e-8, maxit=500, flexible=flex)
    assert sg[0]["iters"] == se[0]["iters"] and sg[0]["status"] == se[0]["status"] == 0
    assert np.array_equal(xg.cpu().numpy(), xe.cpu().numpy())
    graph.close()
    eager.close()
