"""Independent parts of the preconditioner set up concurrently (host thread,
stream and block cache per part) against the same setup done one part after
another: the same hierarchies, the same preconditioner bits and the same
solution, also after rebuilds that reuse the parts' caches."""
import numpy as np
import pytest

import nfgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    ("tsi", lambda: nfgen.tsi2d(nel=24, seed=3), "BGS(AMG)", dict(sweeps=2, order="bwd")),
    ("fsi", lambda: nfgen.fsi3d(n=10, layers=2, seed=0), "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.65])",
     dict(split=[0, 0, 1])),
    ("lung", lambda: nfgen.lung3d(n=8, depth=4, acinus=2, seed=0), "SIMPLE(AMG[smoother=sgs,omega=0.79](BGS);LU)",
     dict(split=[0, 0, 1])),
    ("fsi-fp32", lambda: nfgen.fsi3d(n=10, layers=2, seed=0), "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.65])",
     dict(split=[0, 0, 1], hier_fp32=1)),
]


@pytest.mark.parametrize("name,make,spec,opts", CASES, ids=[c[0] for c in CASES])
def test_parallel_setup_same_bits(name, make, spec, opts):
    assert torch.cuda.is_available()
    from paper_1605_01522_amd import NField
    print(f"case parallel setup {name}", flush=True)
    s = make()
    dev = torch.device("cuda:0")
    par = NField(s.fields, s.blocks, spec, parallel_setup=1, **opts)
    seq = NField(s.fields, s.blocks, spec, parallel_setup=0, **opts)
    rng = np.random.default_rng(2)
    for rebuild in range(3):
        if rebuild:
            par.rebuild()
            seq.rebuild()
        assert par.hier_count() == seq.hier_count()
        for h in range(par.hier_count()):
            assert par.nlevels(h) == seq.nlevels(h)
            for l in range(par.nlevels(h)):
                for f in range(par.nfields(h)):
                    assert par.level_size(h, l, f) == seq.level_size(h, l, f)
        r = torch.tensor(rng.standard_normal((2, s.n)), device=dev)
        assert np.array_equal(par.precond_apply(r).cpu().numpy(), seq.precond_apply(r).cpu().numpy()), (name, rebuild)
    flex = 1 if opts.get("hier_fp32") else 0
    b = torch.tensor(s.rhs[0], device=dev)
    xp, sp_ = par.gmres_solve(b, rtol=1e-8, maxit=500, flexible=flex)
    xs, ss = seq.gmres_solve(b, rtol=1e-8, maxit=500, flexible=flex)
    assert sp_[0]["status"] == ss[0]["status"] == 0 and sp_[0]["iters"] == ss[0]["iters"]
    assert np.array_equal(xp.cpu().numpy(), xs.cpu().numpy())
    assert par.footprint_bytes() > 0
    par.close()
    seq.close()


@pytest.mark.parametrize("parallel", [1, 0])
def test_error_in_a_concurrent_part(parallel):
    """A singular diagonal entry in the second BGS field (set up on a side
    thread): the setup fails with ESINGULAR like the sequential one, and the
    library stays usable."""
    from paper_1605_01522_amd import NField, nfield
    print(f"case parallel setup error path parallel={parallel}", flush=True)
    s = nfgen.tsi2d(nel=20, seed=1)     # both fields above the coarse size
    B = s.blocks[1][1].tolil()
    B[3, 3] = 0.0
    B = B.tocsr()
    B.eliminate_zeros()
    B.sort_indices()
    bad = [[s.blocks[0][0], s.blocks[0][1]], [s.blocks[1][0], B]]
    with pytest.raises(nfield.NFieldError) as e:
        NField(s.fields, bad, "BGS(AMG)", parallel_setup=parallel, sweeps=2, order="bwd")
    assert e.value.code == -3
    g = NField(s.fields, s.blocks, "BGS(AMG)", parallel_setup=parallel, sweeps=2, order="bwd")
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=torch.device("cuda:0")), rtol=1e-8)
    assert st[0]["status"] == 0
    g.close()
