"""Galerkin products formed block by block against the same products formed
entry by entry: the hierarchies have the same sizes and the preconditioners
give the same bits (same pattern, same summation order)."""
import numpy as np
import pytest

import nfgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    ("tsi", lambda: nfgen.tsi2d(nel=24, seed=3), "BGS(AMG)", dict(sweeps=2, order="bwd")),
    ("fsi", lambda: nfgen.fsi3d(n=10, layers=2, seed=0), "SIMPLE(BGS(AMG);AMG[smoother=sgs,omega=0.69])",
     dict(split=[0, 0, 1])),
    ("fsi-mono", lambda: nfgen.fsi3d(n=8, layers=2, seed=1), "AMG(BGS)", dict(coarse_max=50)),
    ("lung-simple", lambda: nfgen.lung3d(n=8, depth=4, acinus=2, seed=0), "SIMPLE(AMG[smoother=sgs,omega=0.79](BGS);LU)",
     dict(split=[0, 0, 1])),
    ("lung-mono", lambda: nfgen.lung3d(n=8, depth=4, acinus=2, seed=0), "AMG(SIMPLE)", dict(split=[0, 0, 1])),
    ("tsi-fp32", lambda: nfgen.tsi2d(nel=24, seed=3), "BGS(AMG)", dict(sweeps=2, order="bwd", hier_fp32=1)),
]


@pytest.mark.parametrize("name,make,spec,opts", CASES, ids=[c[0] for c in CASES])
def test_block_products_same_bits(name, make, spec, opts):
    assert torch.cuda.is_available()
    from paper_1605_01522_amd import NField
    print(f"case block products {name}", flush=True)
    s = make()
    dev = torch.device("cuda:0")
    blk = NField(s.fields, s.blocks, spec, block_products=1, **opts)
    sca = NField(s.fields, s.blocks, spec, block_products=0, **opts)
    assert blk.hier_count() == sca.hier_count()
    for h in range(blk.hier_count()):
        assert blk.nlevels(h) == sca.nlevels(h)
        for l in range(blk.nlevels(h)):
            for f in range(blk.nfields(h)):
                assert blk.level_size(h, l, f) == sca.level_size(h, l, f)
    r = torch.tensor(np.random.default_rng(5).standard_normal((3, s.n)), device=dev)
    zb = blk.precond_apply(r).cpu().numpy()
    zs = sca.precond_apply(r).cpu().numpy()
    assert np.array_equal(zb, zs), (name, np.abs(zb - zs).max())
    blk.close()
    sca.close()
