"""The allocation-free GMRES entry point (nfield_gmres_solve_noalloc): its
Krylov workspace lives in the library's static scratch array.  Checked
against nfield_gmres_solve, which runs the same kernels on the context's own
buffers, on two calls in a row on one device (the second with a smaller
input), and for its size limit."""
import sys

import numpy as np
import pytest

import nfgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1605_01522_amd import nfield
    nfield.lib()
    return torch.device("cuda:0")


def _pair(s, spec, **opts):
    """Two contexts of the same system: one for each entry point, so that the
    allocating one cannot hand its buffers to the other."""
    from paper_1605_01522_amd import NField
    return NField(s.fields, s.blocks, spec, **opts), NField(s.fields, s.blocks, spec, **opts)


def _check(s, spec, flexible, opts, dev):
    ga, gn = _pair(s, spec, **opts)
    B = torch.tensor(s.rhs, device=dev)
    fp0 = gn.footprint_bytes()
    xn, stn = gn.gmres_solve(B, rtol=1e-8, flexible=flexible, noalloc=True)
    torch.cuda.synchronize()
    assert gn.footprint_bytes() == fp0          # nothing allocated through the context
    xa, sta = ga.gmres_solve(B, rtol=1e-8, flexible=flexible)
    torch.cuda.synchronize()
    A = s.assembled()
    for k in range(s.rhs.shape[0]):
        assert stn[k]["status"] == 0 and sta[k]["status"] == 0
        assert stn[k]["iters"] == sta[k]["iters"]
        xk = xn[k].cpu().numpy()
        assert np.linalg.norm(s.rhs[k] - A @ xk) / np.linalg.norm(s.rhs[k]) < 1e-8
    assert torch.equal(xn, xa)                   # the same kernels in the same order
    ga.close()
    gn.close()


def test_noalloc_matches_allocating_solve_twice(dev):
    # first call: 3 columns of the 32 x 32 TSI-like system, plain FP64 GMRES
    _say("case noalloc call 1: tsi2d nel=32, 3 rhs, plain")
    s1 = nfgen.tsi2d(nel=32, seed=1, nrhs=3)
    _check(s1, "BGS(AMG)", 0, dict(sweeps=2, order="bwd"), dev)
    # second call, smaller: 1 column of a 16 x 16 system, FP32 hierarchy in
    # flexible GMRES (the FP32 staging in the scratch too)
    _say("case noalloc call 2: tsi2d nel=16, 1 rhs, precision form")
    s2 = nfgen.tsi2d(nel=16, seed=2, nrhs=1)
    _check(s2, "BGS(AMG)", 1, dict(sweeps=2, order="bwd", hier_fp32=1), dev)


def test_noalloc_rejects_workspace_beyond_scratch(dev):
    """8 columns of restart 63 in flexible form on 49,665 dofs need about
    8 * 49,665 * (64 + 63 + 4) * 8 bytes = 416 MB > 256 MiB: ENOMEM, and x
    is left untouched."""
    _say("case noalloc size limit")
    from paper_1605_01522_amd import NField, nfield
    s = nfgen.tsi2d(nel=128, seed=0, nrhs=8)
    g = NField(s.fields, s.blocks, "BGS(AMG)", sweeps=2, order="bwd")
    B = torch.tensor(s.rhs, device=dev)
    x = torch.full_like(B, 7.0)
    with pytest.raises(nfield.NFieldError) as e:
        g.gmres_solve(B, x, restart=63, flexible=1, noalloc=True)
    assert e.value.code == -2
    assert b"static scratch" in nfield.lib().nfield_last_error()
    assert float(x.min()) == 7.0 and float(x.max()) == 7.0
    # the same call with one column fits
    x1, st = g.gmres_solve(B[0].contiguous(), restart=63, flexible=1, noalloc=True)
    assert st[0]["status"] == 0
    g.close()
