"""Slot batches (nfield_batch_*): columns that join a running batch at an
Arnoldi step boundary and leave it when finished give the same bits, the
same iteration counts and the same status as a solve of each column alone;
the edge cases (zero and non-finite right-hand sides, the iteration limit,
an initial guess) and the host-side argument checks."""
import sys

import numpy as np
import pytest

import nfgen
from bench import SERVE_OPTS, SERVE_SPEC

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


@pytest.fixture(scope="module")
def system():
    return nfgen.tsi2d(nel=24)


def _solve_kw(fp32):
    return dict(restart=4, maxit=200, flexible=1 if fp32 else 0, rtol=1e-8)


@pytest.mark.parametrize("fp32", [True, False], ids=["fp32_hier_flexible", "fp64_plain"])
def test_batch_joins_and_leaves_match_solo_bitwise(dev, system, fp32):
    """Seven columns through four slots: three start together, a fourth joins
    after three steps while they are mid-cycle, and every slot that frees is
    refilled at the next boundary.  GMRES(4) makes every column restart, so
    cycle ends, true-residual tests and cycle starts of some columns fall in
    the steps where others are mid-cycle."""
    from paper_1605_01522_amd import NField
    from paper_1605_01522_amd.nfield import Batch
    _say(f"case batch joins/leaves vs solo, fp32 hierarchy {fp32}")
    s = system
    g = NField(s.fields, s.blocks, SERVE_SPEC, hier_fp32=1 if fp32 else 0, **SERVE_OPTS)
    kw = _solve_kw(fp32)
    rhs = torch.tensor(nfgen.uniform_rhs(s.n, 7, 11), device=dev)
    bat = Batch(g, 4, **kw)
    X = torch.zeros_like(rhs)
    stats = [None] * 7
    slot_col = {}
    nxt = 0
    for q in range(3):
        bat.submit(q, rhs[nxt])
        slot_col[q] = nxt
        nxt += 1
    steps = 0
    joined_mid_cycle = False
    while any(st is None for st in stats):
        if steps == 3:
            assert all(bat.state(q) == 2 for q in range(3))   # all three mid-cycle
            bat.submit(3, rhs[nxt])
            slot_col[3] = nxt
            nxt += 1
            joined_mid_cycle = True
        done, nact = bat.step()
        steps += 1
        for q in done:
            c = slot_col.pop(q)
            stats[c] = bat.take(q, X[c])
            if nxt < 7:
                bat.submit(q, rhs[nxt])
                slot_col[q] = nxt
                nxt += 1
        assert steps < 2000
    torch.cuda.synchronize()
    assert joined_mid_cycle
    iters = 0
    for c in range(7):
        xs, st = g.gmres_solve(rhs[c].contiguous(), **kw)
        assert torch.equal(xs, X[c]), c
        for k in ("iters", "restarts", "status", "relres"):
            assert st[0][k] == stats[c][k], (c, k, st[0][k], stats[c][k])
        assert stats[c]["status"] == 0 and stats[c]["restarts"] >= 1
        iters += st[0]["iters"]
    _say(f"{steps} batch steps for {iters} Arnoldi steps of 7 columns")
    assert steps < iters / 2            # the columns shared their launches
    bat.close()
    g.close()


def test_batch_edge_cases(dev, system):
    """Zero right-hand side: finished at the first step with 0 iterations and
    x = x0 = 0.  Non-finite one: ENAN.  An iteration limit: NOT_CONVERGED
    with the solo iterate.  An initial guess: the solo result from it."""
    from paper_1605_01522_amd import NField, nfield
    from paper_1605_01522_amd.nfield import Batch
    _say("case batch edge cases")
    s = system
    g = NField(s.fields, s.blocks, SERVE_SPEC, hier_fp32=1, **SERVE_OPTS)
    kw = _solve_kw(True)
    rhs = torch.tensor(nfgen.uniform_rhs(s.n, 2, 5), device=dev)
    zero = torch.zeros(s.n, dtype=torch.float64, device=dev)
    bad = rhs[0].clone()
    bad[7] = float("nan")
    x0 = 0.5 * rhs[1]
    bat = Batch(g, 4, **kw)
    bat.submit(0, zero)
    bat.submit(1, bad)
    bat.submit(2, rhs[0])
    bat.submit(3, rhs[1], x0=x0)
    done, nact = bat.step()
    assert sorted(done) == [0, 1] and nact == 2
    x = torch.ones(s.n, dtype=torch.float64, device=dev)
    st = bat.take(0, x)
    torch.cuda.synchronize()
    assert st["status"] == 0 and st["iters"] == 0 and not torch.any(x != 0)
    st = bat.take(1)
    assert st["status"] == -5
    X = {}
    while bat.state(2) != 4 or bat.state(3) != 4:
        bat.step()
    for q in (2, 3):
        X[q] = torch.empty(s.n, dtype=torch.float64, device=dev)
        X[q + 10] = bat.take(q, X[q])
    xs, st2 = g.gmres_solve(rhs[0].contiguous(), **kw)
    assert torch.equal(xs, X[2]) and st2[0]["iters"] == X[12]["iters"]
    xg = x0.clone()
    xs, st3 = g.gmres_solve(rhs[1].contiguous(), xg, **kw)
    assert torch.equal(xs, X[3]) and st3[0]["iters"] == X[13]["iters"]
    bat.close()
    # the iteration limit
    kw3 = dict(kw, maxit=3)
    bat = Batch(g, 2, **kw3)
    bat.submit(0, rhs[0])
    while bat.state(0) != 4:
        bat.step()
    xb = torch.empty(s.n, dtype=torch.float64, device=dev)
    stb = bat.take(0, xb)
    xs, sts = g.gmres_solve(rhs[0].contiguous(), **kw3)
    assert stb["status"] == 1 and sts[0]["status"] == 1 and stb["iters"] == 3
    assert torch.equal(xs, xb) and stb["relres"] == sts[0]["relres"]
    # host-side argument checks
    bat.submit(1, rhs[1])
    with pytest.raises(nfield.NFieldError):
        bat.submit(1, rhs[0])          # slot busy
    with pytest.raises(nfield.NFieldError):
        bat.take(1)                    # not finished
    with pytest.raises(nfield.NFieldError):
        Batch(g, 9, **kw)              # more slots than max_rhs
    while bat.state(1) != 4:
        bat.step()
    bat.take(1)
    assert bat.nbytes() > 0
    bat.close()
    g.close()
