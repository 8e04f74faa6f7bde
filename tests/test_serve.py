"""Serving loop: batch formation and admission (CPU, fake contexts), and on
the GPU a replayed trace whose every request gives the same bits as a solo
solve."""
import numpy as np
import pytest

import nfgen
from paper_1605_01522_amd import serve


class _FakeCtx:
    def __init__(self, nbytes):
        self.nbytes = nbytes
        self.closed = False

    def footprint_bytes(self):
        return self.nbytes

    def close(self):
        self.closed = True


class _Sys:
    def __init__(self, n):
        self.n = n


def _server(budget):
    srv = serve.Server.__new__(serve.Server)
    srv.workers = 2
    srv.max_cols = 8
    srv.budget = budget
    srv.ctx = [serve.OrderedDict() for _ in range(2)]
    srv.busy_keys = [set(), set()]
    srv.bytes_est = {}
    srv.systems = {}
    srv.system_for_key = lambda key: _Sys(100 * key)
    return srv


def _items(reqs):
    return [serve.Served(dict(id=i, key=k, nrhs=c, arrival_s=0.0)) for i, (k, c) in enumerate(reqs)]


def test_batch_joins_same_key_up_to_max_columns():
    srv = _server(1 << 40)
    items = _items([(16, 3), (32, 2), (16, 4), (16, 2), (32, 8)])
    waiting = list(range(5))
    b = srv._take_batch(waiting, items, 0)
    assert b == [0, 2]                       # 3 + 4 columns; the next (2) would exceed 8
    assert waiting == [1, 3, 4]
    b = srv._take_batch(waiting, items, 0)
    assert b == [1]                          # 2 + 8 > 8
    assert srv._take_batch(waiting, items, 0) == [3]


def test_admission_evicts_idle_contexts_and_waits_when_full():
    srv = _server(1000)
    srv.bytes_est = {16: 600, 32: 600}
    srv.ctx[0][16] = _FakeCtx(600)
    items = _items([(32, 1)])
    waiting = [0]
    # an idle context is evicted to make room
    assert srv._take_batch(waiting, items, 1) == [0]
    assert 16 not in srv.ctx[0]
    # a busy context is not evicted: the request waits
    srv.ctx[0][16] = _FakeCtx(600)
    srv.busy_keys[0].add(16)
    items = _items([(32, 1)])
    waiting = [0]
    assert srv._take_batch(waiting, items, 1) is None and waiting == [0]


@pytest.mark.gpu
def test_served_trace_matches_solo_bitwise():
    import torch
    from paper_1605_01522_amd import NField
    grids = (16, 24, 32)
    trace = nfgen.request_trace(24, rate=400.0, grids=grids, seed=3)
    for r in trace:
        r["key"] = r["grid"]
    systems = {g: nfgen.tsi2d(nel=g) for g in grids}
    opts = dict(sweeps=2, order="bwd")
    srv = serve.Server(lambda g: systems[g], "BGS(AMG)", opts, workers=3, max_cols=8)
    items = srv.run(trace, lambda req: nfgen.request_rhs(req, systems[req["grid"]].n), time_scale=1.0)
    summ = serve.summarize(items)
    print(summ, flush=True)
    assert summ["all_converged"]
    assert max(it.batch_cols for it in items) > 1        # some requests shared a launch
    solo = {g: NField(systems[g].fields, systems[g].blocks, "BGS(AMG)", hier_fp32=1, **opts) for g in grids}
    for it in items:
        g = it.req["grid"]
        B = torch.tensor(nfgen.request_rhs(it.req, systems[g].n), device="cuda")
        x, st = solo[g].gmres_solve(B, flexible=1, rtol=1e-8)
        assert np.array_equal(x.cpu().numpy(), it.x), it.req["id"]
        A = systems[g].assembled()
        for k in range(it.req["nrhs"]):
            assert np.linalg.norm(B[k].cpu().numpy() - A @ it.x[k]) < 1e-8 * np.linalg.norm(B[k].cpu().numpy())
    srv.close()
