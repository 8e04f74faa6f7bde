"""Serving loop: column admission at step boundaries, key choice and memory
admission (CPU, fake contexts), and on
the GPU a replayed trace whose every request gives the same bits as a solo
solve."""
import numpy as np
import pytest

import nfgen
from bench import SERVE_OPTS, SERVE_SPEC
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
    srv.max_wait_s = 0.02
    srv.max_keys = 2
    srv._init_state()
    srv.system_for_key = lambda key: _Sys(100 * key)
    return srv


def _items(reqs, t=0.0):
    out = [serve.Served(dict(id=i, key=k, nrhs=c, arrival_s=t)) for i, (k, c) in enumerate(reqs)]
    for it in out:
        it.t_arrive = t
    return out


def _cached(srv, w, key, nbytes):
    c = (_FakeCtx(nbytes), _FakeCtx(0))
    srv.ctx[w][key] = c
    return c


def test_admission_fills_free_slots_in_arrival_order_by_column():
    srv = _server(1 << 40)
    items = _items([(16, 3), (32, 2), (16, 4), (16, 2), (32, 8)])
    waiting = list(range(5))
    # 8 free slots: request 0's 3 columns, request 2's 4, one of request 3's
    adm = srv._admit(waiting, items, 16, 8, 0)
    assert adm == [(0, 0), (0, 1), (0, 2), (2, 0), (2, 1), (2, 2), (2, 3), (3, 0)]
    assert waiting == [1, 3, 4] and items[3].next_col == 1
    # a slot frees at a step boundary: request 3's second column joins
    assert srv._admit(waiting, items, 16, 1, 0) == [(3, 1)]
    assert waiting == [1, 4]
    # a request partly admitted by worker 0 is not split to worker 1
    items[1].worker = 0
    items[1].next_col = 1
    waiting = [1, 4]
    assert srv._admit(waiting, items, 32, 8, 1) == [(4, c) for c in range(8)]
    assert srv._pick_key([1], items, 1) is None


def test_pick_key_takes_the_oldest_request_and_reserves_its_bytes():
    srv = _server(1000)
    srv.bytes_est = {16: 600, 32: 300}
    items = _items([(32, 1), (16, 1)])
    assert srv._pick_key([0, 1], items, 0) == (32, [])
    assert srv.pending == {(0, 32): 300}
    # the reservation counts: 300 reserved + 600 fits 1000, a second 300 would not
    assert srv._pick_key([1], items, 1) == (16, [])
    assert srv._cached_bytes() == 900
    assert srv._pick_key([0], items, 1) is None


def test_admission_evicts_idle_contexts_outside_the_lock_and_waits_when_full():
    srv = _server(1000)
    srv.bytes_est = {16: 600, 32: 600}
    c16 = _cached(srv, 0, 16, 600)
    items = _items([(32, 1)])
    # an idle context is handed back for eviction (closed by the caller)
    key, victims = srv._pick_key([0], items, 1)
    assert key == 32 and victims == [c16] and 16 not in srv.ctx[0] and not c16[0].closed
    # a busy context is not evicted: the request waits
    srv = _server(1000)
    srv.bytes_est = {16: 600, 32: 600}
    _cached(srv, 0, 16, 600)
    srv.busy_keys[0].add(16)
    assert srv._pick_key([0], _items([(32, 1)]), 1) is None and 16 in srv.ctx[0]


def test_a_context_larger_than_the_budget_is_an_error():
    srv = _server(1000)
    srv.bytes_est = {16: 5000}
    with pytest.raises(MemoryError):
        srv._pick_key([0], _items([(16, 1)]), 0)


def test_starving_counts_keys_the_worker_does_not_serve():
    srv = _server(1 << 40)
    items = _items([(16, 1), (32, 1)], t=0.0)
    assert not srv._starving([1], items, {16}, now=0.01)
    assert srv._starving([1], items, {16}, now=0.03)
    assert not srv._starving([1], items, {16, 32}, now=0.03)


def test_pick_key_skips_keys_the_worker_serves():
    srv = _server(1 << 40)
    items = _items([(16, 1), (32, 1)])
    _cached(srv, 0, 16, 10)
    assert srv._pick_key([0, 1], items, 0) == (16, [])
    assert srv._pick_key([0, 1], items, 0, held={16}) == (32, [])


@pytest.mark.gpu
def test_served_trace_matches_solo_bitwise():
    import torch
    from paper_1605_01522_amd import NField
    grids = (16, 24, 32)
    trace = nfgen.request_trace(24, rate=400.0, grids=grids, seed=3)
    for r in trace:
        r["key"] = r["grid"]
    systems = {g: nfgen.tsi2d(nel=g) for g in grids}
    srv = serve.Server(lambda g: systems[g], SERVE_SPEC, SERVE_OPTS, workers=3, max_cols=8)
    items = srv.run(trace, lambda req: nfgen.request_rhs(req, systems[req["grid"]].n), time_scale=1.0)
    summ = serve.summarize(items)
    print(summ, flush=True)
    assert summ["all_converged"]
    assert max(it.batch_cols for it in items) > 1        # some requests shared a launch
    assert any(it.joined_running for it in items)       # some joined a running batch
    solo = {g: NField(systems[g].fields, systems[g].blocks, SERVE_SPEC, hier_fp32=1, **SERVE_OPTS) for g in grids}
    for it in items:
        g = it.req["grid"]
        B = torch.tensor(nfgen.request_rhs(it.req, systems[g].n), device="cuda")
        x, st = solo[g].gmres_solve(B, flexible=1, rtol=1e-8)
        assert np.array_equal(x.cpu().numpy(), it.x), it.req["id"]
        A = systems[g].assembled()
        for k in range(it.req["nrhs"]):
            assert np.linalg.norm(B[k].cpu().numpy() - A @ it.x[k]) < 1e-8 * np.linalg.norm(B[k].cpu().numpy())
    srv.close()


def test_estimate_before_a_keys_first_build():
    """A key not built yet is estimated from the largest footprint per
    unknown seen so far (plus 10 %), or 4,000 bytes per unknown before any
    build; a built key uses its own measured footprint."""
    srv = _server(1 << 40)
    assert srv._estimate(16, 1600) == 4000 * 1600
    srv.bytes_est[16] = 3_200_000            # as recorded by a build of key 16 (n = 1,600)
    srv.bytes_per_dof = 3_200_000 / 1600
    assert srv._estimate(16, 1600) == 3_200_000
    assert srv._estimate(32, 3200) == int(1.1 * 2000.0 * 3200)
