"""Continuous-batching request loop over the nfield C ABI.

Requests (a block system identified by a key, e.g. its grid size, plus one
or more right-hand sides) arrive over time.  The loop keeps the solver
contexts (device-resident hierarchies) cached by key, admits work while the
device memory budget allows it, and runs batches on several HIP streams at
once:

* a worker that becomes free takes the oldest waiting request and joins to
  it every other waiting request of the same key while the batch has at most
  `max_cols` right-hand sides (columns of one multi-column solve);
* each worker owns one stream and one context per key (contexts are not
  shared between streams); a context is built on first use and kept;
* admission: a context is built only if the bytes of every cached context
  plus its estimate fit the budget, evicting least-recently used idle
  contexts first; otherwise the request waits;
* all numerical work is the library's (flexible GMRES, FP64 outer, FP32
  hierarchy by default); columns of a batch never mix, so a request's
  solution is the same alone and in any batch.
"""
import threading
import time
from collections import OrderedDict

import numpy as np

from .nfield import NField


class Served:
    __slots__ = ("req", "x", "stats", "t_arrive", "t_admit", "t_start", "t_done", "batch_cols", "worker")

    def __init__(self, req):
        self.req = req
        self.x = None
        self.stats = None
        self.t_arrive = self.t_admit = self.t_start = self.t_done = None
        self.batch_cols = 0
        self.worker = -1


class Server:
    def __init__(self, system_for_key, spec, opts=None, workers=4, max_cols=8, hier_fp32=True,
                 budget_bytes=64 << 30, restart=50, rtol=1e-8, keep_solutions=True, factory=NField):
        import torch
        self.torch = torch
        self.factory = factory                  # builds a solver context (NField)
        self.system_for_key = system_for_key    # key -> nfgen.BlockSystem-like (fields, blocks)
        self.spec = spec
        self.opts = dict(opts or {})
        self.hier_fp32 = hier_fp32
        self.workers = workers
        self.max_cols = max_cols
        self.budget = budget_bytes
        self.restart = restart
        self.rtol = rtol
        self.keep = keep_solutions
        self.streams = [torch.cuda.Stream() for _ in range(workers)]   # default priority
        self.ctx = [OrderedDict() for _ in range(workers)]              # key -> NField (LRU)
        self.busy_keys = [set() for _ in range(workers)]
        self.bytes_est = {}                                             # key -> footprint seen
        self.lock = threading.Condition()
        self.systems = {}

    # ---------------- memory accounting (callers hold self.lock)
    def _cached_bytes(self):
        return sum(c.footprint_bytes() for w in self.ctx for c in w.values())

    def _estimate(self, key, n):
        return self.bytes_est.get(key, 4000 * n)

    def _make_room(self, need, w):
        """Evict idle contexts (least recently used first) until `need` bytes fit."""
        while self._cached_bytes() + need > self.budget:
            victim = None
            for wi in range(self.workers):
                for k in self.ctx[wi]:
                    if k not in self.busy_keys[wi]:
                        victim = (wi, k)
                        break
                if victim:
                    break
            if victim is None:
                return False
            c = self.ctx[victim[0]].pop(victim[1])
            c.close()
        return True

    def _system(self, key):
        if key not in self.systems:
            self.systems[key] = self.system_for_key(key)
        return self.systems[key]

    # ---------------- the loop
    def run(self, requests, rhs_for, time_scale=1.0):
        """Serve `requests` (dicts with id, arrival_s, key, nrhs); rhs_for(req)
        returns its (nrhs, n) right-hand sides.  Arrivals are replayed in
        real time (scaled by time_scale; 0 = everything arrives at once).
        Returns the list of Served records in request order."""
        torch = self.torch
        items = [Served(r) for r in requests]
        order = sorted(range(len(items)), key=lambda i: items[i].req["arrival_s"])
        waiting = []              # arrived, not started (indices, arrival order)
        state = dict(next=0, done=0, error=None)
        t0 = time.perf_counter()

        def arrived_until(now):
            while state["next"] < len(order):
                i = order[state["next"]]
                if items[i].req["arrival_s"] * time_scale > now:
                    break
                items[i].t_arrive = items[i].req["arrival_s"] * time_scale
                items[i].t_admit = now
                waiting.append(i)
                state["next"] += 1

        def worker(w):
            stream = self.streams[w]
            while True:
                with self.lock:
                    while True:
                        if state["error"] is not None or state["done"] == len(items):
                            return
                        arrived_until(time.perf_counter() - t0)
                        batch = self._take_batch(waiting, items, w)
                        if batch:
                            break
                        # sleep until the next arrival or a state change
                        nxt = None
                        if state["next"] < len(order):
                            nxt = items[order[state["next"]]].req["arrival_s"] * time_scale - \
                                (time.perf_counter() - t0)
                        self.lock.wait(timeout=max(1e-4, min(nxt, 0.05)) if nxt is not None else 0.05)
                    key = items[batch[0]].req["key"]
                    self.busy_keys[w].add(key)
                try:
                    self._solve_batch(w, stream, key, batch, items, rhs_for, t0)
                except Exception as e:      # surfaced to the caller
                    with self.lock:
                        state["error"] = e
                        self.lock.notify_all()
                    return
                with self.lock:
                    self.busy_keys[w].discard(key)
                    state["done"] += len(batch)
                    self.lock.notify_all()

        threads = [threading.Thread(target=worker, args=(w,), daemon=True) for w in range(self.workers)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise state["error"]
        return items

    def _take_batch(self, waiting, items, w):
        """Oldest waiting request plus same-key requests up to max_cols columns,
        if its context exists or can be admitted under the memory budget."""
        for pos, i in enumerate(waiting):
            key = items[i].req["key"]
            if key not in self.ctx[w]:
                sysk = self._system(key)
                if not self._make_room(self._estimate(key, sysk.n), w):
                    continue        # does not fit now; try a request of another key
            cols = items[i].req["nrhs"]
            batch = [i]
            for j in waiting[pos + 1:]:
                if items[j].req["key"] == key and cols + items[j].req["nrhs"] <= self.max_cols:
                    batch.append(j)
                    cols += items[j].req["nrhs"]
            for j in batch:
                waiting.remove(j)
            return batch
        return None

    def _context(self, w, key, stream):
        with self.lock:
            c = self.ctx[w].get(key)
            s = self._system(key)
        if c is None:
            c = self.factory(s.fields, s.blocks, self.spec, stream=stream,
                             hier_fp32=1 if self.hier_fp32 else 0, **self.opts)
            with self.lock:
                self.ctx[w][key] = c
                self.bytes_est[key] = c.footprint_bytes()
        with self.lock:
            self.ctx[w].move_to_end(key)
        return c

    def _solve_batch(self, w, stream, key, batch, items, rhs_for, t0):
        torch = self.torch
        ctx = self._context(w, key, stream)
        n = ctx.n
        rhs = np.concatenate([rhs_for(items[i].req) for i in batch], axis=0)
        t_start = time.perf_counter() - t0
        with torch.cuda.stream(stream):
            B = torch.from_numpy(rhs).pin_memory().to("cuda", non_blocking=True)
            X = torch.zeros_like(B)
            _, stats = ctx.gmres_solve(B, X, stream=stream, restart=self.restart, maxit=1000,
                                       flexible=1 if self.hier_fp32 else 0, rtol=self.rtol)
            Xh = X.cpu() if self.keep else None
        stream.synchronize()
        t_done = time.perf_counter() - t0
        c = 0
        for i in batch:
            k = items[i].req["nrhs"]
            it = items[i]
            it.t_start, it.t_done, it.batch_cols, it.worker = t_start, t_done, rhs.shape[0], w
            it.stats = stats[c:c + k]
            it.x = Xh[c:c + k].numpy() if self.keep else None
            c += k

    def close(self):
        for w in self.ctx:
            for c in w.values():
                c.close()
            w.clear()


def summarize(items):
    """Throughput and latency of a served trace."""
    lat = np.array([it.t_done - it.t_arrive for it in items])
    t_end = max(it.t_done for it in items)
    t_begin = min(it.t_arrive for it in items)
    cols = sum(it.req["nrhs"] for it in items)
    iters = [s["iters"] for it in items for s in it.stats]
    ok = all(s["status"] == 0 for it in items for s in it.stats)
    return dict(requests=len(items), rhs_solves=cols, wall_s=t_end - t_begin,
                solves_per_s=cols / (t_end - t_begin), requests_per_s=len(items) / (t_end - t_begin),
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_batch_cols=float(np.mean([it.batch_cols for it in items])),
                mean_iters=float(np.mean(iters)), all_converged=ok)
