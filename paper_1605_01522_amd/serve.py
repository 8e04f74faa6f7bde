"""Iteration-level continuous batching over the nfield C ABI.

Requests (a block system identified by a key, e.g. its grid size, plus one
or more right-hand sides) arrive over time.  The loop keeps solver contexts
(device-resident hierarchies) cached by key and serves them on several HIP
streams at once:

* each worker owns one stream and, per key, one context with a slot batch
  (nfield_batch_*) of `max_cols` GMRES columns; a context is built on first
  use and kept (contexts are not shared between streams);
* a worker serves up to `max_keys` keys at once (lanes, one by default:
  stepping two batches in turn on one stream lengthens both steps; on the
  512-request TSI trace one lane per stream gave the higher capacity and
  the lower latency), stepping their
  batches in turn; a worker with a free lane takes the key of the oldest
  waiting request it does not serve yet; at every Arnoldi step boundary it
  fills each lane's free slots with waiting columns of that key in arrival
  order, so a request joins a batch that is already running, and a column
  that has finished leaves it and frees its slot for the next boundary;
* once a request of a key it does not serve has waited `max_wait_s`, a
  worker whose lanes are all taken stops admitting, so that a lane drains
  and frees (one busy key cannot hold a worker for ever);
* admission by device memory: a context is built only if the bytes of every
  cached or reserved context plus its estimate fit the budget, evicting
  least-recently used idle contexts first (closed outside the lock);
  otherwise the request waits; a context larger than the whole budget is an
  error;
* all numerical work is the library's (flexible GMRES, FP64 outer, FP32
  hierarchy by default); columns never mix, so a request's solution is the
  same bits as a solve of it alone.
"""
import threading
import time
from collections import OrderedDict

import numpy as np

from .nfield import Batch, NField


class Served:
    __slots__ = ("req", "x", "stats", "t_arrive", "t_admit", "t_start", "t_done", "batch_cols", "worker",
                 "joined_running", "next_col", "cols_done", "B", "X")

    def __init__(self, req):
        self.req = req
        self.x = None
        self.stats = None
        self.t_arrive = self.t_admit = self.t_start = self.t_done = None
        self.batch_cols = 0          # most columns that shared a step with this request's columns
        self.worker = -1
        self.joined_running = False  # its first column joined a batch that was already running
        self.next_col = 0            # columns admitted so far
        self.cols_done = 0
        self.B = self.X = None       # device right-hand sides and solutions while served


class Server:
    def __init__(self, system_for_key, spec, opts=None, workers=4, max_cols=8, hier_fp32=True,
                 budget_bytes=64 << 30, restart=50, rtol=1e-8, maxit=1000, keep_solutions=True, max_wait_s=0.02,
                 max_keys=1, factory=NField, batch_factory=Batch):
        import torch
        self.torch = torch
        self.factory = factory                  # builds a solver context (NField)
        self.batch_factory = batch_factory      # builds its slot batch (Batch)
        self.system_for_key = system_for_key    # key -> nfgen.BlockSystem-like (fields, blocks)
        self.spec = spec
        self.opts = dict(opts or {})
        self.opts.setdefault("max_rhs", max_cols)
        self.hier_fp32 = hier_fp32
        self.workers = workers
        self.max_cols = max_cols
        self.budget = budget_bytes
        self.restart = restart
        self.rtol = rtol
        self.maxit = maxit
        self.keep = keep_solutions
        self.max_wait_s = max_wait_s
        self.max_keys = max_keys                # keys (lanes) one worker serves at once
        self.streams = [torch.cuda.Stream() for _ in range(workers)]   # default priority
        self._init_state()

    def _init_state(self):
        self.ctx = [OrderedDict() for _ in range(self.workers)]        # key -> (NField, Batch), LRU order
        self.busy_keys = [set() for _ in range(self.workers)]
        self.bytes_est = {}                                             # key -> footprint seen
        self.bytes_per_dof = 0.0                                        # largest footprint / n seen
        self.pending = {}                                               # (worker, key) -> bytes reserved
        self.last_use = {}                                              # (worker, key) -> use tick
        self.tick = 0
        self.lock = threading.Condition()
        self.systems = {}

    # ---------------- memory accounting (callers hold self.lock)
    def _cached_bytes(self):
        return sum(c[0].footprint_bytes() for w in self.ctx for c in w.values()) + sum(self.pending.values())

    def _estimate(self, key, n):
        """A key's footprint as measured when it was last built; before that,
        n times the largest footprint per unknown of the contexts built so far
        (plus 10 %), or 4,000 bytes per unknown before any was built."""
        if key in self.bytes_est:
            return self.bytes_est[key]
        if self.bytes_per_dof > 0.0:
            return int(1.1 * self.bytes_per_dof * n)
        return 4000 * n

    def _make_room(self, need):
        """Idle contexts to evict, least recently used first, so that `need`
        more bytes fit the budget: removed from the cache and returned (the
        caller closes them outside the lock); None if even evicting every
        idle context would not make room (nothing is evicted then)."""
        total = self._cached_bytes()
        if total + need <= self.budget:
            return []
        idle = [(wi, k) for wi in range(self.workers) for k in self.ctx[wi]
                if k not in self.busy_keys[wi] and (wi, k) not in self.pending]
        idle.sort(key=lambda v: self.last_use.get(v, 0))
        free = sum(self.ctx[wi][k][0].footprint_bytes() for wi, k in idle)
        if total - free + need > self.budget:
            if need > self.budget:
                raise MemoryError(f"a context of about {need} bytes exceeds the budget of {self.budget} bytes")
            return None
        victims = []
        for wi, k in idle:
            if total + need <= self.budget:
                break
            c = self.ctx[wi].pop(k)
            self.last_use.pop((wi, k), None)
            total -= c[0].footprint_bytes()
            victims.append(c)
        return victims

    def _system(self, key):
        if key not in self.systems:
            self.systems[key] = self.system_for_key(key)
        return self.systems[key]

    # ---------------- scheduling (callers hold self.lock)
    def _pick_key(self, waiting, items, w, held=()):
        """Key of the oldest waiting request (of a key not in `held`, the keys
        this worker serves already) whose context this worker holds or can
        admit under the budget: (key, contexts to close) or None.  A context
        to build has its bytes reserved until it is stored."""
        for i in waiting:
            if items[i].worker not in (-1, w):
                continue            # partly admitted by another worker, which serves the rest
            key = items[i].req["key"]
            if key in held:
                continue
            if key in self.ctx[w]:
                return key, []
            if (w, key) in self.pending:
                continue
            need = self._estimate(key, self._system(key).n)
            victims = self._make_room(need)
            if victims is None:
                continue            # does not fit now; try a request of another key
            self.pending[(w, key)] = need
            return key, victims
        return None

    def _admit(self, waiting, items, key, nfree, w):
        """Up to nfree waiting columns of `key` for worker w, in arrival order:
        a list of (item index, column).  A request is served by one worker
        (the one that admits its first column); requests whose every column
        is admitted leave `waiting`."""
        out = []
        for i in list(waiting):
            if len(out) >= nfree:
                break
            it = items[i]
            if it.req["key"] != key or it.worker not in (-1, w):
                continue
            it.worker = w
            while it.next_col < it.req["nrhs"] and len(out) < nfree:
                out.append((i, it.next_col))
                it.next_col += 1
            if it.next_col == it.req["nrhs"]:
                waiting.remove(i)
        return out

    def _starving(self, waiting, items, keys, now):
        """A request of a key not in `keys` has waited max_wait_s or longer."""
        for i in waiting:
            it = items[i]
            if it.req["key"] not in keys and now - it.t_arrive >= self.max_wait_s:
                return True
        return False

    def _context(self, w, key, stream):
        """This worker's (context, batch) for key, built on first use."""
        with self.lock:
            c = self.ctx[w].get(key)
            s = self._system(key)
        if c is None:
            try:
                ctx = self.factory(s.fields, s.blocks, self.spec, stream=stream,
                                   hier_fp32=1 if self.hier_fp32 else 0, **self.opts)
                bat = self.batch_factory(ctx, self.max_cols, restart=self.restart, maxit=self.maxit,
                                         flexible=1 if self.hier_fp32 else 0, rtol=self.rtol)
            finally:
                with self.lock:
                    self.pending.pop((w, key), None)
            c = (ctx, bat)
            with self.lock:
                self.ctx[w][key] = c
                self.bytes_est[key] = ctx.footprint_bytes()
                self.bytes_per_dof = max(self.bytes_per_dof, self.bytes_est[key] / max(s.n, 1))
        with self.lock:
            self.ctx[w].move_to_end(key)
            self.tick += 1
            self.last_use[(w, key)] = self.tick
        return c

    # ---------------- the loop
    def run(self, requests, rhs_for, time_scale=1.0):
        """Serve `requests` (dicts with id, arrival_s, key, nrhs); rhs_for(req)
        returns its (nrhs, n) right-hand sides.  Arrivals are replayed in
        real time (scaled by time_scale; 0 = everything arrives at once).
        Returns the list of Served records in request order."""
        torch = self.torch
        items = [Served(r) for r in requests]
        order = sorted(range(len(items)), key=lambda i: items[i].req["arrival_s"])
        waiting = []              # arrived requests with columns not yet admitted (arrival order)
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

        def next_arrival(now):
            if state["next"] < len(order):
                return items[order[state["next"]]].req["arrival_s"] * time_scale - now
            return None

        def worker(w):
            stream = self.streams[w]
            lanes = OrderedDict()       # key -> dict(slot_of: slot -> (item, column), active: count)

            def release(key):
                self.busy_keys[w].discard(key)
                del lanes[key]

            while True:
                victims = []
                with self.lock:
                    while True:
                        if state["error"] is not None or state["done"] == len(items):
                            for key in list(lanes):
                                release(key)
                            return
                        now = time.perf_counter() - t0
                        arrived_until(now)
                        if len(lanes) < self.max_keys:
                            pick = self._pick_key(waiting, items, w, held=lanes)
                            if pick is not None:
                                key, v = pick
                                victims += v
                                self.busy_keys[w].add(key)
                                lanes[key] = dict(slot_of=[None] * self.max_cols, active=0)
                                continue
                        if lanes:
                            break
                        nxt = next_arrival(now)
                        self.lock.wait(timeout=max(1e-4, min(nxt, 0.05)) if nxt is not None else 0.05)
                    # a full worker stops admitting while a request of a key it
                    # does not hold starves, so that one of its lanes drains
                    hold = len(lanes) >= self.max_keys and self._starving(waiting, items, lanes, now)
                    adm = {}
                    for key, ln in lanes.items():
                        if ln["active"] == 0 or not hold:
                            adm[key] = self._admit(waiting, items, key, self.max_cols - ln["active"], w)
                try:
                    for v in victims:
                        v[1].close()
                        v[0].close()
                    finished = []
                    for key in list(lanes):
                        ln = lanes[key]
                        _, bat = self._context(w, key, stream)
                        if adm.get(key):
                            self._submit(adm[key], items, bat, ln["slot_of"], ln["active"], stream, rhs_for, t0)
                            ln["active"] += len(adm[key])
                        if ln["active"] == 0:
                            with self.lock:
                                release(key)
                                self.lock.notify_all()
                            continue
                        finished += self._step(items, bat, ln, stream)
                    for i in finished:
                        it = items[i]
                        with torch.cuda.stream(stream):
                            it.x = it.X.cpu().numpy() if self.keep else None
                        stream.synchronize()
                        it.t_done = time.perf_counter() - t0
                        it.B = it.X = None
                    if finished:
                        with self.lock:
                            state["done"] += len(finished)
                            self.lock.notify_all()
                except Exception as e:      # surfaced to the caller
                    with self.lock:
                        state["error"] = e
                        self.lock.notify_all()
                    return

        threads = [threading.Thread(target=worker, args=(w,), daemon=True) for w in range(self.workers)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise state["error"]
        return items

    def _step(self, items, bat, ln, stream):
        """One step of a lane's batch; takes the finished columns and returns
        the requests whose every column has finished."""
        slot_of = ln["slot_of"]
        active = ln["active"]
        done, _ = bat.step(stream)
        for q in range(self.max_cols):
            if slot_of[q] is not None:
                it = items[slot_of[q][0]]
                it.batch_cols = max(it.batch_cols, active)
        finished = []
        for q in done:
            i, col = slot_of[q]
            it = items[i]
            it.stats[col] = bat.take(q, it.X[col], stream=stream)
            slot_of[q] = None
            ln["active"] -= 1
            it.cols_done += 1
            if it.cols_done == it.req["nrhs"]:
                finished.append(i)
        return finished

    def _submit(self, adm, items, bat, slot_of, active, stream, rhs_for, t0):
        """Put admitted columns into free slots (uploading a request's
        right-hand sides at its first admitted column)."""
        torch = self.torch
        now = time.perf_counter() - t0
        free = [q for q in range(self.max_cols) if slot_of[q] is None]
        for (i, col), q in zip(adm, free):
            it = items[i]
            if it.B is None:
                rhs = np.ascontiguousarray(rhs_for(it.req), dtype=np.float64)
                with torch.cuda.stream(stream):
                    it.B = torch.from_numpy(rhs).pin_memory().to("cuda", non_blocking=True)
                    it.X = torch.zeros_like(it.B)
                it.stats = [None] * it.req["nrhs"]
                it.t_start = now
                it.joined_running = active > 0
            bat.submit(q, it.B[col], stream=stream)
            slot_of[q] = (i, col)

    def close(self):
        for w in self.ctx:
            for ctx, bat in w.values():
                bat.close()
                ctx.close()
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
                joined_running_frac=float(np.mean([it.joined_running for it in items])),
                mean_iters=float(np.mean(iters)), all_converged=ok)
