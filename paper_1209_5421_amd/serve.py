"""Serving loop over the quadamg C ABI: continuous batching of solve requests on one GPU.

Requests (a mesh id, its system, a right-hand side) arrive over time. Several dispatcher threads run concurrently;
each repeatedly takes every pending request it may admit and solves them with one ``amg_solve_batch`` call, so
requests that arrive while earlier batches are on the device are dispatched as soon as a dispatcher is free and their
work overlaps on the GPU:

- hierarchies stay resident in a cache keyed by mesh id (a repeat right-hand side skips setup);
- a new hierarchy is admitted only if ``amg_estimate_bytes`` fits in the HBM budget, after evicting idle cached
  hierarchies least recently used first; otherwise the request waits until memory frees up;
- a hierarchy serves one batch at a time (one workspace per hierarchy), so a request whose mesh is in flight waits;
- inside ``amg_solve_batch`` small systems run as one persistent workgroup each in a shared launch and larger ones on
  their own host thread and stream.

Each system's result is independent of the mix it was served in (bit-identical to serving it alone).
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np

from . import amg


@dataclasses.dataclass
class Request:
    rid: int
    mesh_id: object
    problem: object          # meshgen.Problem-like: coords, row_ptr, col, val, box, n, nnz
    rhs: np.ndarray
    arrival: float = 0.0     # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    x: np.ndarray
    iters: int
    relres: float
    status: int
    arrival: float
    start: float
    end: float
    cache_hit: bool
    batch_size: int

    @property
    def latency(self):
        return self.end - self.arrival


class _Entry:
    __slots__ = ("h", "bytes", "busy", "last_use")

    def __init__(self, h, nbytes):
        self.h, self.bytes, self.busy, self.last_use = h, nbytes, False, time.perf_counter()


class Scheduler:
    """Host-side admission and batching state (no device work; callers hold ``lock``).

    ``estimate(problem)`` gives the bytes a new hierarchy will take; ``close(h)`` frees one. A batch holds at most one
    request per mesh and never a mesh already in flight; a new mesh is admitted only if its estimate fits in
    ``mem_budget`` after evicting idle cached hierarchies least recently used first. Requests that cannot start keep
    their arrival order.
    """

    def __init__(self, mem_budget, max_batch, estimate, close):
        self.mem_budget, self.max_batch = int(mem_budget), int(max_batch)
        self.estimate, self.close_h = estimate, close
        self.cache: "collections.OrderedDict[object, _Entry]" = collections.OrderedDict()
        self.mem_used = 0
        self.pending: "collections.deque[Request]" = collections.deque()
        self.lock = threading.Condition()
        self.setups = 0
        self.evictions = 0
        self.retired = []  # evicted hierarchies not yet closed

    def drain_retired(self):
        """Evicted hierarchies, to be closed outside the lock (closing one waits for its stream)."""
        out, self.retired = self.retired, []
        return out

    def _admit_new(self, req) -> bool:
        need = self.estimate(req.problem)
        if need > self.mem_budget:
            raise MemoryError(f"request {req.rid}: hierarchy needs {need} bytes, budget is {self.mem_budget}")
        while self.mem_used + need > self.mem_budget:
            victim = next((k for k, e in self.cache.items() if not e.busy), None)
            if victim is None:
                return False
            e = self.cache.pop(victim)
            self.mem_used -= e.bytes
            if e.h is not None:
                self.retired.append(e.h)  # closed by the caller once it has released the lock
            self.evictions += 1
        self.mem_used += need
        self.cache[req.mesh_id] = _Entry(None, need)  # reserved; set up by the dispatcher that took it
        self.cache[req.mesh_id].busy = True
        return True

    def take_batch(self):
        """[(request, cache_hit)] that may start now; removes them from ``pending``."""
        batch, seen, keep = [], set(), collections.deque()
        while self.pending:
            r = self.pending.popleft()
            if len(batch) >= self.max_batch or r.mesh_id in seen:
                keep.append(r)
                continue
            e = self.cache.get(r.mesh_id)
            if e is not None:
                if e.busy:
                    keep.append(r)
                    continue
                e.busy = True
                self.cache.move_to_end(r.mesh_id)
                batch.append((r, True))
            else:
                if not self._admit_new(r):
                    keep.append(r)
                    continue
                batch.append((r, False))
            seen.add(r.mesh_id)
        self.pending = keep
        return batch

    def installed(self, mesh_id, h, nbytes):
        """A reserved hierarchy was set up: record it and its measured size."""
        e = self.cache[mesh_id]
        self.mem_used += nbytes - e.bytes
        e.h, e.bytes = h, nbytes
        self.setups += 1

    def failed(self, mesh_id):
        """A reserved hierarchy could not be set up: drop the reservation."""
        e = self.cache.pop(mesh_id)
        self.mem_used -= e.bytes
        if e.h is not None:
            self.retired.append(e.h)

    def done(self, mesh_id):
        e = self.cache[mesh_id]
        e.busy = False
        e.last_use = time.perf_counter()

    def release(self, mesh_ids):
        """End of a batch, whatever happened in it: a mesh whose hierarchy never came up loses its reservation, an
        installed one becomes idle; meshes already dropped are skipped."""
        for m in mesh_ids:
            e = self.cache.get(m)
            if e is None:
                continue
            if e.h is None:
                self.failed(m)
            else:
                self.done(m)

    def close_all(self):
        for h in self.drain_retired():
            self.close_h(h)
        for e in self.cache.values():
            if e.h is not None:
                self.close_h(e.h)
        self.cache.clear()
        self.mem_used = 0


# share of the HBM budget the library's freed-block cache may hold; hierarchies are admitted against the rest, so the
# cache never takes memory the admitted hierarchies or the caller's own tensors were counted on
CACHE_SHARE = 0.1


class Server:
    def __init__(self, device="cuda:0", mem_budget=64 << 30, dispatchers=4, max_batch=128, precision=1, tol=1e-8,
                 keep_x=True, streams_per_dispatcher=4, batch=1):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        cache_limit = int(CACHE_SHARE * mem_budget)
        amg.cache_control(self.device.index or 0, cache_limit)
        mem_budget = int(mem_budget) - cache_limit
        self.dispatchers = int(dispatchers)
        self.streams_per_dispatcher = int(streams_per_dispatcher)
        self.batch = int(batch)
        self.precision = int(precision)
        self.tol = float(tol)
        self.keep_x = keep_x
        amg.load()
        self.sched = Scheduler(mem_budget, max_batch,
                               lambda p: amg.estimate_bytes(p.n, p.nnz, precision=self.precision),
                               lambda h: h.close())
        self.lock = self.sched.lock
        self.results: dict = {}
        self.batches = []

    # -- dispatch ---------------------------------------------------------------------------------------------
    def _dispatcher(self, t0, stop, errors):
        torch, sched = self.torch, self.sched
        # one stream per batch slot (torch hands out streams of its pool round-robin): a batch's large systems, each
        # on its hierarchy's stream, overlap with one another and with the launch that runs its small systems
        streams = [torch.cuda.Stream(device=self.device) for _ in range(self.streams_per_dispatcher)]
        with torch.cuda.device(self.device):
            while True:
                with self.lock:
                    while not sched.pending and not stop["done"]:
                        self.lock.wait(0.05)
                    if not sched.pending and stop["done"]:
                        return
                    try:
                        batch = sched.take_batch()
                    except MemoryError as exc:
                        errors.append(exc)
                        sched.pending.clear()
                        self.lock.notify_all()
                        return
                    if not batch:
                        self.lock.wait(0.002)
                        continue
                    retired = sched.drain_retired()
                for h in retired:
                    h.close()
                self._run_batch(batch, streams, t0, errors)

    def _run_batch(self, batch, streams, t0, errors):
        """Set up the batch's new hierarchies and solve it with one amg_solve_batch call. Whatever happens, every
        request of the batch gets a result and every mesh it holds is released (done, or dropped if its hierarchy
        never came up), so no mesh stays marked in flight."""
        torch, sched = self.torch, self.sched
        t_start = time.perf_counter() - t0
        results = {}
        try:
            hs, bs, xs, ok = [], [], [], []
            for j, (r, hit) in enumerate(batch):
                st = streams[j % len(streams)]
                with torch.cuda.stream(st):
                    if not hit:
                        p = r.problem
                        try:
                            h = amg.Hierarchy(_dev(torch, p.coords, torch.float64, self.device),
                                              _dev(torch, p.row_ptr, torch.int64, self.device),
                                              _dev(torch, p.col, torch.int32, self.device),
                                              _dev(torch, p.val, torch.float64, self.device), box=p.box,
                                              precision=self.precision, stream=st, batch=self.batch)
                        except amg.AMGError as exc:
                            results[r.rid] = Result(r.rid, None, 0, float("nan"), exc.code, r.arrival, t_start,
                                                    time.perf_counter() - t0, False, len(batch))
                            continue
                        with self.lock:
                            sched.installed(r.mesh_id, h, h.bytes())
                    else:
                        h = sched.cache[r.mesh_id].h
                        h.set_stream(st)
                        h.set_precision(self.precision)
                    b = _dev(torch, r.rhs, torch.float64, self.device)
                    hs.append(h)
                    ok.append((r, hit))
                    bs.append(b)
                    xs.append(torch.empty_like(b))
            for st in streams:
                st.synchronize()
            code, infos = amg.solve_batch(hs, bs, xs, [self.tol] * len(hs)) if hs else (0, [])
            xs_host = [x.cpu().numpy() for x in xs] if self.keep_x else [None] * len(xs)
            t_end = time.perf_counter() - t0
            for (r, hit), x, info in zip(ok, xs_host, infos):
                results[r.rid] = Result(r.rid, x, info["iters"], info["relres"], info["status"], r.arrival, t_start,
                                        t_end, hit, len(batch))
        except Exception as exc:  # recorded; serve() raises the first one after the stream ends
            errors.append(exc)
        finally:
            t_end = time.perf_counter() - t0
            with self.lock:
                for r, hit in batch:
                    self.results[r.rid] = results.get(r.rid) or Result(r.rid, None, 0, float("nan"), amg.DEVICE,
                                                                       r.arrival, t_start, t_end, hit, len(batch))
                sched.release([r.mesh_id for r, _ in batch])
                self.batches.append(len(batch))
                self.lock.notify_all()

    def serve(self, requests):
        """Serve requests at their arrival times (seconds from now); returns {rid: Result}."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        stop, errors = {"done": False}, []
        t0 = time.perf_counter()
        threads = [threading.Thread(target=self._dispatcher, args=(t0, stop, errors), daemon=True)
                   for _ in range(self.dispatchers)]
        for t in threads:
            t.start()
        for r in reqs:
            delay = r.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            with self.lock:
                self.sched.pending.append(r)
                self.lock.notify_all()
        with self.lock:
            stop["done"] = True
            self.lock.notify_all()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
        return self.results

    @property
    def setups(self):
        return self.sched.setups

    @property
    def evictions(self):
        return self.sched.evictions

    def close(self):
        self.sched.close_all()


def _dev(torch, a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def summarize(results, wall=None, dof=None):
    """Latency percentiles and throughput of a served stream; ``dof`` maps request id -> unknowns (adds DOF/s)."""
    lat = np.array([r.latency for r in results.values()]) * 1e3
    ends = max(r.end for r in results.values())
    starts = min(r.arrival for r in results.values())
    span = wall if wall else (ends - starts)
    out = {
        "requests": len(results),
        "makespan_s": span,
        "solves_per_s": len(results) / span,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "cache_hit_rate": float(np.mean([r.cache_hit for r in results.values()])),
        "mean_batch": float(np.mean([r.batch_size for r in results.values()])),
        "all_converged": bool(all(r.status == 0 and r.relres <= 1e-8 * (1 + 1e-9) for r in results.values())),
    }
    if dof is not None:
        out["dof_per_s"] = sum(dof[r] for r in results) / span
    return out
