"""Continuous-batching serving loop over several partitioned systems.

Requests (a system key and 1..64 right-hand sides) arrive over time.  Each
resident system owns one solver context on its own HIP stream and a worker
thread; its right-hand sides occupy slots of the context's resident CG state
(dd_batch_*): arriving requests are admitted between CG iterations as slots
free up, finished ones are retired, so requests for the same system share
every sweep over the factors and coupling blocks while they overlap, and
different systems run concurrently on their own streams.  A system becomes
resident only if its device footprint fits the HBM budget; idle systems are
evicted least-recently-used first (their factors are then recomputed on the
next request).  Stalled mixed-precision refinements are finished with FP64
factors on a second context, whose footprint is counted with the system's.

All device work is done by the C ABI (paper_2306_00094_amd); this module only
schedules it.  Latency = completion - arrival (host monotonic clock).
"""
from __future__ import annotations

import collections
import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import (DD_FP64, DD_MIXED, DD_SLOT_DONE, DD_SLOT_FALLBACK, DD_SLOT_FREE, Solver,
               dd_batch_admit, dd_batch_begin, dd_batch_end, dd_batch_retire, dd_batch_step,
               dd_default_opts, dd_footprint)

MAX_SLOTS = 64


@dataclass
class Request:
    key: object
    b: np.ndarray                 # n_dof x nrhs (host)
    arrival: float = 0.0          # seconds since the run started
    rid: int = 0
    done: float = float("nan")
    u: np.ndarray | None = None
    info: list = field(default_factory=list)
    fallback: bool = False

    @property
    def nrhs(self) -> int:
        return self.b.shape[1]

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _System:
    """One resident system: solver context, worker thread and request queue."""

    def __init__(self, server, key, dd):
        import torch
        self.server, self.key, self.dd = server, key, dd
        self.torch = torch
        self.stream = torch.cuda.Stream()           # default priority
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.last_used = time.monotonic()
        self.running = {}                            # rid -> (request, slots, device b)
        self.slots_free = list(range(MAX_SLOTS))
        self.stop = False
        self.solver = None
        self.fallback_solver = None
        self.thread = threading.Thread(target=self._work, daemon=True)

    # ---- worker --------------------------------------------------------
    def _open(self):
        with self.torch.cuda.stream(self.stream):
            self.solver = Solver(self.dd, max_nrhs=MAX_SLOTS, stream=self.stream)
            self.solver.factor(self.server.prec)
            dd_batch_begin(self.solver.ctx, self.server.prec, self.server.opts)

    def _admit(self):
        torch = self.torch
        while True:
            with self.cv:
                if not self.queue or len(self.slots_free) < self.queue[0].nrhs:
                    return
                req = self.queue.popleft()
            slots = sorted(self.slots_free)[:req.nrhs]
            for s in slots:
                self.slots_free.remove(s)
            with torch.cuda.stream(self.stream):
                bt = torch.from_numpy(np.ascontiguousarray(req.b.T)).to("cuda", non_blocking=False)
            dd_batch_admit(self.solver.ctx, slots, bt, int(req.b.shape[0]))
            self.running[req.rid] = (req, slots, bt)

    def _retire(self, states):
        torch = self.torch
        for rid, (req, slots, bt) in list(self.running.items()):
            st = [states[s] for s in slots]
            if any(x not in (DD_SLOT_DONE, DD_SLOT_FALLBACK) for x in st):
                continue
            with torch.cuda.stream(self.stream):
                u = torch.empty_like(bt)
            info = dd_batch_retire(self.solver.ctx, slots, u, int(req.b.shape[0]))
            uh = u.cpu().numpy().T.copy()
            if any(x == DD_SLOT_FALLBACK for x in st):
                uh, info = self._fallback(req, st, uh, info)
            req.u, req.info = uh, info
            req.done = self.server.now()
            self.slots_free.extend(slots)
            del self.running[rid]
            self.server._complete(req)

    def _fallback(self, req, st, uh, info):
        torch = self.torch
        if self.fallback_solver is None:
            with torch.cuda.stream(self.stream):
                self.fallback_solver = Solver(self.dd, max_nrhs=MAX_SLOTS, stream=self.stream)
                self.fallback_solver.factor(DD_FP64)
        cols = [j for j, x in enumerate(st) if x == DD_SLOT_FALLBACK]
        with torch.cuda.stream(self.stream):
            b = torch.from_numpy(np.ascontiguousarray(req.b[:, cols].T)).to("cuda")
            opts = dd_default_opts(tol=self.server.opts.tol, max_it=self.server.opts.max_it)
            r = self.fallback_solver.solve(b, prec=DD_FP64, opts=opts, raise_on_noconv=False)
        ub = r.u.cpu().numpy().T
        for k, j in enumerate(cols):
            uh[:, j] = ub[:, k]
            info[j] = dict(r.info[k], used_fallback=1)
        req.fallback = True
        return uh, info

    def _work(self):
        try:
            self._open()
            while True:
                with self.cv:
                    while not self.queue and not self.running and not self.stop:
                        self.cv.wait(timeout=0.05)
                    if self.stop and not self.queue and not self.running:
                        break
                self._admit()
                if self.running:
                    states = dd_batch_step(self.solver.ctx, self.server.iters_per_step, MAX_SLOTS)
                    self._retire(states)
                self.last_used = time.monotonic()
        except BaseException as e:            # surface worker errors to the caller
            self.server._error(e)
        finally:
            self._close()

    def _close(self):
        if self.solver is not None:
            try:
                dd_batch_end(self.solver.ctx)
            except Exception:
                pass
            self.solver.close()
            self.solver = None
        if self.fallback_solver is not None:
            self.fallback_solver.close()
            self.fallback_solver = None
        self.server._released(self)

    def idle(self) -> bool:
        with self.cv:
            return not self.queue and not self.running

    def submit(self, req):
        with self.cv:
            self.queue.append(req)
            self.cv.notify()

    def shutdown(self):
        with self.cv:
            self.stop = True
            self.cv.notify()


class Server:
    """Schedules requests over systems with an HBM budget (bytes, None = no limit)."""

    def __init__(self, systems: dict, prec: int = DD_MIXED, opts=None,
                 hbm_budget: int | None = None, iters_per_step: int = 4):
        self.systems = systems                      # key -> DDProblem
        self.prec = prec
        # mixed precision: the FP32-data products gather FP32 vector copies
        # (the serving batches are wide; FP64 solves ignore the option)
        self.opts = opts if opts is not None else dd_default_opts(tol=1e-9, gather32=1)
        self.hbm_budget = hbm_budget
        self.iters_per_step = iters_per_step
        # device bytes held by a resident system: its context, and for mixed
        # precision with the FP64 fallback also the second (FP64) context that
        # finishes stalled requests, reserved up front so that admission by
        # footprint never under-counts
        fb = prec == DD_MIXED and self.opts.fp64_fallback != 0
        self.footprint = {k: dd_footprint(dd, prec, MAX_SLOTS)
                          + (dd_footprint(dd, DD_FP64, MAX_SLOTS) if fb else 0)
                          for k, dd in systems.items()}
        self.resident = {}                          # key -> _System
        self.closing = set()                        # evicted systems still holding memory
        self.lock = threading.Lock()
        self.done = []
        self.done_cv = threading.Condition()
        self.errors = []
        self.evictions = 0
        self.t0 = time.monotonic()

    def now(self) -> float:
        return time.monotonic() - self.t0

    def _error(self, e):
        with self.done_cv:
            self.errors.append(e)
            self.done_cv.notify_all()

    def _complete(self, req):
        with self.done_cv:
            self.done.append(req)
            self.done_cv.notify_all()

    def _released(self, sysobj):
        with self.lock:
            if self.resident.get(sysobj.key) is sysobj:
                del self.resident[sysobj.key]
            self.closing.discard(sysobj)
        with self.done_cv:
            self.done_cv.notify_all()

    def _resident_bytes(self):
        return (sum(self.footprint[k] for k in self.resident)
                + sum(self.footprint[s.key] for s in self.closing))

    def _make_resident(self, key):
        """Return the resident system for key, evicting idle ones if needed
        (None if it does not fit yet)."""
        with self.lock:
            s = self.resident.get(key)
            if s is not None:
                return s
            need = self.footprint[key]
            if self.hbm_budget is not None:
                if need > self.hbm_budget:
                    raise MemoryError(f"system {key} needs {need} bytes > budget {self.hbm_budget}")
                if self._resident_bytes() + need > self.hbm_budget:
                    # evict idle systems least-recently-used first; their memory
                    # counts until their worker has released it
                    idle = sorted((x for x in self.resident.values() if x.idle() and not x.stop),
                                  key=lambda x: x.last_used)
                    free = self.hbm_budget - self._resident_bytes()
                    for victim in idle:
                        if free >= need:
                            break
                        victim.shutdown()
                        del self.resident[victim.key]
                        self.closing.add(victim)
                        self.evictions += 1
                        free += self.footprint[victim.key]
                    return None
            s = _System(self, key, self.systems[key])
            self.resident[key] = s
            s.thread.start()
            return s

    def run(self, requests, timeout: float = 600.0, keep_resident: bool = False):
        """Release the requests at their arrival times (seconds from start) and
        wait for all completions.  Returns the completed requests of this run.
        With keep_resident the systems (factors, Krylov state) stay on the
        device for the next run; otherwise they are released at the end."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(reqs)
        waiting = collections.deque()
        with self.done_cv:
            self.done = []
        self.t0 = time.monotonic()
        deadline = self.t0 + timeout
        while pending or waiting or len(self.done) < len(reqs):
            if self.errors:
                raise self.errors[0]
            if time.monotonic() > deadline:
                raise TimeoutError(f"serving run exceeded {timeout} s")
            t = self.now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            for _ in range(len(waiting)):
                r = waiting.popleft()
                s = self._make_resident(r.key)
                if s is None:
                    waiting.append(r)
                else:
                    s.submit(r)
            with self.done_cv:
                nxt = pending[0].arrival - self.now() if pending else 0.005
                self.done_cv.wait(timeout=max(0.0005, min(nxt, 0.005)))
        if not keep_resident:
            self.shutdown()
        return self.done

    def shutdown(self):
        with self.lock:
            systems = list(self.resident.values())
        for s in systems:
            s.shutdown()
        for s in systems:
            s.thread.join(timeout=60)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """n arrival times of a Poisson process with the given rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def summarize(done, wall: float | None = None) -> dict:
    lat = np.array([r.latency for r in done])
    cols = sum(r.nrhs for r in done)
    first = min(r.arrival for r in done)
    last = max(r.done for r in done)
    span = wall if wall is not None else (last - first)
    return dict(requests=len(done), solves=cols, seconds=span, solves_per_s=cols / span,
                p50_ms=1e3 * float(np.percentile(lat, 50)), p99_ms=1e3 * float(np.percentile(lat, 99)),
                mean_ms=1e3 * float(lat.mean()),
                fallbacks=sum(1 for r in done if r.fallback))
