"""Continuous-batching server for angle-averaged metasurface evaluations.

Requests (a geometry, an objective, a light distribution, optionally a
gradient) arrive over time.  Their work has two parts:

* factorisation of a geometry not in the cache: one host thread drives each
  factorisation engine (``rcp_engine_*``, ``engines`` of them, each on its own
  stream), in which every geometry in flight (up to 8 per engine,
  ``factor_slots`` in all) advances one pass per round of shared kernel
  launches, whatever its grid size; a geometry admitted while others are in
  progress joins the emptier engine at its next round (continuous batching at
  the level of the factorisation passes); two engines overlap one's chains of
  pivot inversions with the other's tile updates;
* evaluation on factors that are ready: up to ``eval_slots`` evaluations run
  at once, each on its own HIP stream, beside the engine's stream.  Plain
  requests for the same geometry that are waiting go together (up to
  ``group``): one multi-right-hand-side reciprocal sweep serves them all.

A fresh geometry is admitted when the device memory its factors need
(``rcp_factor_bytes``) fits in the budget (idle cached factors are evicted,
least recently used first); a grouped evaluation's workspace counts against
the same budget.  Requests that need new factors are admitted first come,
first served; a request whose geometry is cached but busy (being factored or
evaluated) waits on it without holding back others.  Factors stay cached
(keyed by geometry) until their memory is needed.  Latency is measured from
arrival to result.

The device work goes through an executor: ``GpuExecutor`` calls librecip;
``FakeExecutor`` models costs and memory on the host so the scheduling logic
can be tested without a GPU.  ``serve_sequential`` is the baseline: one
request at a time, factored alone and evaluated, nothing cached.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass
from typing import Any, Callable, Dict, List, Optional

from workloads import Problem, Request


def geometry_key(p: Problem):
    """Everything the factors depend on (grid, PML, permittivity description)."""
    return (p.nx, p.ny, p.npml, p.h, p.wavelength, p.pml_R, p.pml_m, p.eps_bg, p.eps_sub,
            p.eps_pillar, p.sub_rows, p.pillar_row0, p.pillar_rows, p.pillar_centers, p.widths)


@dataclass
class Result:
    rid: int
    F: Optional[float] = None
    grad_widths: Any = None
    error: Optional[str] = None
    arrival: float = 0.0
    start: float = 0.0
    done: float = 0.0
    cache_hit: bool = False
    slot: int = -1
    group: int = 1               # requests served by the same evaluation call

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class ServerError(RuntimeError):
    pass


class Arena:
    """First-fit placement of byte ranges in [0, size), 256-byte aligned, free
    neighbours merged.  The server's memory ledger: every factor set and group
    workspace gets an explicit offset in one device region, so an admitted
    request never meets an allocator that cannot place its buffer."""

    ALIGN = 256

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]     # sorted (offset, length)
        self.used = 0

    @classmethod
    def aligned(cls, n: int) -> int:
        return (int(n) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def place(self, n: int) -> Optional[int]:
        n = self.aligned(n)
        for k, (o, length) in enumerate(self.free):
            if length >= n:
                if length == n:
                    del self.free[k]
                else:
                    self.free[k] = (o + n, length - n)
                self.used += n
                return o
        return None

    def release(self, off: int, n: int) -> None:
        n = self.aligned(n)
        self.used -= n
        k = 0
        while k < len(self.free) and self.free[k][0] < off:
            k += 1
        self.free.insert(k, (off, n))
        if k + 1 < len(self.free) and off + n == self.free[k + 1][0]:
            self.free[k] = (off, n + self.free[k + 1][1])
            del self.free[k + 1]
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == off:
            self.free[k - 1] = (self.free[k - 1][0], self.free[k - 1][1] + self.free[k][1])
            del self.free[k]


# ---------------------------------------------------------------------------
# executors


class GpuExecutor:
    """librecip on one GPU: the factorisation engine on its own stream, the
    evaluations on the streams of the evaluation slots."""

    def __init__(self, precision: int = 0, device: str = "cuda", ahead: int = 2):
        import torch
        import paper_2207_10701_amd as rcp
        self.torch = torch
        self.rcp = rcp
        self.precision = precision
        self.device = torch.device(device)
        self.ahead = ahead           # engine steps enqueued ahead of the GPU

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def factor_bytes(self, p: Problem) -> int:
        return self.rcp.factor_bytes(p, self.precision)

    def open_arena(self, nbytes: int) -> None:
        """The device region the server's ledger places buffers in."""
        self.arena = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)

    def close_arena(self) -> None:
        self.arena = None

    def _view(self, off: int, nbytes: int):
        return self.arena[off:off + nbytes]

    # -- factorisation engine (one host thread) --
    def new_engine(self):
        eng = self.rcp.FactorEngine(self.precision, stream=self.new_stream())
        eng._marks = []
        return eng

    def engine_add(self, eng, p: Problem, off: int):
        torch, rcp = self.torch, self.rcp
        with torch.cuda.stream(eng.stream):
            widths = torch.tensor(p.widths, dtype=torch.float64, device=self.device)
            eps = rcp.eps_from_widths(p, widths, device=self.device, stream=eng.stream)
            return eng.add(p, eps, buffer=self._view(off, self.factor_bytes(p)))

    def engine_step(self, eng, rounds: int):
        """Enqueue up to `rounds` rounds; keep at most `ahead` steps queued on the
        GPU, so that a geometry admitted now joins within a few rounds."""
        done = eng.step(rounds)
        ev = self.torch.cuda.Event()
        ev.record(eng.stream)
        eng._marks.append(ev)
        if len(eng._marks) > self.ahead:
            eng._marks.pop(0).synchronize()
        return [(fac, None if err is None else str(err)) for fac, err in done]

    def engine_size(self, eng) -> int:
        return len(eng)

    def engine_close(self, eng) -> None:
        eng.close()

    # -- evaluations --
    def factor(self, p: Problem, stream) -> Any:
        """One geometry factored alone (the sequential baseline)."""
        torch, rcp = self.torch, self.rcp
        with torch.cuda.stream(stream):
            widths = torch.tensor(p.widths, dtype=torch.float64, device=self.device)
            eps = rcp.eps_from_widths(p, widths, device=self.device, stream=stream)
            fac = rcp.Factors(p, eps, self.precision, stream=stream)
        return fac

    def evaluate(self, fac, p: Problem, adjoint: bool, stream):
        torch, rcp = self.torch, self.rcp
        with torch.cuda.stream(stream):
            if adjoint:
                F, g = rcp.adjoint_grad(fac, p, stream=stream)
                gw = rcp.width_grad(p, g, stream=stream)
            else:
                F = rcp.reciprocal_average(fac, p, stream=stream)
                gw = None
            stream.synchronize()
        return F.item(), (gw.cpu().numpy() if gw is not None else None)

    def many_work_bytes(self, fac, count: int) -> int:
        """Device workspace of a grouped evaluation of count requests."""
        return int(self.rcp.lib.rcp_reciprocal_many_work_bytes(fac.handle, count))

    def evaluate_many(self, fac, problems, stream, work_off: int):
        """Plain evaluations of several requests on one factor set (workspace
        at work_off in the arena)."""
        torch, rcp = self.torch, self.rcp
        need = self.many_work_bytes(fac, len(problems))
        with torch.cuda.stream(stream):
            F = rcp.reciprocal_average_many(fac, problems, stream=stream,
                                            work=self._view(work_off, need))
            stream.synchronize()
        return [float(v) for v in F.cpu().numpy()]

    def release(self, fac) -> None:
        fac.release()
        fac.buf = None


class _FakeEngine:
    def __init__(self):
        self.items: List[list] = []      # [fac, rounds left]


class FakeExecutor:
    """Host-only stand-in: modelled durations and memory, deterministic results.
    The engine model: a geometry needs factor_rounds(p) rounds; a round costs
    round_seconds whatever shares it (the kernels' launches are shared)."""

    def __init__(self, factor_seconds: Callable[[Problem], float] = lambda p: 0.002,
                 eval_seconds: float = 0.0005, bytes_per_cell: int = 1000,
                 fail_on: Optional[Callable[[Problem], bool]] = None,
                 round_seconds: float = 0.0005):
        self.factor_seconds = factor_seconds
        self.eval_seconds = eval_seconds
        self.bytes_per_cell = bytes_per_cell
        self.fail_on = fail_on
        self.round_seconds = round_seconds
        self.factor_calls = 0
        self.group_sizes: List[int] = []
        self.round_sizes: List[int] = []     # geometries sharing each engine round
        self.live = 0
        self.peak_live = 0
        self.lock = threading.Lock()

    def new_stream(self):
        return None

    def factor_bytes(self, p: Problem) -> int:
        return p.nx * p.ny * self.bytes_per_cell

    def _made(self, p: Problem):
        with self.lock:
            self.factor_calls += 1
            self.live += self.factor_bytes(p)
            self.peak_live = max(self.peak_live, self.live)
        return {"p": p, "bytes": self.factor_bytes(p)}

    def open_arena(self, nbytes: int) -> None:
        pass

    def close_arena(self) -> None:
        pass

    def new_engine(self):
        return _FakeEngine()

    def engine_add(self, eng, p: Problem, off: int):
        fac = self._made(p)
        rounds = max(1, int(round(self.factor_seconds(p) / self.round_seconds)))
        eng.items.append([fac, rounds])
        return fac

    def engine_step(self, eng, rounds: int):
        done = []
        for _ in range(rounds):
            if not eng.items or done:
                break
            time.sleep(self.round_seconds)
            self.round_sizes.append(len(eng.items))
            for it in eng.items:
                it[1] -= 1
            for it in [it for it in eng.items if it[1] <= 0]:
                eng.items.remove(it)
                p = it[0]["p"]
                bad = self.fail_on is not None and self.fail_on(p)
                done.append((it[0], f"RCP_ESINGULAR: modelled failure for {p.name}" if bad else None))
        return done

    def engine_size(self, eng) -> int:
        return len(eng.items)

    def engine_close(self, eng) -> None:
        for it in eng.items:
            self.release(it[0])
        eng.items.clear()

    def factor(self, p: Problem, stream):
        if self.fail_on is not None and self.fail_on(p):
            raise ServerError(f"RCP_ESINGULAR: modelled failure for {p.name}")
        time.sleep(self.factor_seconds(p))
        return self._made(p)

    def evaluate(self, fac, p: Problem, adjoint: bool, stream):
        time.sleep(self.eval_seconds)
        F = float(sum(p.widths)) + p.c + p.th1 + p.th2
        return F, ([1.0] * len(p.widths) if adjoint else None)

    def many_work_bytes(self, fac, count: int) -> int:
        p = fac["p"]
        return 32 * count * p.nx * p.ny

    def evaluate_many(self, fac, problems, stream, work_off: int):
        time.sleep(self.eval_seconds)   # one sweep for all of them
        with self.lock:
            self.group_sizes.append(len(problems))
        return [float(sum(p.widths)) + p.c + p.th1 + p.th2 for p in problems]

    def release(self, fac) -> None:
        with self.lock:
            self.live -= fac["bytes"]


# ---------------------------------------------------------------------------
# server


@dataclass
class _Entry:
    key: Any
    p: Problem
    nbytes: int
    off: int = 0                 # place in the arena
    fac: Any = None
    users: int = 0               # evaluations running on it (one at a time)
    last_used: float = 0.0
    ready: bool = False          # factors complete
    error: Optional[str] = None  # factorisation failed


class Server:
    """Continuous batching: the factorisation engine plus evaluation slots,
    memory-ledger admission and a factor cache."""

    def __init__(self, executor, factor_slots: int = 8, eval_slots: int = 4,
                 hbm_budget: int = 200 << 30, cache: bool = True, group: int = 16,
                 rounds_per_step: int = 4, order: str = "arrival", engines: int = 1):
        if not 1 <= engines <= 4:
            raise ValueError("engines must be 1 to 4")
        if not 1 <= factor_slots <= 8 * engines:
            raise ValueError("factor_slots must be 1 to 8 per engine")
        if eval_slots < 1:
            raise ValueError("eval_slots must be >= 1")
        if not 1 <= group <= 64:
            raise ValueError("group must be 1 to 64")
        if order not in ("arrival", "largest_first"):
            raise ValueError("order is 'arrival' or 'largest_first'")
        self.order = order
        self.ex = executor
        self.factor_slots = factor_slots
        self.group = group
        self.budget = int(hbm_budget)
        self.cache_enabled = cache
        self.rounds = rounds_per_step
        self.cache: Dict[Any, _Entry] = {}
        self.arena = Arena(self.budget)     # factor sets and group workspaces
        executor.open_arena(self.budget)
        self.cv = threading.Condition()
        self.free_slots = list(range(eval_slots))
        self.streams = [executor.new_stream() for _ in range(eval_slots)]
        self.results: Dict[int, Result] = {}
        # per engine: admitted, not yet in it; and its geometries (queued or in it)
        self.to_factor: List[List[_Entry]] = [[] for _ in range(engines)]
        self.assigned = [0] * engines
        self.factoring = 0                  # entries in the engine or queued for it
        self.peak_bytes = 0
        self.max_inflight = 0               # evaluations at once
        self.max_factoring = 0              # geometries in the engines at once
        self.engine_time = 0.0              # wall time with geometries in an engine (summed over engines)
        self.engine_geom_time = 0.0         # ... times the geometries in it
        self.inflight = 0
        # each engine on its own stream, driven by a thread of its own: while one
        # waits on its chains of pivot inversions the other's tile updates run
        self.engines = [executor.new_engine() for _ in range(engines)]
        self._stop = False
        self._ft = [threading.Thread(target=self._factor_loop, args=(i,), daemon=True)
                    for i in range(engines)]
        for th in self._ft:
            th.start()

    # -- memory ledger ----------------------------------------------------------------
    @property
    def used(self) -> int:
        return self.arena.used

    def _place(self, need: int) -> Optional[int]:
        """An offset for need bytes, evicting idle cached factors (least recently
        used first) until they fit; None if they cannot."""
        while True:
            off = self.arena.place(need)
            if off is not None:
                self.peak_bytes = max(self.peak_bytes, self.arena.used)
                return off
            # idle: ready, not in use, and no waiting request needs it
            idle = [e for e in self.cache.values()
                    if e.users == 0 and e.ready and not self._wanted(e)]
            if not idle:
                return None
            self._drop(min(idle, key=lambda e: e.last_used))

    def _drop(self, entry: _Entry) -> None:
        if self.cache.get(entry.key) is entry:
            del self.cache[entry.key]
        if entry.fac is not None:
            self.ex.release(entry.fac)
            entry.fac = None
        self.arena.release(entry.off, entry.nbytes)

    # -- the engine's thread ----------------------------------------------------------------
    def _factor_loop(self, i: int):
        made: Dict[int, _Entry] = {}
        eng, queue = self.engines[i], self.to_factor[i]
        while True:
            with self.cv:
                while not self._stop and not queue and self.ex.engine_size(eng) == 0:
                    self.cv.wait()
                if self._stop and not queue and self.ex.engine_size(eng) == 0:
                    return
                adds = queue[:]
                queue.clear()
            for entry in adds:
                try:
                    fac = self.ex.engine_add(eng, entry.p, entry.off)
                    made[id(fac)] = entry
                    entry.fac = fac
                except Exception as e:     # bad geometry: fail its requests only
                    with self.cv:
                        entry.error = str(e)
                        entry.ready = True
                        self.factoring -= 1
                        self.assigned[i] -= 1
                        self.cv.notify_all()
            with self.cv:
                self.max_factoring = max(self.max_factoring,
                                         sum(self.ex.engine_size(e) for e in self.engines))
            if self.ex.engine_size(eng) == 0:
                continue
            n_in = self.ex.engine_size(eng)
            t_step = time.perf_counter()
            done = self.ex.engine_step(eng, self.rounds)
            dt = time.perf_counter() - t_step
            with self.cv:
                self.engine_time += dt
                self.engine_geom_time += dt * n_in
            if done:
                with self.cv:
                    for fac, err in done:
                        entry = made.pop(id(fac))
                        entry.ready = True
                        entry.error = err
                        self.factoring -= 1
                        self.assigned[i] -= 1
                    self.cv.notify_all()

    # -- evaluations (run on a slot's thread) -----------------------------------------------
    def _evaluate(self, reqs: List[Request], slot: int, entry: _Entry, t0: float,
                  arrivals: List[float], work: tuple, fresh: List[bool]):
        start = time.perf_counter() - t0
        err, Fs, grads = None, [None] * len(reqs), [None] * len(reqs)
        try:
            if len(reqs) > 1:
                Fs = self.ex.evaluate_many(entry.fac, [r.problem for r in reqs], self.streams[slot],
                                           work[0])
            else:
                Fs[0], grads[0] = self.ex.evaluate(entry.fac, reqs[0].problem, reqs[0].adjoint,
                                                   self.streams[slot])
        except Exception as e:
            err = str(e)
        done = time.perf_counter() - t0
        with self.cv:
            if work[1]:
                self.arena.release(*work)
            entry.users -= 1
            entry.last_used = done
            if not self.cache_enabled and not self._wanted(entry):
                self._drop(entry)
            self.free_slots.append(slot)
            self.free_slots.sort()
            self.inflight -= 1
            for r, a, F, g, fr in zip(reqs, arrivals, Fs, grads, fresh):
                self.results[r.rid] = Result(rid=r.rid, F=F, grad_widths=g, error=err, arrival=a,
                                             start=start, done=done, cache_hit=not fr, slot=slot,
                                             group=len(reqs))
            self.cv.notify_all()

    def _wanted(self, entry: _Entry) -> bool:
        return any(geometry_key(r.problem) == entry.key for r in getattr(self, "_waiting", ()))

    # -- driver -----------------------------------------------------------------------------
    def run(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Serve a request stream.  realtime: replay the arrival times; otherwise
        every request is present at the start (latency counted from there)."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        threads = []
        self._waiting: List[Request] = []
        self._fresh: Dict[int, bool] = {}     # rid -> the request brought its geometry in
        nxt = 0
        with self.cv:
            while nxt < len(pending) or self._waiting:
                now = time.perf_counter() - t0
                while nxt < len(pending) and (not realtime or pending[nxt].arrival <= now):
                    self._waiting.append(pending[nxt])
                    nxt += 1
                if self._schedule(t0, realtime, threads):
                    continue
                timeout = 0.05
                if realtime and nxt < len(pending):
                    timeout = min(timeout, max(pending[nxt].arrival - now, 0.0))
                self.cv.wait(timeout=timeout)
        for th in threads:
            th.join()
        return [self.results[r.rid] for r in requests]

    def _admit_fresh(self, t0: float, realtime: bool) -> bool:
        """Start the factorisation of geometries not in the cache, in the order of
        the policy (arrival, or the largest factorisation first), while engine
        slots and memory last: the first that does not fit holds back the rest
        (no request overtakes one it is ordered behind)."""
        fresh, seen = [], set()
        for r in self._waiting:
            key = geometry_key(r.problem)
            if key not in self.cache and key not in seen:
                seen.add(key)
                fresh.append(r)
        if self.order == "largest_first":
            fresh.sort(key=lambda r: -float(r.problem.ny) ** 3 * r.problem.nx)
        changed = False
        for req in fresh:
            if self.factoring >= self.factor_slots:
                break
            need = self.ex.factor_bytes(req.problem)
            if Arena.aligned(need) > self.budget:
                self.results[req.rid] = Result(
                    rid=req.rid, error=f"request {req.rid} needs {need} bytes, budget "
                                       f"{self.budget}",
                    arrival=req.arrival if realtime else 0.0, done=time.perf_counter() - t0)
                self._waiting = [r for r in self._waiting if r.rid != req.rid]
                changed = True
                continue
            off = self._place(need)
            if off is None:
                break
            key = geometry_key(req.problem)
            entry = _Entry(key, req.problem, need, off)
            self.cache[key] = entry
            i = min(range(len(self.engines)), key=lambda j: self.assigned[j])   # the emptier engine
            self.to_factor[i].append(entry)
            self.assigned[i] += 1
            self.factoring += 1
            self._fresh[req.rid] = True
            changed = True
            self.cv.notify_all()
        return changed

    def _schedule(self, t0: float, realtime: bool, threads: list) -> bool:
        """Admit fresh geometries and start evaluations that can start; True if
        anything changed."""
        changed = False
        i = 0
        while i < len(self._waiting):
            req = self._waiting[i]
            key = geometry_key(req.problem)
            entry = self.cache.get(key)
            if entry is None or not entry.ready or entry.users > 0 or not self.free_slots:
                i += 1           # parked on its geometry
                continue
            if entry.error is not None:     # its factorisation failed
                for r in [r for r in self._waiting if geometry_key(r.problem) == key]:
                    self.results[r.rid] = Result(rid=r.rid, error=entry.error,
                                                 arrival=r.arrival if realtime else 0.0,
                                                 done=time.perf_counter() - t0)
                self._waiting = [r for r in self._waiting if geometry_key(r.problem) != key]
                self._drop(entry)
                changed = True
                i = 0
                continue
            # evaluate: this request and, for plain ones, others waiting on it
            # (the entry is in use from here: eviction must not take it)
            entry.users += 1
            group, work = [req], (0, 0)
            if not req.adjoint and self.group > 1:
                for other in self._waiting[i + 1:]:
                    if len(group) >= self.group:
                        break
                    if not other.adjoint and geometry_key(other.problem) == key:
                        group.append(other)
                while len(group) > 1:       # the grouped call's workspace: same ledger
                    wb = self.ex.many_work_bytes(entry.fac, len(group))
                    woff = self._place(wb)
                    if woff is not None:
                        work = (woff, wb)
                        break
                    group.pop()
            taken = {r.rid for r in group}
            self._waiting = [r for r in self._waiting if r.rid not in taken]
            slot = self.free_slots.pop(0)
            self.inflight += 1
            self.max_inflight = max(self.max_inflight, self.inflight)
            arrivals = [r.arrival if realtime else 0.0 for r in group]
            fresh = [self._fresh.pop(r.rid, False) for r in group]
            th = threading.Thread(target=self._evaluate,
                                  args=(group, slot, entry, t0, arrivals, work, fresh), daemon=True)
            th.start()
            threads.append(th)
            changed = True
        changed |= self._admit_fresh(t0, realtime)
        return changed

    def engine_occupancy(self) -> float:
        """Time-weighted mean number of geometries in an engine while it ran."""
        return self.engine_geom_time / self.engine_time if self.engine_time > 0 else 0.0

    def close(self):
        with self.cv:
            self._stop = True
            self.cv.notify_all()
        for th in self._ft:
            th.join()
        with self.cv:
            for e in list(self.cache.values()):
                if e.fac is not None:
                    self.ex.release(e.fac)
            self.cache.clear()
            self.arena = Arena(self.budget)
        for eng in self.engines:
            self.ex.engine_close(eng)
        self.ex.close_arena()


def serve_sequential(executor, requests: List[Request], realtime: bool = True) -> List[Result]:
    """Baseline: one request at a time in arrival order, its geometry factored
    alone, evaluated, and released (plain FP64 when the executor's precision
    is)."""
    stream = executor.new_stream()
    t0 = time.perf_counter()
    out = []
    for req in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        if realtime:
            wait = req.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        res = Result(rid=req.rid, arrival=req.arrival if realtime else 0.0, slot=0)
        res.start = time.perf_counter() - t0
        fac = None
        try:
            fac = executor.factor(req.problem, stream)
            res.F, res.grad_widths = executor.evaluate(fac, req.problem, req.adjoint, stream)
        except Exception as e:
            res.error = str(e)
        if fac is not None:
            executor.release(fac)
        res.done = time.perf_counter() - t0
        out.append(res)
    by = {r.rid: r for r in out}
    return [by[r.rid] for r in requests]


def summarize(results: List[Result]) -> dict:
    ok = [r for r in results if r.error is None]
    lat = sorted(r.latency for r in ok)

    def pct(q):
        if not lat:
            return float("nan")
        k = (len(lat) - 1) * q
        lo, hi = math.floor(k), math.ceil(k)
        return lat[lo] + (lat[hi] - lat[lo]) * (k - lo)

    makespan = max((r.done for r in results), default=0.0) - min((r.arrival for r in results),
                                                                  default=0.0)
    return {"requests": len(results), "ok": len(ok), "failed": len(results) - len(ok),
            "cache_hits": sum(r.cache_hit for r in ok),
            "p50_ms": 1e3 * pct(0.50), "p99_ms": 1e3 * pct(0.99),
            "makespan_s": makespan, "evals_per_s": len(ok) / makespan if makespan > 0 else 0.0}
