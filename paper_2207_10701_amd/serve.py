"""Continuous-batching server for angle-averaged metasurface evaluations.

Requests (a geometry, an objective, a light distribution, optionally a
gradient) arrive over time.  The server keeps up to ``slots`` requests in
flight, each on its own HIP stream driven by its own host thread, so their
kernels overlap on the device.  A request is admitted when a slot is free and
the device memory its factors need (``rcp_factor_bytes``) fits in the budget;
factors of finished requests stay cached (keyed by geometry) until their
memory is needed, so repeated geometries skip the factorisation.  When a
request starts on cached factors, the requests for the same geometry that
have already arrived (plain evaluations, up to ``group``) go with it: one
multi-right-hand-side reciprocal sweep serves all of them.  Admission is
first come, first served among requests that need memory for new factors; a request
whose cached geometry is busy waits on it without holding back others.
Latency is measured from arrival to result.

The device work goes through an executor: ``GpuExecutor`` calls librecip;
``FakeExecutor`` models costs and memory on the host so the scheduling logic
can be tested without a GPU.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass, field
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


# ---------------------------------------------------------------------------
# executors


class GpuExecutor:
    """Runs a request on one HIP stream through librecip."""

    def __init__(self, precision: int = 0, device: str = "cuda"):
        import torch
        import paper_2207_10701_amd as rcp
        self.torch = torch
        self.rcp = rcp
        self.precision = precision
        self.device = torch.device(device)

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def factor_bytes(self, p: Problem) -> int:
        return self.rcp.factor_bytes(p, self.precision)

    def factor(self, p: Problem, stream) -> Any:
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

    def evaluate_many(self, fac, problems, stream):
        """Plain evaluations of several requests on one factor set."""
        torch, rcp = self.torch, self.rcp
        with torch.cuda.stream(stream):
            F = rcp.reciprocal_average_many(fac, problems, stream=stream)
            stream.synchronize()
        return [float(v) for v in F.cpu().numpy()]

    def release(self, fac) -> None:
        fac.release()
        fac.buf = None


class FakeExecutor:
    """Host-only stand-in: modelled durations and memory, deterministic results."""

    def __init__(self, factor_seconds: Callable[[Problem], float] = lambda p: 0.002,
                 eval_seconds: float = 0.0005, bytes_per_cell: int = 1000,
                 fail_on: Optional[Callable[[Problem], bool]] = None):
        self.factor_seconds = factor_seconds
        self.eval_seconds = eval_seconds
        self.bytes_per_cell = bytes_per_cell
        self.fail_on = fail_on
        self.factor_calls = 0
        self.group_sizes: List[int] = []
        self.live = 0
        self.peak_live = 0
        self.lock = threading.Lock()

    def new_stream(self):
        return None

    def factor_bytes(self, p: Problem) -> int:
        return p.nx * p.ny * self.bytes_per_cell

    def factor(self, p: Problem, stream):
        if self.fail_on is not None and self.fail_on(p):
            raise ServerError(f"RCP_ESINGULAR: modelled failure for {p.name}")
        time.sleep(self.factor_seconds(p))
        with self.lock:
            self.factor_calls += 1
            self.live += self.factor_bytes(p)
            self.peak_live = max(self.peak_live, self.live)
        return {"p": p, "bytes": self.factor_bytes(p)}

    def evaluate(self, fac, p: Problem, adjoint: bool, stream):
        time.sleep(self.eval_seconds)
        F = float(sum(p.widths)) + p.c + p.th1 + p.th2
        return F, ([1.0] * len(p.widths) if adjoint else None)

    def many_work_bytes(self, fac, count: int) -> int:
        p = fac["p"]
        return 32 * count * p.nx * p.ny

    def evaluate_many(self, fac, problems, stream):
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
    fac: Any
    nbytes: int
    users: int = 0
    last_used: float = 0.0
    ready: bool = False          # False while the first request is still factoring


class Server:
    """Continuous batching with memory-ledger admission and a factor cache."""

    def __init__(self, executor, slots: int = 4, hbm_budget: int = 200 << 30,
                 cache: bool = True, group: int = 16):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        if not 1 <= group <= 64:
            raise ValueError("group must be 1 to 64")
        self.group = group
        self.ex = executor
        self.nslots = slots
        self.budget = int(hbm_budget)
        self.cache_enabled = cache
        self.cache: Dict[Any, _Entry] = {}
        self.used = 0                       # bytes of factors held (cached, in use, being made)
        self.cv = threading.Condition()
        self.free_slots = list(range(slots))
        self.streams = [executor.new_stream() for _ in range(slots)]
        self.results: Dict[int, Result] = {}
        self.peak_bytes = 0
        self.max_inflight = 0
        self.inflight = 0

    # -- memory ledger ----------------------------------------------------------------
    def _evict_for(self, need: int) -> bool:
        """Free idle cached factors (least recently used first) until need fits."""
        while self.used + need > self.budget:
            idle = [e for e in self.cache.values() if e.users == 0 and e.ready]
            if not idle:
                return False
            victim = min(idle, key=lambda e: e.last_used)
            del self.cache[victim.key]
            self.used -= victim.nbytes
            self.ex.release(victim.fac)
        return True

    _PARK = object()      # the request waits on its cached entry; later ones may start
    _BLOCK = object()     # no memory for new factors: later fresh requests wait too

    def _try_admit(self, req: Request, fresh_blocked: bool):
        """(slot, entry) if req can start now, else _PARK or _BLOCK."""
        key = geometry_key(req.problem)
        entry = self.cache.get(key)
        if entry is not None:
            # factors hold per-call work vectors: one user at a time, and a
            # geometry being factored is waited for rather than factored twice
            if entry.users > 0 or not entry.ready:
                return self._PARK
            entry.users += 1
            return self.free_slots.pop(0), entry
        if fresh_blocked:      # first come, first served among requests needing memory
            return self._BLOCK
        need = self.ex.factor_bytes(req.problem)
        if need > self.budget:
            raise ServerError(f"request {req.rid} needs {need} bytes, budget {self.budget}")
        if not self._evict_for(need):
            return self._BLOCK
        entry = _Entry(key, None, need, users=1, ready=False)
        self.used += need
        if self.cache_enabled:
            self.cache[key] = entry
        return self.free_slots.pop(0), entry

    # -- per-request work (runs on the slot's thread) ----------------------------------------
    def _run(self, req: Request, slot: int, entry: _Entry, t0: float, arrival: float):
        res = Result(rid=req.rid, arrival=arrival, slot=slot)
        res.start = time.perf_counter() - t0
        stream = self.streams[slot]
        fresh = not entry.ready
        fac = entry.fac
        try:
            if fresh:
                fac = self.ex.factor(req.problem, stream)
            else:
                res.cache_hit = True
            res.F, res.grad_widths = self.ex.evaluate(fac, req.problem, req.adjoint, stream)
        except Exception as e:      # a failed request frees its slot and memory only
            res.error = str(e)
        res.done = time.perf_counter() - t0
        with self.cv:
            entry.users -= 1
            entry.last_used = res.done
            if fresh:
                keep = self.cache_enabled and fac is not None and res.error is None
                if keep:
                    entry.fac = fac
                    entry.ready = True
                else:
                    if self.cache.get(entry.key) is entry:
                        del self.cache[entry.key]
                    self.used -= entry.nbytes
                    if fac is not None:
                        self.ex.release(fac)
            self.free_slots.append(slot)
            self.free_slots.sort()
            self.inflight -= 1
            self.results[req.rid] = res
            self.cv.notify_all()

    def _run_group(self, reqs: List[Request], slot: int, entry: _Entry, t0: float,
                   arrivals: List[float], work_bytes: int):
        """Plain evaluations of several requests on the same cached factors."""
        start = time.perf_counter() - t0
        err, Fs = None, [None] * len(reqs)
        try:
            Fs = self.ex.evaluate_many(entry.fac, [r.problem for r in reqs], self.streams[slot])
        except Exception as e:
            err = str(e)
        done = time.perf_counter() - t0
        with self.cv:
            self.used -= work_bytes
            entry.users -= 1
            entry.last_used = done
            self.free_slots.append(slot)
            self.free_slots.sort()
            self.inflight -= 1
            for r, a, F in zip(reqs, arrivals, Fs):
                self.results[r.rid] = Result(rid=r.rid, F=F, error=err, arrival=a, start=start,
                                             done=done, cache_hit=True, slot=slot,
                                             group=len(reqs))
            self.cv.notify_all()

    # -- driver -----------------------------------------------------------------------------
    def run(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Serve a request stream.  realtime: replay the arrival times; otherwise
        every request is present at the start (latency counted from there).

        Arrived requests are scanned in arrival order at every change.  A request
        whose geometry is cached but busy (in use, or still being factored) is
        parked and the scan goes on, so it never holds back unrelated requests;
        it starts, or joins a group, once its entry is free.  A fresh request
        that does not fit in memory holds back later fresh requests (first come,
        first served for memory), not requests on cached factors."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        threads = []
        waiting: List[Request] = []
        nxt = 0
        with self.cv:
            while nxt < len(pending) or waiting:
                now = time.perf_counter() - t0
                while nxt < len(pending) and (not realtime or pending[nxt].arrival <= now):
                    waiting.append(pending[nxt])
                    nxt += 1
                started = self._admit_waiting(waiting, t0, now, realtime, threads)
                if started:
                    continue
                timeout = 0.05
                if realtime and nxt < len(pending):
                    timeout = min(timeout, max(pending[nxt].arrival - now, 0.0))
                if waiting or nxt < len(pending):
                    self.cv.wait(timeout=timeout)
        for th in threads:
            th.join()
        return [self.results[r.rid] for r in requests]

    def _admit_waiting(self, waiting: List[Request], t0: float, now: float, realtime: bool,
                       threads: list) -> bool:
        """Start every waiting request that can start now; True if any did."""
        started = False
        fresh_blocked = False
        i = 0
        while i < len(waiting) and self.free_slots:
            req = waiting[i]
            arrival = req.arrival if realtime else 0.0
            try:
                adm = self._try_admit(req, fresh_blocked)
            except ServerError as e:
                self.results[req.rid] = Result(rid=req.rid, error=str(e), arrival=arrival,
                                               done=time.perf_counter() - t0)
                waiting.pop(i)
                started = True
                continue
            if adm is self._PARK:
                i += 1
                continue
            if adm is self._BLOCK:
                fresh_blocked = True
                i += 1
                continue
            slot, entry = adm
            waiting.pop(i)
            started = True
            self.inflight += 1
            self.max_inflight = max(self.max_inflight, self.inflight)
            group, work = [req], 0
            if entry.ready and not req.adjoint and self.group > 1:
                key = geometry_key(req.problem)
                for other in waiting[i:]:
                    if len(group) >= self.group:
                        break
                    if not other.adjoint and geometry_key(other.problem) == key:
                        group.append(other)
                # the grouped call's workspace comes out of the same memory budget
                while len(group) > 1:
                    work = self.ex.many_work_bytes(entry.fac, len(group))
                    if self._evict_for(work):
                        break
                    group.pop()
                    work = 0
                if len(group) > 1:
                    self.used += work
                    taken = {r.rid for r in group[1:]}
                    waiting[i:] = [r for r in waiting[i:] if r.rid not in taken]
            self.peak_bytes = max(self.peak_bytes, self.used)
            if len(group) > 1:
                arrivals = [r.arrival if realtime else 0.0 for r in group]
                th = threading.Thread(target=self._run_group,
                                      args=(group, slot, entry, t0, arrivals, work), daemon=True)
            else:
                th = threading.Thread(target=self._run, args=(req, slot, entry, t0, arrival),
                                      daemon=True)
            th.start()
            threads.append(th)
        return started

    def close(self):
        with self.cv:
            for e in list(self.cache.values()):
                self.ex.release(e.fac)
            self.cache.clear()
            self.used = 0


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
