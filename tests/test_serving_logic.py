"""Scheduling logic of the continuous-batching server, on the host (fake executor)."""
import threading
import time
from dataclasses import replace

import pytest

import workloads as W
from paper_2207_10701_amd.serve import FakeExecutor, Server, geometry_key, summarize


def stream(n, **kw):
    return W.serving_stream(n, rate=2000.0, seed=5001, scale=0.05, **kw)


def test_all_requests_served_and_results_deterministic():
    reqs = stream(24)
    ex = FakeExecutor()
    out = Server(ex, slots=3, hbm_budget=10 ** 12).run(reqs)
    assert [r.rid for r in out] == [q.rid for q in reqs]
    assert all(r.error is None for r in out)
    alone = FakeExecutor()
    for q, r in zip(reqs, out):
        F, _ = alone.evaluate(None, q.problem, q.adjoint, None)
        assert r.F == F
    s = summarize(out)
    assert s["ok"] == 24 and s["p99_ms"] >= s["p50_ms"] >= 0


def test_slots_bound_concurrency_and_overlap():
    reqs = stream(16)
    srv = Server(FakeExecutor(factor_seconds=lambda p: 0.02), slots=4, hbm_budget=10 ** 12)
    srv.run(reqs, realtime=False)
    assert srv.max_inflight == 4


def test_memory_budget_limits_inflight_and_rejects_oversized():
    reqs = stream(12)
    ex = FakeExecutor(factor_seconds=lambda p: 0.01)
    biggest = max(ex.factor_bytes(r.problem) for r in reqs)
    budget = int(biggest * 1.5)
    srv = Server(ex, slots=8, hbm_budget=budget, cache=False)
    out = srv.run(reqs, realtime=False)
    assert all(r.error is None for r in out)
    assert srv.peak_bytes <= budget
    assert ex.peak_live <= budget
    tiny = Server(FakeExecutor(), slots=2, hbm_budget=biggest // 2, cache=False)
    out2 = tiny.run(reqs, realtime=False)
    big = [r for r, q in zip(out2, reqs) if FakeExecutor().factor_bytes(q.problem) > biggest // 2]
    assert big and all("budget" in r.error for r in big)
    assert any(r.error is None for r in out2)


def test_factor_cache_hits_and_eviction():
    reqs = W.serving_stream(20, rate=2000.0, seed=7, scale=0.05, geometry_pool=3)
    ex = FakeExecutor()
    srv = Server(ex, slots=2, hbm_budget=10 ** 12)
    out = srv.run(reqs, realtime=False)
    keys = {geometry_key(q.problem) for q in reqs}
    assert ex.factor_calls == len(keys)
    assert sum(r.cache_hit for r in out) == len(reqs) - len(keys)
    # a budget that holds one factor set at a time forces evictions but still serves all
    one = max(ex.factor_bytes(q.problem) for q in reqs)
    ex2 = FakeExecutor()
    srv2 = Server(ex2, slots=1, hbm_budget=one)
    out2 = srv2.run(reqs, realtime=False)
    assert all(r.error is None for r in out2)
    assert ex2.peak_live <= one


def test_failed_request_does_not_poison_others():
    reqs = stream(10)
    bad = reqs[3].problem.name
    ex = FakeExecutor(fail_on=lambda p: p.name == bad)
    out = Server(ex, slots=3, hbm_budget=10 ** 12).run(reqs, realtime=False)
    assert out[3].error is not None and "ESINGULAR" in out[3].error
    assert all(r.error is None for i, r in enumerate(out) if i != 3)


def test_cached_factors_are_not_shared_by_concurrent_requests():
    p = W.small_problem(2, 4, seed=3)
    reqs = [W.Request(rid=i, arrival=0.0, problem=p, adjoint=False) for i in range(6)]
    users = {"now": 0, "max": 0}
    lock = threading.Lock()

    class Probe(FakeExecutor):
        def evaluate(self, fac, p, adjoint, stream):
            with lock:
                users["now"] += 1
                users["max"] = max(users["max"], users["now"])
            time.sleep(0.005)
            with lock:
                users["now"] -= 1
            return super().evaluate(fac, p, adjoint, stream)

    out = Server(Probe(), slots=4, hbm_budget=10 ** 12).run(reqs, realtime=False)
    assert all(r.error is None for r in out)
    assert users["max"] == 1


def test_realtime_replay_respects_arrivals():
    reqs = [W.Request(rid=i, arrival=0.01 * i, problem=W.small_problem(2, 4, seed=i),
                      adjoint=False) for i in range(5)]
    out = Server(FakeExecutor(), slots=2, hbm_budget=10 ** 12).run(reqs)
    for q, r in zip(reqs, out):
        assert r.start >= q.arrival - 1e-3


def test_requests_on_cached_factors_share_one_sweep():
    """Requests for a geometry whose factors are cached and ready go together
    (plain evaluations, up to `group`); adjoint requests never do; results are
    those of single evaluations; group=1 turns grouping off."""
    reqs = stream(40, geometry_pool=2, adjoint_frac=0.25)
    ex = FakeExecutor(factor_seconds=lambda p: 0.02)
    out = Server(ex, slots=1, hbm_budget=10 ** 12, group=8).run(reqs, realtime=False)
    assert all(r.error is None for r in out)
    alone = FakeExecutor()
    for q, r in zip(reqs, out):
        F, _ = alone.evaluate(None, q.problem, q.adjoint, None)
        assert r.F == F
        if q.adjoint:
            assert r.grad_widths is not None
    assert ex.group_sizes and max(ex.group_sizes) > 1 and max(ex.group_sizes) <= 8
    grouped = sum(ex.group_sizes)
    plain = sum(1 for q in reqs if not q.adjoint)
    assert grouped <= plain
    assert ex.factor_calls == 2       # one per geometry of the pool
    ex1 = FakeExecutor(factor_seconds=lambda p: 0.02)
    out1 = Server(ex1, slots=1, hbm_budget=10 ** 12, group=1).run(reqs, realtime=False)
    assert not ex1.group_sizes
    assert [r.F for r in out1] == [r.F for r in out]


def test_group_size_recorded():
    reqs = stream(20, geometry_pool=1, adjoint_frac=0.0)
    out = Server(FakeExecutor(factor_seconds=lambda p: 0.02), slots=1, hbm_budget=10 ** 12,
                 group=6).run(reqs, realtime=False)
    sizes = [r.group for r in out]
    assert sizes[0] == 1 and max(sizes) == 6
    assert all(r.cache_hit for r, g in zip(out, sizes) if g > 1)


def test_request_on_busy_geometry_does_not_block_later_ones():
    """A request whose geometry is still being factored waits on it; an unrelated
    request that arrives after it starts at once (no head-of-line blocking)."""
    pg = W.small_problem(2, 4, seed=3)
    ph = W.small_problem(3, 4, seed=4)
    reqs = [W.Request(rid=0, arrival=0.0, problem=pg, adjoint=False),
            W.Request(rid=1, arrival=0.001, problem=pg, adjoint=True),
            W.Request(rid=2, arrival=0.002, problem=ph, adjoint=False)]
    ex = FakeExecutor(factor_seconds=lambda p: 0.3 if p is pg else 0.001)
    out = Server(ex, slots=3, hbm_budget=10 ** 12).run(reqs)
    assert all(r.error is None for r in out)
    assert out[2].done < out[0].done       # H finished while G was still factoring
    assert out[1].start >= out[0].done - 1e-3 and out[1].cache_hit
    assert ex.factor_calls == 2


def test_group_workspace_counts_against_the_budget():
    """A grouped evaluation's workspace is reserved in the memory ledger; when it
    does not fit, the group shrinks (down to single evaluations)."""
    p = W.small_problem(2, 4, seed=3)
    reqs = [W.Request(rid=i, arrival=0.0, problem=p, adjoint=False) for i in range(9)]
    ex = FakeExecutor()
    fb = ex.factor_bytes(p)
    one = 32 * p.nx * p.ny
    srv = Server(ex, slots=1, hbm_budget=fb + 4 * one, group=8)
    out = srv.run(reqs, realtime=False)
    assert all(r.error is None for r in out)
    assert max(r.group for r in out) == 4
    assert srv.peak_bytes <= fb + 4 * one
