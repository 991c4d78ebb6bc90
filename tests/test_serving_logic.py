"""Scheduling logic of the continuous-batching server, on the host (fake executor)."""
import threading
import time

import pytest

import workloads as W
from paper_2207_10701_amd.serve import (Arena, FakeExecutor, Server, geometry_key,
                                        serve_sequential, summarize)


def stream(n, **kw):
    return W.serving_stream(n, rate=2000.0, seed=5001, scale=0.05, **kw)


def serve(ex, reqs, realtime=True, **kw):
    srv = Server(ex, **kw)
    try:
        out = srv.run(reqs, realtime=realtime)
    finally:
        srv.close()
    return srv, out


def test_all_requests_served_and_results_deterministic():
    reqs = stream(24)
    ex = FakeExecutor()
    _, out = serve(ex, reqs, eval_slots=3, hbm_budget=10 ** 12)
    assert [r.rid for r in out] == [q.rid for q in reqs]
    assert all(r.error is None for r in out)
    alone = FakeExecutor()
    for q, r in zip(reqs, out):
        F, _ = alone.evaluate(None, q.problem, q.adjoint, None)
        assert r.F == F
        assert (r.grad_widths is not None) == q.adjoint
    s = summarize(out)
    assert s["ok"] == 24 and s["p99_ms"] >= s["p50_ms"] >= 0


def test_fresh_geometries_share_engine_rounds():
    """Geometries that arrive together are factored in the same rounds, up to
    factor_slots at a time."""
    reqs = [W.Request(rid=i, arrival=0.0, problem=W.small_problem(2, 4, seed=100 + i),
                      adjoint=False) for i in range(6)]
    ex = FakeExecutor(factor_seconds=lambda p: 0.01, round_seconds=0.001)
    srv, out = serve(ex, reqs, realtime=False, factor_slots=8, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out)
    assert max(ex.round_sizes) == 6 and srv.max_factoring == 6
    ex2 = FakeExecutor(factor_seconds=lambda p: 0.01, round_seconds=0.001)
    srv2, out2 = serve(ex2, reqs, realtime=False, factor_slots=2, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out2)
    assert max(ex2.round_sizes) == 2


def test_geometry_joins_the_engine_while_others_are_in_progress():
    """A short factorisation that arrives while a long one runs joins the
    engine at once and finishes first (no waiting for the long one)."""
    pa = W.small_problem(2, 4, seed=1)
    pb = W.small_problem(3, 4, seed=2)
    reqs = [W.Request(rid=0, arrival=0.0, problem=pa, adjoint=False),
            W.Request(rid=1, arrival=0.02, problem=pb, adjoint=False)]
    ex = FakeExecutor(factor_seconds=lambda p: 0.2 if p is pa else 0.01, round_seconds=0.001)
    _, out = serve(ex, reqs, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out)
    assert out[1].done < out[0].done
    assert max(ex.round_sizes) == 2


def test_eval_slots_bound_concurrency_and_overlap():
    p = W.small_problem(2, 4, seed=9)
    reqs = [W.Request(rid=i, arrival=0.0, problem=W.small_problem(2, 4, seed=200 + i),
                      adjoint=True) for i in range(12)]
    ex = FakeExecutor(eval_seconds=0.02)
    srv, out = serve(ex, reqs, realtime=False, eval_slots=4, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out)
    assert srv.max_inflight == 4


def test_memory_budget_limits_inflight_and_rejects_oversized():
    reqs = stream(12)
    ex = FakeExecutor(factor_seconds=lambda p: 0.01)
    biggest = max(ex.factor_bytes(r.problem) for r in reqs)
    budget = int(biggest * 1.5)
    srv, out = serve(ex, reqs, realtime=False, hbm_budget=budget, cache=False)
    assert all(r.error is None for r in out)
    assert srv.peak_bytes <= budget
    assert ex.peak_live <= budget
    _, out2 = serve(FakeExecutor(), reqs, realtime=False, hbm_budget=biggest // 2, cache=False)
    big = [r for r, q in zip(out2, reqs) if FakeExecutor().factor_bytes(q.problem) > biggest // 2]
    assert big and all("budget" in r.error for r in big)
    assert any(r.error is None for r in out2)


def test_factor_cache_hits_and_eviction():
    reqs = W.serving_stream(20, rate=2000.0, seed=7, scale=0.05, geometry_pool=3)
    ex = FakeExecutor()
    _, out = serve(ex, reqs, realtime=False, eval_slots=2, hbm_budget=10 ** 12)
    keys = {geometry_key(q.problem) for q in reqs}
    assert ex.factor_calls == len(keys)
    assert sum(r.cache_hit for r in out) == len(reqs) - len(keys)
    # a budget that holds one factor set at a time forces evictions but still serves all
    one = max(ex.factor_bytes(q.problem) for q in reqs)
    ex2 = FakeExecutor()
    _, out2 = serve(ex2, reqs, realtime=False, eval_slots=1, hbm_budget=one)
    assert all(r.error is None for r in out2)
    assert ex2.peak_live <= one


def test_failed_factorisation_does_not_poison_others():
    reqs = stream(10)
    bad = reqs[3].problem.name
    ex = FakeExecutor(fail_on=lambda p: p.name == bad)
    _, out = serve(ex, reqs, realtime=False, hbm_budget=10 ** 12)
    assert out[3].error is not None and "ESINGULAR" in out[3].error
    assert all(r.error is None for i, r in enumerate(out) if i != 3)
    assert ex.live == 0


def test_cached_factors_are_not_shared_by_concurrent_evaluations():
    p = W.small_problem(2, 4, seed=3)
    reqs = [W.Request(rid=i, arrival=0.0, problem=p, adjoint=True) for i in range(6)]
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

    _, out = serve(Probe(), reqs, realtime=False, eval_slots=4, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out)
    assert users["max"] == 1


def test_realtime_replay_respects_arrivals():
    reqs = [W.Request(rid=i, arrival=0.01 * i, problem=W.small_problem(2, 4, seed=i),
                      adjoint=False) for i in range(5)]
    _, out = serve(FakeExecutor(), reqs, eval_slots=2, hbm_budget=10 ** 12)
    for q, r in zip(reqs, out):
        assert r.start >= q.arrival - 1e-3


def test_requests_on_cached_factors_share_one_sweep():
    """Plain requests waiting on one geometry go together (up to `group`);
    adjoint requests never do; results are those of single evaluations;
    group=1 turns grouping off."""
    reqs = stream(40, geometry_pool=2, adjoint_frac=0.25)
    ex = FakeExecutor(factor_seconds=lambda p: 0.02)
    _, out = serve(ex, reqs, realtime=False, eval_slots=1, hbm_budget=10 ** 12, group=8)
    assert all(r.error is None for r in out)
    alone = FakeExecutor()
    for q, r in zip(reqs, out):
        F, _ = alone.evaluate(None, q.problem, q.adjoint, None)
        assert r.F == F
        if q.adjoint:
            assert r.grad_widths is not None and r.group == 1
    assert ex.group_sizes and max(ex.group_sizes) > 1 and max(ex.group_sizes) <= 8
    assert sum(ex.group_sizes) <= sum(1 for q in reqs if not q.adjoint)
    assert ex.factor_calls == 2       # one per geometry of the pool
    ex1 = FakeExecutor(factor_seconds=lambda p: 0.02)
    _, out1 = serve(ex1, reqs, realtime=False, eval_slots=1, hbm_budget=10 ** 12, group=1)
    assert not ex1.group_sizes
    assert [r.F for r in out1] == [r.F for r in out]


def test_group_size_recorded():
    reqs = stream(20, geometry_pool=1, adjoint_frac=0.0)
    _, out = serve(FakeExecutor(factor_seconds=lambda p: 0.02), reqs, realtime=False,
                   eval_slots=1, hbm_budget=10 ** 12, group=6)
    sizes = [r.group for r in out]
    assert max(sizes) == 6 and sum(1 for s in sizes if s == 6) >= 12


def test_request_on_busy_geometry_does_not_block_later_ones():
    """A request whose geometry is still being factored waits on it; an unrelated
    request that arrives after it starts at once (no head-of-line blocking)."""
    pg = W.small_problem(2, 4, seed=3)
    ph = W.small_problem(3, 4, seed=4)
    reqs = [W.Request(rid=0, arrival=0.0, problem=pg, adjoint=False),
            W.Request(rid=1, arrival=0.001, problem=pg, adjoint=True),
            W.Request(rid=2, arrival=0.002, problem=ph, adjoint=False)]
    ex = FakeExecutor(factor_seconds=lambda p: 0.3 if p is pg else 0.002, round_seconds=0.001)
    _, out = serve(ex, reqs, eval_slots=3, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out)
    assert out[2].done < out[0].done       # H finished while G was still factoring
    assert out[1].start >= out[0].start and out[1].cache_hit
    assert ex.factor_calls == 2


def test_group_workspace_counts_against_the_budget():
    """A grouped evaluation's workspace is reserved in the memory ledger; when it
    does not fit, the group shrinks (down to single evaluations)."""
    p = W.small_problem(2, 4, seed=3)
    reqs = [W.Request(rid=i, arrival=0.0, problem=p, adjoint=False) for i in range(9)]
    ex = FakeExecutor()
    fb = ex.factor_bytes(p)
    one = 32 * p.nx * p.ny
    budget = Arena.aligned(fb) + Arena.aligned(4 * one)
    srv, out = serve(ex, reqs, realtime=False, eval_slots=1, hbm_budget=budget, group=8)
    assert all(r.error is None for r in out)
    assert max(r.group for r in out) == 4
    assert srv.peak_bytes <= budget


def test_sequential_baseline_serves_one_at_a_time():
    reqs = stream(6)
    ex = FakeExecutor(factor_seconds=lambda p: 0.005)
    out = serve_sequential(ex, reqs, realtime=False)
    assert all(r.error is None for r in out)
    spans = sorted((r.start, r.done) for r in out)
    assert all(a[1] <= b[0] + 1e-6 for a, b in zip(spans, spans[1:]))
    assert ex.factor_calls == 6 and ex.live == 0


def test_server_arguments():
    with pytest.raises(ValueError):
        Server(FakeExecutor(), factor_slots=9)
    with pytest.raises(ValueError):
        Server(FakeExecutor(), factor_slots=17, engines=2)
    for engines in (0, 5):
        with pytest.raises(ValueError):
            Server(FakeExecutor(), engines=engines)
    with pytest.raises(ValueError):
        Server(FakeExecutor(), eval_slots=0)
    Server(FakeExecutor(), factor_slots=16, engines=2).close()


def test_two_engines_share_the_fresh_geometries():
    """With two engines, geometries that arrive together go to the emptier one:
    twelve split six and six, each engine's rounds shared by its six; every
    result is the one a lone evaluation gives."""
    reqs = [W.Request(rid=i, arrival=0.0, problem=W.small_problem(2, 4, seed=300 + i),
                      adjoint=i % 3 == 0) for i in range(12)]
    ex = FakeExecutor(factor_seconds=lambda p: 0.02, round_seconds=0.001)
    srv, out = serve(ex, reqs, realtime=False, factor_slots=16, engines=2, hbm_budget=10 ** 12)
    assert all(r.error is None for r in out)
    assert srv.max_factoring == 12 and max(ex.round_sizes) == 6
    alone = FakeExecutor()
    for q, r in zip(reqs, out):
        F, _ = alone.evaluate(None, q.problem, q.adjoint, None)
        assert r.F == F


def test_two_engines_respect_the_slot_limit_and_fail_alone():
    """factor_slots bounds the geometries in both engines together; a failing
    geometry in one engine fails only its own requests."""
    reqs = [W.Request(rid=i, arrival=0.0, problem=W.small_problem(2, 4, seed=320 + i),
                      adjoint=False) for i in range(10)]
    bad = reqs[3].problem
    ex = FakeExecutor(factor_seconds=lambda p: 0.01, round_seconds=0.001, fail_on=lambda p: p is bad)
    srv, out = serve(ex, reqs, realtime=False, factor_slots=5, engines=2, hbm_budget=10 ** 12)
    assert srv.max_factoring <= 5 and max(ex.round_sizes) <= 3
    assert [r.error is not None for r in out] == [i == 3 for i in range(10)]


def test_arena_places_first_fit_and_merges_free_neighbours():
    a = Arena(10 * 256)
    x = a.place(300)            # two units
    y = a.place(256)
    z = a.place(5 * 256)
    assert (x, y, z) == (0, 512, 768) and a.used == 8 * 256
    assert a.place(3 * 256) is None
    a.release(y, 256)
    assert a.place(2 * 256) == 2048          # the hole of one unit is too small
    a.release(x, 300)
    a.release(z, 5 * 256)
    assert a.free == [(0, 2048)]             # 0..512, 512..768 and 768..2048 merged
    assert a.place(8 * 256) == 0 and a.used == 10 * 256


def test_largest_first_order_starts_the_biggest_factorisation_first():
    reqs = [W.Request(rid=i, arrival=0.0, problem=W.small_problem(2 + i, 4, seed=60 + i),
                      adjoint=False) for i in range(4)]
    for order, first in (("arrival", 0), ("largest_first", 3)):
        ex = FakeExecutor(factor_seconds=lambda p: 0.01, round_seconds=0.001)
        srv, out = serve(ex, reqs, realtime=False, factor_slots=1, hbm_budget=10 ** 12, order=order)
        assert all(r.error is None for r in out)
        assert min(out, key=lambda r: r.done).rid == first


def test_factors_a_waiting_request_needs_are_not_evicted():
    """With memory for two factor sets and no free evaluation slot, factors that
    completed for a waiting request stay until it is served (no re-factoring)."""
    reqs = [W.Request(rid=i, arrival=0.0, problem=W.small_problem(2, 4, seed=80 + i),
                      adjoint=True) for i in range(5)]
    ex = FakeExecutor(factor_seconds=lambda p: 0.005, eval_seconds=0.03, round_seconds=0.001)
    one = ex.factor_bytes(reqs[0].problem)
    _, out = serve(ex, reqs, realtime=False, eval_slots=1, hbm_budget=2 * Arena.aligned(one))
    assert all(r.error is None for r in out)
    assert ex.factor_calls == 5
