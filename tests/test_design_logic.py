"""Host logic of the batched inverse-design loop (no GPU): lockstep batching of
several L-BFGS-B runs on known objectives."""
from dataclasses import replace

import numpy as np

import workloads as W
from paper_2207_10701_amd.design import Lockstep, maximize


def quad_batch(targets, calls):
    def fn(batch):
        calls.append(len(batch))
        out = []
        for p, x in batch:
            t = targets[p.name]
            F = -float(np.sum((x - t) ** 2))
            out.append((F, -2.0 * (x - t)))
        return out
    return fn


def test_lockstep_batches_every_running_optimizer_and_finds_the_bounded_optimum():
    base = W.small_problem(3, 3, seed=1)
    probs = [replace(base, name=f"d{k}", widths=W.seeded_widths(3, 50 + k)) for k in range(5)]
    targets = {p.name: np.array([0.2 + 0.1 * k, 0.95, 0.05 + 0.5 * (k % 2)])
               for k, p in enumerate(probs)}
    calls = []
    res, lock = maximize(probs, quad_batch(targets, calls), iters=50, lo=0.1, hi=0.9)
    for k, r in enumerate(res):
        want = np.clip(targets[probs[k].name], 0.1, 0.9)
        np.testing.assert_allclose(r.widths, want, atol=1e-6)
        assert r.F >= r.F0
    # every round carried all optimizers still running, never more than there are
    assert max(calls) == len(probs) and min(calls) >= 1
    assert sum(calls) == lock.evaluations and len(calls) == lock.rounds
    assert lock.rounds < lock.evaluations


def test_lockstep_reports_a_failing_batch_to_every_optimizer():
    base = W.small_problem(3, 3, seed=1)
    probs = [replace(base, name=f"d{k}") for k in range(3)]

    def bad(batch):
        raise ValueError("boom")

    try:
        maximize(probs, bad, iters=3)
    except RuntimeError as e:
        assert "batched evaluation failed" in str(e)
    else:
        raise AssertionError("no error raised")


def test_angle_study_bookkeeping():
    """The study's lens is the best design for the smallest cone, and its gains
    compare each light's optimum with that lens under the same light (synthetic
    objective: F = (1 - |x - t|^2) / angle, t depending on the light)."""
    import math
    from paper_2207_10701_amd.design import angle_study
    base = W.small_problem(3, 3, seed=1)

    def fn(batch):
        out = []
        for p, x in batch:
            ang = p.c if p.light == W.CONE else p.th2
            t = 0.3 if p.light == W.CONE else 0.7
            F = (1.0 - float(np.sum((x - t) ** 2))) / ang
            out.append((F, -2.0 * (x - t) / ang))
        return out

    out = angle_study(base, fn, [1.0, 4.0], annulus_deg=(2.0, 4.0), designs=2, iters=30)
    cones = out["cones"]
    assert [c["c_deg"] for c in cones] == [1.0, 4.0]
    assert cones[0]["F_opt"] > cones[1]["F_opt"]
    for c in cones:   # optimum x = t: F c = 1
        assert abs(c["F_opt_times_c"] - 1.0) < 1e-6
    gains = {g["light"]: g for g in out["gains_over_lens"]}
    # the lens (x = 0.3) under the annulus: 1 - 3 * 0.16 over th2
    assert abs(gains["annulus"]["F_lens"] - (1 - 3 * 0.16) / math.radians(4.0)) < 1e-6
    assert abs(gains["annulus"]["gain"] - 1.0 / (1 - 3 * 0.16)) < 1e-6
    assert abs(gains["cone"]["gain"] - 1.0) < 1e-6


def test_collimator_gains_bookkeeping():
    """Gains are the best optimized F over the mean F of the random starts,
    under each light (synthetic objective with its optimum F = 1)."""
    from paper_2207_10701_amd.design import collimator_gains
    base = W.small_problem(3, 3, seed=1, objective=W.COLLIMATOR)

    def fn(batch):
        out = []
        for p, x in batch:
            t = 0.4 if p.light == W.CONE else 0.6
            out.append((1.0 - float(np.sum((x - t) ** 2)), -2.0 * (x - t)))
        return out

    res = collimator_gains(base, fn, designs=3, iters=30)
    assert [r["light"] for r in res] == ["cone", "annulus"]
    for r in res:
        assert abs(r["F_opt"] - 1.0) < 1e-9
        assert abs(r["gain"] - 1.0 / r["F_random_mean"]) < 1e-9
