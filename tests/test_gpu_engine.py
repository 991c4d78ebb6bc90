"""The factorisation engine: geometries of different grid sizes share kernel
launches and join while others are in progress; every geometry's factors are
the same bits as the batched two-panel sweep's, and its averages match the
oracle."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import average as ora

pytestmark = pytest.mark.gpu


def mixed_problems():
    """Grids of 3, 4, 5 and 6 tiles per block edge (odd and even panel counts,
    ragged block sizes), concentrators and collimators, cones and annuli."""
    return [
        W.small_problem(4, 4, seed=7),                                       # 100 rows, 4 tiles
        W.small_problem(6, 3, seed=11, objective=W.COLLIMATOR, light=W.ANNULUS,
                        th1_deg=6.0, th2_deg=22.0, monitor_y=2.0, phi=0.1),  # 80 rows, 3 tiles
        W.small_problem(3, 6, seed=12, c_deg=25.0),                          # 140 rows, 5 tiles
        W.small_problem(5, 8, seed=13, focus_height=4.0),                    # 180 rows, 6 tiles
        replace(W.small_problem(4, 5, seed=14), name="ragged"),              # 120 rows, 4 tiles
    ]


def test_engine_mix_equals_batched_sweep_and_oracle(rcp):
    import torch
    probs = mixed_problems()
    eps = [rcp.eps_from_widths(p) for p in probs]
    eng = rcp.FactorEngine()
    facs = {}
    # three geometries start together, two more join after a few rounds
    for k in range(3):
        facs[k] = eng.add(probs[k], eps[k])
    done = []
    for _ in range(5):
        done += eng.step(rounds=1)
    for k in range(3, 5):
        facs[k] = eng.add(probs[k], eps[k])
    done += eng.run()
    assert len(done) == 5 and all(err is None for _, err in done)
    assert len(eng) == 0
    for k, p in enumerate(probs):
        F, z = rcp.reciprocal_average(facs[k], p, want_z=True)
        # the same geometry factored by the batched sweep (two chains per geometry,
        # two panels per pass): identical bits
        pair = rcp.factor_batch([p, p], [eps[k], eps[k]])
        Fb, zb = rcp.reciprocal_average(pair[0], p, want_z=True)
        assert torch.equal(z, zb), p.name
        assert F.item() == Fb.item()
        ref = ora.reciprocal(ora.setup(p))
        assert abs(F.item() - ref) / ref < 1e-10, p.name
    eng.close()


def test_engine_refined_fp32_and_adjoint(rcp):
    """FP32 factors from the engine, refined solves: F and the gradient against
    the oracle (1e-6 and 1e-5)."""
    from gradcheck import assert_grad_close
    probs = mixed_problems()[1:4]
    eng = rcp.FactorEngine(rcp.RCP_FP32_REFINED)
    facs = [eng.add(p, rcp.eps_from_widths(p)) for p in probs]
    done = eng.run()
    assert all(err is None for _, err in done)
    for fac, p in zip(facs, probs):
        F, g = rcp.adjoint_grad(fac, p)
        ref = ora.adjoint(ora.setup(p))
        assert abs(F.item() - ref.F) / ref.F < 1e-6
        assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-5)
    eng.close()


def test_engine_reports_a_singular_geometry_and_keeps_the_others(rcp):
    import torch
    p = W.small_problem(3, 4, seed=3)
    q = W.small_problem(4, 4, seed=7)
    bad = rcp.eps_from_widths(p)
    bad[p.nx // 2, p.ny // 2] = float("nan")
    eng = rcp.FactorEngine()
    eng.add(p, bad)
    good = eng.add(q, rcp.eps_from_widths(q))
    done = eng.run()
    errs = [err for _, err in done]
    assert sum(e is not None for e in errs) == 1
    e = next(e for e in errs if e is not None)
    assert e.code == -3 and "pivot" in str(e)
    F = rcp.reciprocal_average(good, q).item()
    ref = ora.reciprocal(ora.setup(q))
    assert abs(F - ref) / ref < 1e-10
    eng.close()


def test_engine_admission_limits(rcp):
    p = W.small_problem(2, 4, seed=3)
    eng = rcp.FactorEngine()
    eps = rcp.eps_from_widths(p)
    for _ in range(8):
        eng.add(p, eps)
    with pytest.raises(rcp.RecipError):
        eng.add(p, eps)
    done = eng.run()
    assert len(done) == 8 and all(err is None for _, err in done)
    import torch
    tiny = replace(p, ny=32)                            # one tile per block edge
    with pytest.raises(rcp.RecipError):
        eng.add(tiny, torch.ones((tiny.nx, tiny.ny), dtype=torch.float64, device="cuda"))
    eng.close()
