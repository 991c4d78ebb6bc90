"""Batched inverse design on the GPU against the same optimizer driven by the
FP64 oracle: identical L-BFGS-B trajectories to rounding, and the average grows."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import average as ora

pytestmark = pytest.mark.gpu


def oracle_batch(batch):
    out = []
    for p, x in batch:
        g = ora.adjoint(ora.setup(replace(p, widths=tuple(float(v) for v in x))))
        out.append((g.F, g.grad_widths))
    return out


@pytest.mark.parametrize("ndesigns", [1, 3])
def test_design_trajectories_match_oracle(rcp, ndesigns):
    from paper_2207_10701_amd.design import gpu_batch_fn, maximize
    base = W.small_problem(3, 3, seed=31, npml=8, focus_height=1.0)
    probs = [replace(base, name=f"d{k}", widths=W.seeded_widths(len(base.widths), 700 + k))
             for k in range(ndesigns)]
    rg, lg = maximize(probs, gpu_batch_fn(), iters=6)
    ro, lo = maximize(probs, oracle_batch, iters=6)
    assert lg.rounds == lo.rounds
    for a, b in zip(rg, ro):
        assert len(a.history) == len(b.history)
        np.testing.assert_allclose(a.history, b.history, rtol=1e-8)
        np.testing.assert_allclose(a.widths, b.widths, atol=1e-7)
        assert a.F > 1.05 * a.F0
