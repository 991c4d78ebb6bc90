"""Batches of 9 to 16 geometries (rcp_factor_batch above eight): two groups,
each factored in its own launches on one of two library streams, forked from
and joined back into the caller's stream.  A geometry's factors are the same in
any batch of two or more, so each set must equal its factorisation in a batch
of two bit for bit, whatever its group, and match the oracle."""
from dataclasses import replace
from functools import lru_cache

import pytest

import workloads as W
from oracle import average as ora

pytestmark = pytest.mark.gpu

BASE = W.small_problem(4, 4, seed=7)


@lru_cache(maxsize=None)
def _oracle_F(p):
    return ora.reciprocal(ora.setup(p))


def _problems(count, seed0):
    return [replace(BASE, widths=W.seeded_widths(len(BASE.widths), seed0 + g)) for g in range(count)]


@pytest.mark.parametrize("count,precision,wait", [(9, "fp64", True), (16, "fp64", False),
                                                  (16, "fp32", True), (11, "fp32", False)])
def test_two_groups_equal_pairs_and_oracle(rcp, count, precision, wait):
    import torch
    prec = rcp.RCP_FP64 if precision == "fp64" else rcp.RCP_FP32_REFINED
    probs = _problems(count, 500)
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps, prec, wait=wait)
    assert len(facs) == count
    if not wait:
        for f in facs:
            f.status()
    Fb = [rcp.reciprocal_average(f, p).item() for f, p in zip(facs, probs)]
    h = (count + 1) // 2
    for g in (0, h - 1, h, count - 1):   # both ends of both groups
        other = (g + 1) % count
        pair = rcp.factor_batch([probs[g], probs[other]], [eps[g], eps[other]], prec)
        assert rcp.reciprocal_average(pair[0], probs[g]).item() == Fb[g]
    for g in (1, count - 2):
        ref = _oracle_F(probs[g])
        assert abs(Fb[g] - ref) / ref < (1e-10 if precision == "fp64" else 1e-8)
    torch.cuda.synchronize()


def test_two_groups_on_a_side_stream(rcp):
    """The groups fork from and join back into a stream that is not the current one."""
    import torch
    probs = _problems(10, 520)
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    ref = [rcp.reciprocal_average(f, p).item() for f, p in zip(rcp.factor_batch(probs, eps), probs)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    facs = rcp.factor_batch(probs, eps, stream=side, wait=False)
    with torch.cuda.stream(side):
        F = [rcp.reciprocal_average(f, p, stream=side) for f, p in zip(facs, probs)]
    side.synchronize()
    assert [x.item() for x in F] == ref


def test_two_groups_name_the_singular_geometry(rcp):
    probs = _problems(9, 540)
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    eps[7][probs[7].nx // 2, probs[7].ny // 2] = float("nan")   # in the second group
    with pytest.raises(rcp.RecipError) as ei:
        rcp.factor_batch(probs, eps)
    assert ei.value.code == -3 and "geometry 7" in str(ei.value)
    facs = rcp.factor_batch(probs, eps, wait=False)   # no raise here
    for g, f in enumerate(facs):
        if g == 7:
            with pytest.raises(rcp.RecipError):
                f.status()
        else:
            f.status()
