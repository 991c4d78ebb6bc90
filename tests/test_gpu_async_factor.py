"""Factorisation without a host wait (rcp_factor_batch_async): the pivot check
runs on the device into each factor set's status word and is read when the
caller asks (rcp_factors_status, rcp_factors_status_dev)."""
import pytest

import workloads as W
from oracle import average as ora

pytestmark = pytest.mark.gpu


def _word_in_buffer(fac):
    """The status word lies in the set's own factor buffer."""
    a = fac.status_dev()
    b = fac.buf.data_ptr()
    assert b <= a < b + fac.buf.numel()


def test_async_batch_equals_the_waiting_batch(rcp):
    ps = [W.small_problem(4, 4, seed=3), W.small_problem(4, 4, seed=7)]
    eps = [rcp.eps_from_widths(p) for p in ps]
    sync = rcp.factor_batch(ps, eps)
    asyn = rcp.factor_batch(ps, eps, wait=False)
    for f in asyn:
        f.status()
        _word_in_buffer(f)
    for p, a, b in zip(ps, sync, asyn):
        assert rcp.reciprocal_average(a, p).item() == rcp.reciprocal_average(b, p).item()


def test_async_batch_reports_the_singular_set_when_asked(rcp):
    p = W.small_problem(4, 4, seed=3)
    q = W.small_problem(4, 4, seed=7)
    bad = rcp.eps_from_widths(p)
    bad[p.nx // 2, p.ny // 2] = float("nan")
    fb, fg = rcp.factor_batch([p, q], [bad, rcp.eps_from_widths(q)], wait=False)   # no raise here
    fg.status()
    with pytest.raises(rcp.RecipError) as ei:
        fb.status()
    assert ei.value.code == -3 and "pivot" in str(ei.value)
    # the NaN sits in block nx // 2 (the middle block, last of the twisted
    # elimination), whose panel holding row ny // 2 is the first to fail
    nt = -(-p.ny // 32)
    assert f"pivot block {(p.ny // 2) // 32} of column block {p.nx // 2}" in str(ei.value), str(ei.value)
    assert nt >= 1
    _word_in_buffer(fb)
    F = rcp.reciprocal_average(fg, q).item()
    ref = ora.reciprocal(ora.setup(q))
    assert abs(F - ref) / ref < 1e-10
