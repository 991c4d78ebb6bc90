"""The allocation-free grouped reciprocal average (workspace in the library's
static device array) against the entry point that takes a workspace: the same
F to the bit, on two calls in a row, the second with a smaller input."""
import ctypes as C
from dataclasses import replace

import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def requests(base):
    return [
        base,
        W.with_light(base, light=W.ANNULUS, th1=0.1, th2=0.4),
        replace(base, objective=W.COLLIMATOR, monitor_row=base.ny - base.npml - 5, phi=0.1),
        replace(W.with_light(base, light=W.CONE, c=0.05), focus=(base.focus[0] + 7, base.focus[1])),
        replace(base, objective=W.COLLIMATOR, monitor_row=base.ny - base.npml - 9,
                light=W.ANNULUS, th1=0.2, th2=0.5),
    ]


def noalloc(rcp, fac, probs):
    """Through the C ABI; F (the output) is the caller's."""
    import torch
    from paper_2207_10701_amd import _lib
    K = len(probs)
    F = torch.full((K,), float("nan"), dtype=torch.float64, device="cuda")
    objs = (_lib.Objective * K)(*[rcp.objective_struct(p) for p in probs])
    lights = (_lib.Light * K)(*[rcp.light_struct(p) for p in probs])
    rc = _lib.lib.rcp_reciprocal_average_many_noalloc(
        fac.handle, K, objs, lights, F.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return rc, F


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_workspace_entry_point(rcp, precision):
    import torch
    prec = rcp.RCP_FP64 if precision == "fp64" else rcp.RCP_FP32_REFINED
    big = W.small_problem(5, 4, seed=8)
    small = W.small_problem(3, 4, seed=9)
    for base, count in ((big, 5), (small, 2)):      # the second call: a smaller input
        probs = requests(base)[:count]
        fac = rcp.Factors(base, rcp.eps_from_widths(base), prec)
        ref = rcp.reciprocal_average_many(fac, probs)
        rc, F = noalloc(rcp, fac, probs)
        assert rc == 0, rcp.lib.rcp_last_error()
        torch.cuda.synchronize()
        assert torch.equal(F, ref), (F, ref)


def test_noalloc_rejects_workspaces_beyond_the_array(rcp):
    import torch
    from paper_2207_10701_amd import _lib
    p = W.config4_large()                 # 2040 x 440 cells: 28.7 MB per field
    fac = rcp.Factors(p, rcp.eps_from_widths(p))
    need = int(_lib.lib.rcp_reciprocal_many_work_bytes(fac.handle, 10))
    assert need > (256 << 20)
    rc, F = noalloc(rcp, fac, [p] * 10)
    assert rc == _lib.RCP_ENOMEM and b"scratch" in _lib.lib.rcp_last_error()
    torch.cuda.synchronize()
    assert torch.isnan(F).all()           # nothing was launched
    rc, F = noalloc(rcp, fac, [p] * 4)    # within the array: runs
    assert rc == 0
    ref = rcp.reciprocal_average_many(fac, [p] * 4)
    torch.cuda.synchronize()
    assert torch.equal(F, ref)
