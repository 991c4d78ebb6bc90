"""Serving on the GPU: results in the concurrent mix equal results alone."""
import pytest

import workloads as W
from oracle import average as ora

pytestmark = pytest.mark.gpu


def test_mix_equals_alone_and_oracle(rcp):
    import torch
    from paper_2207_10701_amd.serve import GpuExecutor, Server, summarize
    reqs = W.serving_stream(8, rate=500.0, seed=5001, scale=0.04, geometry_pool=5)
    ex = GpuExecutor()
    srv = Server(ex, slots=3, hbm_budget=8 << 30)
    out = srv.run(reqs, realtime=True)
    srv.close()
    assert all(r.error is None for r in out), [r.error for r in out]
    assert srv.max_inflight >= 2
    s = summarize(out)
    assert s["ok"] == len(reqs)
    # each request alone, on the default stream, with fresh factors
    for q, r in zip(reqs, out):
        eps = rcp.eps_from_widths(q.problem, device="cuda")
        fac = rcp.Factors(q.problem, eps)
        if q.adjoint:
            F, g = rcp.adjoint_grad(fac, q.problem)
        else:
            F = rcp.reciprocal_average(fac, q.problem)
        torch.cuda.synchronize()
        assert abs(F.item() - r.F) <= 1e-10 * abs(F.item())
    # two of them against the oracle
    for q, r in list(zip(reqs, out))[:2]:
        ref = ora.reciprocal(ora.setup(q.problem))
        assert abs(r.F - ref) / ref < 1e-10
