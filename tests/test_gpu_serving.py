"""Serving on the GPU: results in the concurrent mix equal results alone."""
import pytest

import workloads as W
from oracle import average as ora

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("engines", [1, 2])
def test_mix_equals_alone_and_oracle(rcp, engines):
    import torch
    from paper_2207_10701_amd.serve import GpuExecutor, Server, summarize
    reqs = W.serving_stream(8, rate=500.0, seed=5001, scale=0.04, geometry_pool=5)
    ex = GpuExecutor()
    srv = Server(ex, eval_slots=3, hbm_budget=8 << 30, engines=engines)
    out = srv.run(reqs, realtime=True)
    srv.close()
    assert all(r.error is None for r in out), [r.error for r in out]
    assert srv.max_factoring >= 2
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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reciprocal_average_many_equals_single_calls(rcp, precision):
    """Several objectives and lights on one factor set (concentrator/collimator,
    cone/annulus): one multi-RHS sweep (FP64) or refined solves one by one
    (FP32 factors) give each single call's F; the FP64 ones match the oracle."""
    import torch
    from dataclasses import replace
    prec = rcp.RCP_FP64 if precision == "fp64" else rcp.RCP_FP32_REFINED
    base = W.small_problem(5, 4, seed=8)
    probs = [
        base,
        W.with_light(base, light=W.ANNULUS, th1=0.1, th2=0.4),
        replace(base, objective=W.COLLIMATOR, monitor_row=base.ny - base.npml - 5, phi=0.1),
        replace(W.with_light(base, light=W.CONE, c=0.05), focus=(base.focus[0] + 7, base.focus[1])),
        replace(base, objective=W.COLLIMATOR, monitor_row=base.ny - base.npml - 9,
                light=W.ANNULUS, th1=0.2, th2=0.5),
    ]
    fac = rcp.Factors(base, rcp.eps_from_widths(base, device="cuda"), prec)
    F = rcp.reciprocal_average_many(fac, probs).cpu().numpy()
    for k, q in enumerate(probs):
        Fs = rcp.reciprocal_average(fac, q).item()
        assert abs(F[k] - Fs) <= 1e-12 * abs(Fs), (k, F[k], Fs)
        if prec == rcp.RCP_FP64 and k in (0, 2):
            ref = ora.reciprocal(ora.setup(q))
            assert abs(F[k] - ref) / ref < 1e-10
    torch.cuda.synchronize()


def test_pool_requests_grouped_on_cached_factors(rcp):
    """A pool stream served with grouping: requests that share cached factors
    run as one multi-RHS evaluation; every result equals the request alone."""
    import torch
    from paper_2207_10701_amd.serve import GpuExecutor, Server
    reqs = W.serving_stream(12, rate=500.0, seed=5003, scale=0.04, geometry_pool=2,
                            adjoint_frac=0.0)
    ex = GpuExecutor()
    srv = Server(ex, eval_slots=1, hbm_budget=8 << 30, group=8)
    out = srv.run(reqs, realtime=False)
    srv.close()
    assert all(r.error is None for r in out), [r.error for r in out]
    assert sum(r.cache_hit for r in out) >= len(reqs) - 2
    for q, r in zip(reqs, out):
        fac = rcp.Factors(q.problem, rcp.eps_from_widths(q.problem, device="cuda"))
        F = rcp.reciprocal_average(fac, q.problem).item()
        torch.cuda.synchronize()
        assert abs(F - r.F) <= 1e-10 * abs(F)


def test_wrappers_on_a_side_stream_outside_any_stream_context(rcp):
    """A wrapper called with stream=side while another stream is current allocates
    its temporaries on side: memory the current stream allocates and overwrites
    right after the call cannot be the memory side's kernels still read."""
    import torch
    from dataclasses import replace
    base = W.small_problem(5, 4, seed=8)
    probs = [base, W.with_light(base, light=W.ANNULUS, th1=0.1, th2=0.4),
             replace(base, objective=W.COLLIMATOR, monitor_row=base.ny - base.npml - 5, phi=0.1)]
    fac = rcp.Factors(base, rcp.eps_from_widths(base, device="cuda"))
    ref = rcp.reciprocal_average_many(fac, probs).cpu().tolist()
    single = [rcp.reciprocal_average(fac, q).item() for q in probs]
    assert all(abs(a - b) <= 1e-12 * abs(b) for a, b in zip(ref, single))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for _ in range(3):
        F = rcp.reciprocal_average_many(fac, probs, stream=side)
        junk = [torch.full((1 << 20,), 7.0, dtype=torch.float64, device="cuda") for _ in range(8)]
        side.synchronize()
        assert F.cpu().tolist() == ref
        del junk


def test_misaligned_workspace_is_rejected(rcp):
    import torch
    from paper_2207_10701_amd import _lib
    p = W.small_problem(4, 4, seed=7)
    fac = rcp.Factors(p, rcp.eps_from_widths(p, device="cuda"))
    need = int(_lib.lib.rcp_reciprocal_many_work_bytes(fac.handle, 2))
    work = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(rcp.RecipError) as e:
        rcp.reciprocal_average_many(fac, [p, p], work=work[8:])
    assert e.value.code == _lib.RCP_EINVAL and "aligned" in str(e.value)


@pytest.mark.timeout(600)
def test_literal_serving_stream_mix_equals_alone(rcp):
    """The serving stream as stated (64 requests at 200/s, widths 20-300 and
    depths 10-60 wavelengths, fresh geometries, 20% adjoint) through the
    engine server: the two largest requests give the same F (1e-10) as when
    factored and evaluated alone, and the smallest matches the oracle."""
    import numpy as np
    import torch
    from paper_2207_10701_amd.serve import GpuExecutor, Server
    reqs = W.serving_stream(64, rate=200.0, seed=5001, scale=1.0, adjoint_frac=0.2)
    work = np.array([4.0 * q.problem.ny ** 3 * q.problem.nx for q in reqs])
    print(f"serving stream: {len(reqs)} requests, {work.sum() / 1e12:.0f} TFLOP", flush=True)
    free, _ = torch.cuda.mem_get_info()
    ex = GpuExecutor()
    srv = Server(ex, hbm_budget=int(free - (24 << 30)))
    out = srv.run(reqs, realtime=True)
    srv.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    assert all(r.error is None for r in out), [r.error for r in out if r.error][:3]
    assert srv.max_factoring >= 4
    for k in np.argsort(-work)[:2]:
        q, r = reqs[k], out[k]
        fac = rcp.Factors(q.problem, rcp.eps_from_widths(q.problem))
        if q.adjoint:
            F, g = rcp.adjoint_grad(fac, q.problem)
            gw = rcp.width_grad(q.problem, g).cpu().numpy()
            assert np.linalg.norm(gw - r.grad_widths) <= 1e-9 * np.linalg.norm(gw)
        else:
            F = rcp.reciprocal_average(fac, q.problem)
        assert abs(F.item() - r.F) <= 1e-10 * abs(F.item()), (k, F.item(), r.F)
        del fac
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    k = int(np.argmin(work))
    ref = ora.reciprocal(ora.setup(reqs[k].problem))
    assert abs(out[k].F - ref) / ref < 1e-10
