"""GPU broadband average (one geometry at the wavelengths of a spectral rule,
factored side by side) against the FP64 oracle.

Tolerances: FP64 path 1e-10 relative on averages, 1e-9 on gradients; refined
FP32 factors 1e-6 on averages, 1e-5 on gradients.
"""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from gradcheck import assert_grad_close
from oracle import average as ora

pytestmark = pytest.mark.gpu

CONC = W.small_problem(4, 4, seed=7)
COLL = W.small_problem(5, 4, seed=8, objective=W.COLLIMATOR, light=W.ANNULUS,
                       th1_deg=6.0, th2_deg=25.0, monitor_y=3.0, phi=0.1)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def factor_rule(rcp, p, lams, precision=None):
    precision = rcp.RCP_FP64 if precision is None else precision
    probs = [ora.at_wavelength(p, lam) for lam in lams]
    eps = [rcp.eps_from_widths(q, device="cuda") for q in probs]
    return probs, rcp.factor_batch(probs, eps, precision)


@pytest.mark.parametrize("p,n", [(CONC, 3), (COLL, 4), (W.config1(), 8)],
                         ids=["concentrator-3", "collimator-4", "config1-8"])
def test_broadband_matches_oracle(rcp, p, n):
    lams, wts = W.spectral_rule(n, 0.85, 1.15)
    probs, facs = factor_rule(rcp, p, lams)
    F, g = rcp.broadband_grad(facs, wts, probs)
    ref = ora.broadband(p, lams, wts)
    F = F.cpu().numpy()
    np.testing.assert_allclose(F[:-1], ref.F, rtol=1e-10)
    assert abs(F[-1] - ref.total) <= 1e-10 * abs(ref.total)
    assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-9)
    assert_grad_close(rcp.width_grad(p, g).cpu().numpy(), ref.grad_widths, 1e-9)


def test_broadband_terms_equal_lone_wavelengths(rcp):
    """Each term equals the single-wavelength average of a lone factorisation."""
    p = CONC
    lams, wts = W.spectral_rule(3, 0.85, 1.15)
    probs, facs = factor_rule(rcp, p, lams)
    F, _ = rcp.broadband_grad(facs, wts, probs)
    for k, q in enumerate(probs):
        lone = rcp.Factors(q, rcp.eps_from_widths(q, device="cuda"))
        Fl = rcp.reciprocal_average(lone, q).item()
        assert abs(F[k].item() - Fl) <= 1e-12 * abs(Fl)


def test_broadband_refined_fp32(rcp):
    p = COLL
    lams, wts = W.spectral_rule(2, 0.9, 1.1)
    probs, facs = factor_rule(rcp, p, lams, rcp.RCP_FP32_REFINED)
    F, g = rcp.broadband_grad(facs, wts, probs)
    ref = ora.broadband(p, lams, wts)
    np.testing.assert_allclose(F.cpu().numpy()[:-1], ref.F, rtol=1e-6)
    assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-5)


def test_broadband_argument_checks(rcp):
    p = CONC
    lams, wts = W.spectral_rule(2, 0.9, 1.1)
    probs, facs = factor_rule(rcp, p, lams)
    with pytest.raises(rcp.RecipError, match="finite"):
        rcp.broadband_grad(facs, [1.0, float("nan")], probs)
    with pytest.raises(ValueError):
        rcp.broadband_grad(facs, [1.0], probs)


@pytest.mark.timeout(900)
def test_config2_broadband_at_full_size(rcp):
    """Config 2 (2040 x 1080) at the eight wavelengths of the bench's rule: the
    terms equal lone factorisations, the first term matches the oracle, and the
    average obeys the dimensional scaling F(lambda, h) = F(1, h / lambda)."""
    import torch
    p = W.config2()
    lams, wts = W.spectral_rule(8, 0.9, 1.1)
    probs, facs = factor_rule(rcp, p, lams)
    F, g = rcp.broadband_grad(facs, wts, probs)
    F = F.cpu().numpy()
    assert abs(F[-1] - float(np.dot(wts, F[:-1]))) <= 1e-13 * abs(F[-1])
    assert np.isfinite(g.cpu().numpy()).all()
    del facs
    torch.cuda.synchronize()
    q0 = probs[0]
    lone = rcp.Factors(q0, rcp.eps_from_widths(q0, device="cuda"))
    assert abs(rcp.reciprocal_average(lone, q0).item() - F[0]) <= 1e-12 * abs(F[0])
    del lone
    lam = lams[0]
    qs = replace(p, h=p.h / lam, pillar_centers=tuple(c / lam for c in p.pillar_centers),
                 widths=tuple(w / lam for w in p.widths))
    scaled = rcp.Factors(qs, rcp.eps_from_widths(qs, device="cuda"))
    assert abs(rcp.reciprocal_average(scaled, qs).item() - F[0]) <= 1e-10 * abs(F[0])
    del scaled
    ref = ora.reciprocal(ora.setup(q0))
    assert abs(F[0] - ref) <= 1e-10 * abs(ref)
