"""GPU dense form (any correlation W, many outputs) against the FP64 oracle.

Both sides take the same inputs from ``workloads`` (angles, amplitude
correlation, outputs, or a seeded Hermitian W) and build everything else on
their own.  Tolerances: FP64 path 1e-10 relative on fields and averages, 1e-9 on
gradients; refined FP32 factors 1e-8 on fields and 1e-6 on averages.
"""
from functools import lru_cache

import numpy as np
import pytest

import workloads as W
from gradcheck import assert_grad_close
from oracle import average as ora
from oracle import light

pytestmark = pytest.mark.gpu


@lru_cache(maxsize=None)
def oracle_setup(p):
    return ora.setup(p)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def gpu_factors(rcp, p, precision=None):
    import torch
    precision = rcp.RCP_FP64 if precision is None else precision
    fac = rcp.Factors(p, rcp.eps_from_widths(p, device="cuda"), precision)
    torch.cuda.synchronize()
    return fac


CONC = W.small_problem(4, 4, seed=7)
ANN = W.small_problem(5, 4, seed=8, objective=W.COLLIMATOR, light=W.ANNULUS,
                      th1_deg=6.0, th2_deg=25.0, monitor_y=3.0, phi=0.1)
# 90 line cells and 116 rows: ragged against the 64-row and 16-column tiles
ODD = W.small_problem(3, 5, seed=9, npml=8, c_deg=30.0)
CASES = {"conc": CONC, "ann": ANN, "odd": ODD}


def ensemble(p, n, sigma=3.0, tilt=4.0):
    th = W.ensemble_angles(p, n)
    return th, W.gaussian_correlated_amplitudes(th, sigma_deg=sigma, tilt=tilt)


def torch_in(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name,n", [("conc", 24), ("ann", 38), ("odd", 37), ("conc", 130)])
def test_correlation_matrix_matches_oracle(rcp, name, n):
    p = CASES[name]
    if p.light == W.ANNULUS and n % 2:
        n += 1
    th, Ca = ensemble(p, n)
    Wg = rcp.correlation_matrix(p, torch_in(th), torch_in(Ca)).cpu().numpy()
    Wo = light.ensemble_correlation(p, th, Ca)
    assert Wg.shape == Wo.shape == (p.m_aperture, p.m_aperture)
    assert np.abs(Wg - Wo).max() <= 1e-12 * np.abs(Wo).max()


@pytest.mark.parametrize("name,spots,modes", [("conc", 1, 0), ("conc", 2, 1), ("ann", 4, 4),
                                              ("odd", 12, 5), ("conc", 30, 10)])
def test_dense_average_matches_oracle(rcp, name, spots, modes):
    """One output takes the vector sweep, two or more one multi-RHS sweep (16 x 16
    output tiles below 64 right-hand sides)."""
    p = CASES[name]
    outs = W.output_set(p, spots, modes, seed=3100 + spots)
    th, Ca = ensemble(p, 24)
    fac = gpu_factors(rcp, p)
    Wg = rcp.correlation_matrix(p, torch_in(th), torch_in(Ca))
    F, V = rcp.reciprocal_average_dense(fac, outs, Wg, want_v=True)
    Fo, Vo = ora.reciprocal_dense(oracle_setup(p), outs, light.ensemble_correlation(p, th, Ca))
    F = F.cpu().numpy()
    assert rel(V.cpu().numpy().T, Vo) < 1e-10
    np.testing.assert_allclose(F[:-1], Fo, rtol=1e-10)
    assert abs(F[-1] - Fo.sum()) <= 1e-10 * abs(Fo.sum())


@pytest.mark.parametrize("K", [3, 9])
def test_dense_average_of_a_seeded_hermitian_matrix(rcp, K):
    p = ODD
    outs = W.output_set(p, K - 1, 1, seed=3200 + K)
    Wm = W.random_hermitian(p.m_aperture, seed=93)
    fac = gpu_factors(rcp, p)
    F = rcp.reciprocal_average_dense(fac, outs, torch_in(Wm)).cpu().numpy()
    Fo, _ = ora.reciprocal_dense(oracle_setup(p), outs, Wm)
    assert np.abs(F[:-1] - Fo).max() <= 1e-10 * np.abs(Fo).max()


def test_dense_toeplitz_matrix_equals_fft_form(rcp):
    """W = the closed-form Toeplitz correlation: each F_k equals the FFT path's F."""
    p = CONC
    outs = W.output_set(p, 3, 2, seed=3300)
    fac = gpu_factors(rcp, p)
    F = rcp.reciprocal_average_dense(fac, outs, torch_in(light.toeplitz_matrix(p))).cpu().numpy()
    for k, o in enumerate(outs):
        Ff = rcp.reciprocal_average(fac, o).item()
        assert abs(F[k] - Ff) <= 1e-11 * abs(Ff)


@pytest.mark.parametrize("name,spots,modes", [("conc", 1, 1), ("odd", 7, 2), ("ann", 3, 8)])
def test_dense_adjoint_matches_oracle(rcp, name, spots, modes):
    p = CASES[name]
    outs = W.output_set(p, spots, modes, seed=3400 + spots)
    th, Ca = ensemble(p, 20, sigma=4.0, tilt=2.0)
    fac = gpu_factors(rcp, p)
    Wg = rcp.correlation_matrix(p, torch_in(th), torch_in(Ca))
    F, g = rcp.adjoint_grad_dense(fac, outs, Wg)
    ref = ora.adjoint_dense(oracle_setup(p), outs, light.ensemble_correlation(p, th, Ca))
    np.testing.assert_allclose(F.cpu().numpy()[:-1], ref.F, rtol=1e-10)
    assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-9)
    gw = rcp.width_grad(p, g).cpu().numpy()
    assert_grad_close(gw, ref.grad_widths, 1e-9)


def test_dense_refined_fp32_matches_oracle(rcp):
    p = ODD
    outs = W.output_set(p, 6, 3, seed=3500)
    th, Ca = ensemble(p, 30)
    fac = gpu_factors(rcp, p, rcp.RCP_FP32_REFINED)
    Wg = rcp.correlation_matrix(p, torch_in(th), torch_in(Ca))
    F, V = rcp.reciprocal_average_dense(fac, outs, Wg, want_v=True)
    Fa, g = rcp.adjoint_grad_dense(fac, outs, Wg)
    ref = ora.adjoint_dense(oracle_setup(p), outs, light.ensemble_correlation(p, th, Ca))
    assert rel(V.cpu().numpy().T, ref.V) < 1e-8
    np.testing.assert_allclose(F.cpu().numpy()[:-1], ref.F, rtol=1e-6)
    assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-5)


def test_dense_repeated_calls_reuse_the_workspace(rcp):
    """A second, smaller call on the same workspace gives the result of a fresh one."""
    import torch
    p = CONC
    fac = gpu_factors(rcp, p)
    th, Ca = ensemble(p, 24)
    Wg = rcp.correlation_matrix(p, torch_in(th), torch_in(Ca))
    big = W.output_set(p, 20, 4, seed=3600)
    small = big[:5]
    need = int(rcp.lib.rcp_dense_work_bytes(fac.handle, len(big), p.m_aperture))
    work = torch.full((need,), 255, dtype=torch.uint8, device="cuda")
    rcp.reciprocal_average_dense(fac, big, Wg, work=work)
    F2 = rcp.reciprocal_average_dense(fac, small, Wg, work=work).cpu().numpy()
    F1 = rcp.reciprocal_average_dense(fac, small, Wg).cpu().numpy()
    assert np.array_equal(F1, F2)


def test_dense_argument_errors(rcp):
    import torch
    p = CONC
    fac = gpu_factors(rcp, p)
    Wg = torch.zeros((p.m_aperture, p.m_aperture), dtype=torch.complex128, device="cuda")
    with pytest.raises(rcp.RecipError, match="outside the physical region"):
        bad = W.output_set(p, 1)[0]
        from dataclasses import replace
        rcp.reciprocal_average_dense(fac, [replace(bad, focus=(0, 0))], Wg)
    # the C ABI rejects a workspace below rcp_dense_work_bytes (the binding would allocate one)
    import ctypes as C
    from paper_2207_10701_amd import _lib
    outs = W.output_set(p, 2)
    objs = (_lib.Objective * 2)(*[rcp.objective_struct(o) for o in outs])
    lt = rcp.light_struct(p)
    need = int(rcp.lib.rcp_dense_work_bytes(fac.handle, 2, p.m_aperture))
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    F = torch.empty(3, dtype=torch.float64, device="cuda")
    rc = rcp.lib.rcp_reciprocal_average_dense(fac.handle, 2, objs, C.byref(lt), Wg.data_ptr(),
                                              F.data_ptr(), None, work.data_ptr(), need - 1, None)
    assert rc == _lib.RCP_ENOMEM and b"workspace" in rcp.lib.rcp_last_error()


@pytest.mark.timeout(900)
def test_config2_dense_matches_oracle_at_full_size(rcp):
    """Benchmark size (2040 x 1080, 2000 line cells): 16 outputs, a 1000-planewave
    Gaussian-correlated ensemble; F_k, v_k and the gradient against the oracle."""
    p = W.config2()
    outs = W.output_set(p, 12, 4, seed=3700)
    th, Ca = ensemble(p, 1000, sigma=1.0, tilt=5.0)
    fac = gpu_factors(rcp, p)
    Wg = rcp.correlation_matrix(p, torch_in(th), torch_in(Ca))
    F, V = rcp.reciprocal_average_dense(fac, outs, Wg, want_v=True)
    Fa, g = rcp.adjoint_grad_dense(fac, outs, Wg)
    Wo = light.ensemble_correlation(p, th, Ca)
    rng = np.random.default_rng(3701)
    js = rng.integers(0, p.m_aperture, 64)
    ls = rng.integers(0, p.m_aperture, 64)
    Wgs = Wg[torch_in(js), torch_in(ls)].cpu().numpy()
    assert np.abs(Wgs - Wo[js, ls]).max() <= 1e-12 * np.abs(Wo).max()
    ref = ora.adjoint_dense(ora.setup(p), outs, Wo)
    assert rel(V.cpu().numpy().T, ref.V) < 1e-10
    np.testing.assert_allclose(F.cpu().numpy()[:-1], ref.F, rtol=1e-10)
    np.testing.assert_allclose(Fa.cpu().numpy()[:-1], ref.F, rtol=1e-10)
    assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-9)
