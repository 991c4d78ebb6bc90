"""GPU path at the benchmark configurations, against the oracle where it is
affordable (config 1) and against properties that hold at any size (config 2)."""
import math
from functools import lru_cache

import numpy as np
import pytest

import workloads as W
from gradcheck import assert_grad_close
from oracle import average as ora
from oracle import light

pytestmark = pytest.mark.gpu


@lru_cache(maxsize=None)
def config1_oracle():
    p = W.config1()
    s = ora.setup(p)
    return p, s, ora.adjoint(s)


def test_config1_fp64_and_refined_fp32(rcp):
    p, s, ref = config1_oracle()
    eps = rcp.eps_from_widths(p)
    f64 = rcp.Factors(p, eps)
    F, v, z = rcp.reciprocal_average(f64, p, want_v=True, want_z=True)
    zr = ref.z
    assert np.linalg.norm(z.cpu().numpy().ravel() - zr) / np.linalg.norm(zr) < 1e-10
    assert abs(F.item() - ref.F) / ref.F < 1e-10
    # Eq. 6 with 64 Gauss-Legendre nodes on the same factors equals Eq. 7 (converged)
    Fb = rcp.brute_force_average(f64, 64, p, rhs_chunk=32)
    assert abs(Fb.item() - ref.F) / ref.F < 1e-10
    Fa, g = rcp.adjoint_grad(f64, p)
    gd = g.cpu().numpy()
    assert_grad_close(gd, ref.grad_eps, 1e-9)
    gw = rcp.width_grad(p, g).cpu().numpy()
    assert_grad_close(gw, ref.grad_widths, 1e-9)
    f32 = rcp.Factors(p, eps, rcp.RCP_FP32_REFINED)
    F32, z32 = rcp.reciprocal_average(f32, p, want_z=True)
    assert np.linalg.norm(z32.cpu().numpy().ravel() - zr) / np.linalg.norm(zr) < 1e-8
    assert abs(F32.item() - ref.F) / ref.F < 1e-6
    F32a, g32 = rcp.adjoint_grad(f32, p)
    assert_grad_close(g32.cpu().numpy(), ref.grad_eps, 1e-5)


def test_config1_autograd_function(rcp):
    import torch
    p, s, ref = config1_oracle()
    w = torch.tensor(p.widths, dtype=torch.float64, device="cuda", requires_grad=True)
    F = rcp.IncoherentFOM.apply(w, p)
    F.backward()
    assert abs(F.item() - ref.F) / ref.F < 1e-10
    gw = w.grad.cpu().numpy()
    assert_grad_close(gw, ref.grad_widths, 1e-9)


def test_config1_autograd_over_pixel_permittivity(rcp):
    """IncoherentFOM over a per-pixel permittivity map: F and dF/deps of the
    pillar geometry's map against the oracle's adjoint."""
    import torch
    p, s, ref = config1_oracle()
    eps = rcp.eps_from_widths(p).clone().requires_grad_(True)
    F = rcp.IncoherentFOM.apply(eps, p)
    F.backward()
    assert abs(F.item() - ref.F) / ref.F < 1e-10
    assert_grad_close(eps.grad.cpu().numpy(), ref.grad_eps, 1e-9)
    with pytest.raises(ValueError):
        rcp.IncoherentFOM.apply(torch.zeros((p.nx, p.ny + 1), dtype=torch.float64, device="cuda"), p)


def test_symbol_table_light_matches_closed_form(rcp):
    import torch
    p = W.small_problem(4, 4, seed=7)
    eps = rcp.eps_from_widths(p)
    fac = rcp.Factors(p, eps)
    F = rcp.reciprocal_average(fac, p).item()
    M = p.m_aperture
    d = (np.arange(-(M - 1), M) * p.h)
    table = light.correlation_closed_form(p, d).astype(np.complex128)
    Ft = rcp.reciprocal_average(fac, p, symbol=torch.from_numpy(table).cuda()).item()
    assert abs(F - Ft) / F < 1e-12


def test_singular_geometry_reports_esingular(rcp):
    p = W.small_problem(3, 4, seed=3)
    eps = rcp.eps_from_widths(p)
    eps[p.nx // 2, p.ny // 2] = float("nan")
    with pytest.raises(rcp.RecipError) as e:
        rcp.Factors(p, eps)
    assert e.value.code == -3 and "pivot" in str(e.value)


def test_refinement_without_steps_reports_enoconv(rcp):
    import torch
    p = W.small_problem(3, 4, seed=3)
    fac = rcp.Factors(p, rcp.eps_from_widths(p), rcp.RCP_FP32_REFINED)
    b = torch.from_numpy(W.complex_normal((1, p.nx, p.ny), seed=4)).cuda()
    with pytest.raises(rcp.RecipError) as e:
        rcp.solve(fac, b, tol=1e-14, max_refine=0)
    assert e.value.code == -4 and "residual" in str(e.value)
    X, (it, res) = rcp.solve(fac, b, tol=1e-11, max_refine=8)
    assert 1 <= it <= 8 and res <= 1e-11


def test_config2_reciprocal_equals_converged_brute_force(rcp):
    """Full benchmark size: Eq. 7 equals Eq. 6 once the quadrature resolves the
    integrand (N > K c L / 2 = 164 nodes here), and the solve has a tiny residual."""
    import torch
    p = W.config2()
    eps = rcp.eps_from_widths(p)
    fac = rcp.Factors(p, eps)
    F = rcp.reciprocal_average(fac, p).item()
    Fb = rcp.brute_force_average(fac, 256, p, rhs_chunk=128).item()
    assert abs(F - Fb) / F < 1e-10
    K = p.n_source * 2 * math.pi
    assert 256 > K * p.c * (p.m_aperture * p.h) / 2
    b = torch.from_numpy(W.complex_normal((1, p.nx, p.ny), seed=21)).cuda()
    X, (it, res) = rcp.solve(fac, b)
    # computed through the refinement residual kernel (FP64 stencil)
    fac2 = rcp.Factors(p, eps, rcp.RCP_FP32_REFINED)
    X32, (it32, res32) = rcp.solve(fac2, b, tol=1e-12, max_refine=10)
    assert res32 <= 1e-12
    rel = (torch.linalg.vector_norm(X32 - X) / torch.linalg.vector_norm(X)).item()
    assert rel < 1e-9


@lru_cache(maxsize=None)
def config2_setup():
    return ora.setup(W.config2())


@lru_cache(maxsize=None)
def config2_oracle():
    return ora.adjoint(config2_setup())


@pytest.mark.timeout(900)
def test_config2_matches_oracle_at_full_size(rcp):
    """Benchmark size (2040 x 1080): GPU reciprocal field, F and adjoint against the
    FP64 oracle (SuperLU, ~75 s on one core)."""
    p = W.config2()
    eps = rcp.eps_from_widths(p)
    fac = rcp.Factors(p, eps)
    F, z = rcp.reciprocal_average(fac, p, want_z=True)
    Fa, g = rcp.adjoint_grad(fac, p)
    zg = z.cpu().numpy().ravel()
    gg = g.cpu().numpy()
    ref = config2_oracle()
    assert np.linalg.norm(zg - ref.z) / np.linalg.norm(ref.z) < 1e-10
    assert abs(F.item() - ref.F) / ref.F < 1e-10
    assert_grad_close(gg, ref.grad_eps, 1e-9)


@pytest.mark.timeout(900)
def test_config2_batch_of_eight_as_benchmarked(rcp):
    """The benchmark's launch configuration: eight config-2 geometries (the
    benchmark's widths) factored side by side, sixteen chains in every launch
    (two per XCD).  Geometry 0 (the config-2 widths) against the oracle: field, F
    and adjoint; the last two bit-identical to their factorisation as a batch of
    two (four chains); batched adjoints equal single ones."""
    import torch
    from dataclasses import replace
    p = W.config2()
    probs = [replace(p, widths=W.seeded_widths(len(p.widths), 1002 + 97 * k)) for k in range(8)]
    assert probs[0].widths == p.widths
    eps = [rcp.eps_from_widths(q) for q in probs]
    facs = rcp.factor_batch(probs, eps)
    F0, z0 = rcp.reciprocal_average(facs[0], probs[0], want_z=True)
    Fs = [rcp.reciprocal_average(f, q).item() for f, q in zip(facs, probs)]
    Fb, gb = rcp.adjoint_grad_batch(facs, probs)
    F7, g7 = rcp.adjoint_grad(facs[7], probs[7])
    assert Fb[7].item() == F7.item() and torch.equal(gb[7], g7)
    z0 = z0.cpu().numpy().ravel()
    g0 = gb[0].cpu().numpy()
    del facs, F7, g7
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    pair = rcp.factor_batch(probs[6:], eps[6:])
    for f, q, F in zip(pair, probs[6:], Fs[6:]):
        assert rcp.reciprocal_average(f, q).item() == F
    del pair
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    assert len(set(Fs)) == 8
    ref = config2_oracle()
    assert np.linalg.norm(z0 - ref.z) / np.linalg.norm(ref.z) < 1e-10
    assert abs(F0.item() - ref.F) / ref.F < 1e-10
    assert abs(Fs[0] - ref.F) / ref.F < 1e-10
    assert_grad_close(g0, ref.grad_eps, 1e-9)


@pytest.mark.timeout(900)
def test_config3_refined_fp32_vs_fp64_and_oracle(rcp):
    """Collimator, annulus 10-30 deg and mirror (4040 x 440): complex-FP32 factors with
    FP64 refinement against the FP64 path (field 1e-8, F 1e-6), FP64 F against the
    oracle (1e-10)."""
    import torch
    p = W.config3()
    eps = rcp.eps_from_widths(p)
    f64 = rcp.Factors(p, eps)
    F64, z64 = rcp.reciprocal_average(f64, p, want_z=True)
    f32 = rcp.Factors(p, eps, rcp.RCP_FP32_REFINED)
    F32, z32 = rcp.reciprocal_average(f32, p, want_z=True)
    iters, res = f32.last_solve_stats()
    assert iters >= 1 and res <= 1e-12
    zerr = (torch.linalg.vector_norm(z32 - z64) / torch.linalg.vector_norm(z64)).item()
    assert zerr < 1e-8
    assert abs(F32.item() - F64.item()) / F64.item() < 1e-6
    Fo = ora.reciprocal(ora.setup(p))
    assert abs(F64.item() - Fo) / Fo < 1e-10


def test_config4_large_gradients_match_central_differences(rcp):
    """Adjoint step at scale (2040 x 440): dF/dwidth on 20 seeded pillars and dF/deps
    on 20 seeded pixels of the 100 x 10 wavelength region above the substrate,
    against central differences of the FP64 F (2-norm and per component, 1e-5),
    for the FP64 adjoint and the adjoint on complex-FP32 factors with FP64
    refinement; the two adjoint maps also agree with each other per component.
    Finite-difference geometries are factored eight at a time."""
    import torch
    from dataclasses import replace
    p = W.config4_large()
    rng = np.random.default_rng(1014)
    eps0 = rcp.eps_from_widths(p)
    fac = rcp.Factors(p, eps0)
    F0, g = rcp.adjoint_grad(fac, p)
    gw = rcp.width_grad(p, g).cpu().numpy()
    gd = g.cpu().numpy()
    del fac
    fac32 = rcp.Factors(p, eps0, rcp.RCP_FP32_REFINED)
    F32, g32 = rcp.adjoint_grad(fac32, p)
    gw32 = rcp.width_grad(p, g32).cpu().numpy()
    gd32 = g32.cpu().numpy()
    del fac32
    assert abs(F32.item() - F0.item()) / F0.item() < 1e-6
    assert_grad_close(gd32, gd, 1e-5)
    assert_grad_close(gw32, gw, 1e-5)
    # perturbed geometries: +-dw on each of 20 widths, +-de on each of 20 pixels
    dw, de = 1e-6, 1e-4   # widths: pillar edges stay inside their cells; pixels: smooth in eps
    wsel = rng.choice(len(p.widths), 20, replace=False)
    # the one-sided derivative at a pillar edge needs the perturbed edges to stay
    # inside one cell: no selected edge lies within 10 dw of a cell face
    for k in wsel:
        for edge in (p.pillar_centers[k] - p.widths[k] / 2, p.pillar_centers[k] + p.widths[k] / 2):
            off = edge / p.h - round(edge / p.h)
            assert abs(off) * p.h > 10 * dw, (k, edge)
    i0, i1 = p.aperture
    rows = np.arange(p.sub_rows, p.sub_rows + 200)
    pix = [(int(rng.integers(i0, i1)), int(rng.choice(rows))) for _ in range(20)]
    cases = []
    for k in wsel:
        for sgn in (1, -1):
            w = np.array(p.widths, dtype=np.float64)
            w[k] += sgn * dw
            q = replace(p, widths=tuple(w))
            cases.append((q, rcp.eps_from_widths(q)))
    for (i, j) in pix:
        for sgn in (1, -1):
            e = eps0.clone()
            e[i, j] += sgn * de
            cases.append((p, e))
    F = []
    for b in range(0, len(cases), 8):
        chunk = cases[b:b + 8]
        facs = rcp.factor_batch([c[0] for c in chunk], [c[1] for c in chunk])
        F += [rcp.reciprocal_average(f, c[0]).item() for f, c in zip(facs, chunk)]
        del facs
        torch.cuda.synchronize()
    F = np.array(F)
    fd_w = (F[0:40:2] - F[1:40:2]) / (2 * dw)
    fd_e = (F[40::2] - F[41::2]) / (2 * de)
    for ww, ee in ((gw, gd), (gw32, gd32)):
        assert_grad_close(ww[wsel], fd_w, 1e-5)
        assert_grad_close(np.array([ee[i, j] for i, j in pix]), fd_e, 1e-5)


@pytest.mark.timeout(900)
def test_config2_brute_force_as_benchmarked(rcp):
    """The benchmark's brute force: 1000 Gauss-Legendre nodes over the +-20 deg cone
    as one chunk of 1000 right-hand sides on the config-2 factors (the 1000-row
    multi-RHS sweep).  Per-angle focal intensities on 32 seeded nodes against the
    oracle's forward solves (1e-10), and the quadrature against the reciprocal F
    (converged: 1000 nodes >> K c L / 2 = 164)."""
    p = W.config2()
    eps = rcp.eps_from_widths(p)
    fac = rcp.Factors(p, eps)
    F = rcp.reciprocal_average(fac, p).item()
    Fb, pa = rcp.brute_force_average(fac, 1000, p, rhs_chunk=1000, per_angle=True)
    assert abs(Fb.item() - F) / F < 1e-10
    pa = pa.cpu().numpy()
    th, wt = light.gauss_legendre(p, 1000)
    assert abs(float(np.sum(wt * light.alpha(p, th) * pa)) - Fb.item()) < 1e-12 * F
    del fac
    sub = np.sort(np.random.default_rng(1002).choice(1000, 32, replace=False))
    ref = ora.per_angle_fom(config2_setup(), th[sub])
    assert np.linalg.norm(pa[sub] - ref) / np.linalg.norm(ref) < 1e-10
    assert np.max(np.abs(pa[sub] - ref) / ref) < 1e-9
    assert abs(config2_oracle().F - F) / F < 1e-10
