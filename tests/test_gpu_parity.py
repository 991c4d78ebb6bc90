"""GPU path (librecip through its C ABI) against the FP64 CPU oracle.

Tolerances: FP64 path 1e-10 relative on fields and averages; refined FP32 path
1e-8 on fields and 1e-6 on averages; gradients 1e-5 relative (the FP64 path is
held to 1e-9).
"""
from functools import lru_cache

import numpy as np
import pytest

import workloads as W
from gradcheck import assert_grad_close
from oracle import average as ora
from oracle import fdfd, light

pytestmark = pytest.mark.gpu


@lru_cache(maxsize=None)
def oracle_setup(p):
    return ora.setup(p)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def gpu_factors(rcp, p, precision=None):
    import torch
    precision = rcp.RCP_FP64 if precision is None else precision
    eps = rcp.eps_from_widths(p, device="cuda")
    fac = rcp.Factors(p, eps, precision)
    torch.cuda.synchronize()
    return fac, eps


PROBLEMS = {
    "conc_cone": W.small_problem(4, 4, seed=7),
    "coll_annulus": W.small_problem(5, 4, seed=8, objective=W.COLLIMATOR, light=W.ANNULUS,
                                    th1_deg=6.0, th2_deg=25.0, monitor_y=3.0, phi=0.1),
    "conc_odd": W.small_problem(3, 5, seed=9, npml=8, c_deg=30.0),
    # 276 rows: nine 32-row tiles with a ragged last one, so each wave of the
    # vector sweep takes two tiles
    "conc_tall": W.small_problem(2, 13, seed=10, npml=8, focus_height=9.0),
    # 696 rows: 22 tiles per edge (a ragged last one), above the size where the
    # vector sweep switches from the one-launch product to the tile-once
    # product with its per-tile shares and row sums
    "conc_tile_once": W.small_problem(2, 34, seed=12, npml=8, focus_height=25.0),
}


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_eps_map_matches_oracle(rcp, name):
    p = PROBLEMS[name]
    eps = rcp.eps_from_widths(p, device="cuda").cpu().numpy()
    ref = fdfd.permittivity(p)
    assert np.max(np.abs(eps - ref)) < 1e-12


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_solve_fp64_matches_superlu(rcp, name):
    import torch
    p = PROBLEMS[name]
    fac, _ = gpu_factors(rcp, p)
    s = oracle_setup(p)
    B = W.complex_normal((3, p.nx * p.ny), seed=11)
    X, _ = rcp.solve(fac, torch.from_numpy(B.reshape(3, p.nx, p.ny)).cuda())
    ref = s.solve(B.T).T
    assert rel(X.cpu().numpy().reshape(3, -1), ref) < 1e-10
    # conjugate-transpose solve: A^{-dag} b = conj(A^{-1} conj b)
    Xc, _ = rcp.solve(fac, torch.from_numpy(B[:1].reshape(1, p.nx, p.ny)).cuda(),
                      conj_transpose=True)
    refc = np.conj(s.solve(np.conj(B[0])))
    assert rel(Xc.cpu().numpy().ravel(), refc) < 1e-10


def test_solve_multi_rhs_gemm_path(rcp):
    import torch
    p = PROBLEMS["conc_cone"]
    fac, _ = gpu_factors(rcp, p)
    s = oracle_setup(p)
    R = 70                       # several 64-row tiles with a ragged tail
    B = W.complex_normal((R, p.nx * p.ny), seed=12)
    X, _ = rcp.solve(fac, torch.from_numpy(B.reshape(R, p.nx, p.ny)).cuda())
    ref = s.solve(B.T).T
    assert rel(X.cpu().numpy().reshape(R, -1), ref) < 1e-10


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_reciprocal_average_fp64(rcp, name):
    p = PROBLEMS[name]
    fac, _ = gpu_factors(rcp, p)
    F, v, z = rcp.reciprocal_average(fac, p, want_v=True, want_z=True)
    s = oracle_setup(p)
    z_ref = ora.reciprocal_field(s)
    F_ref = ora.reciprocal(s)
    assert rel(z.cpu().numpy().ravel(), z_ref) < 1e-10
    assert rel(v.cpu().numpy(), ora.line_field(s, z_ref)) < 1e-10
    assert abs(F.item() - F_ref) / abs(F_ref) < 1e-10


@pytest.mark.parametrize("name", ["conc_cone", "coll_annulus"])
def test_brute_force_fp64(rcp, name):
    p = PROBLEMS[name]
    fac, _ = gpu_factors(rcp, p)
    s = oracle_setup(p)
    n = 24
    F, pa = rcp.brute_force_average(fac, n, p, rhs_chunk=10, per_angle=True)
    th, wt = light.gauss_legendre(p, n)
    pa_ref = ora.per_angle_fom(s, th)
    assert rel(pa.cpu().numpy(), pa_ref) < 1e-10
    F_ref = float(np.sum(wt * light.alpha(p, th) * pa_ref))
    assert abs(F.item() - F_ref) / F_ref < 1e-10


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_adjoint_fp64(rcp, name):
    p = PROBLEMS[name]
    fac, _ = gpu_factors(rcp, p)
    F, g = rcp.adjoint_grad(fac, p)
    ref = ora.adjoint(oracle_setup(p))
    assert abs(F.item() - ref.F) / abs(ref.F) < 1e-10
    assert_grad_close(g.cpu().numpy(), ref.grad_eps, 1e-9)
    gw = rcp.width_grad(p, g)
    assert_grad_close(gw.cpu().numpy(), ref.grad_widths, 1e-9)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_refined_fp32_vs_fp64(rcp, name):
    p = PROBLEMS[name]
    f64, _ = gpu_factors(rcp, p)
    f32, _ = gpu_factors(rcp, p, rcp.RCP_FP32_REFINED)
    F64, z64 = rcp.reciprocal_average(f64, p, want_z=True)
    F32, z32 = rcp.reciprocal_average(f32, p, want_z=True)
    iters, res = f32.last_solve_stats()
    assert iters >= 1
    assert rel(z32.cpu().numpy(), z64.cpu().numpy()) < 1e-8
    assert abs(F32.item() - F64.item()) / F64.item() < 1e-6
    Fa, ga = rcp.adjoint_grad(f32, p)
    Fb, gb = rcp.adjoint_grad(f64, p)
    assert rel(ga.cpu().numpy(), gb.cpu().numpy()) < 1e-5


def test_factor_batch_matches_single_and_oracle(rcp):
    """Geometries factored side by side (two panels per pass) agree with one at a
    time (one panel per launch) to rounding, and with the oracle."""
    import torch
    from dataclasses import replace
    base = PROBLEMS["conc_cone"]
    probs = [replace(base, widths=W.seeded_widths(len(base.widths), 300 + g)) for g in range(3)]
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps)
    Fb = [rcp.reciprocal_average(f, p).item() for f, p in zip(facs, probs)]
    for p, e, fb in zip(probs, eps, Fb):
        single = rcp.Factors(p, e)
        Fs = rcp.reciprocal_average(single, p).item()
        assert abs(Fs - fb) <= 1e-12 * abs(Fs)
        ref = ora.reciprocal(oracle_setup(p))
        assert abs(fb - ref) / ref < 1e-10
    torch.cuda.synchronize()


@pytest.mark.parametrize("count", [5, 8])
def test_factor_batch_up_to_eight_geometries(rcp, count):
    """Ten chains (plain workgroup split) and sixteen (two chains per XCD) in one
    launch.  Batches take two panels per pass: every geometry is bit-identical to
    its factorisation in a batch of two, and agrees with the one-panel-per-launch
    factorisation of a lone geometry and with the oracle."""
    import torch
    from dataclasses import replace
    base = PROBLEMS["conc_cone"]
    probs = [replace(base, widths=W.seeded_widths(len(base.widths), 400 + g)) for g in range(count)]
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps)
    Fb = [rcp.reciprocal_average(f, p).item() for f, p in zip(facs, probs)]
    for g in (0, count // 2, count - 1):
        other = (g + 1) % count
        pair = rcp.factor_batch([probs[g], probs[other]], [eps[g], eps[other]])
        assert rcp.reciprocal_average(pair[0], probs[g]).item() == Fb[g]
        single = rcp.Factors(probs[g], eps[g])
        Fs = rcp.reciprocal_average(single, probs[g]).item()
        assert abs(Fs - Fb[g]) <= 1e-12 * abs(Fs)
        ref = ora.reciprocal(oracle_setup(probs[g]))
        assert abs(Fb[g] - ref) / ref < 1e-10
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["conc_cone", "conc_tall"])
def test_factor_pairs_match_oracle_solves(rcp, name):
    """Two-panel passes (even and odd tile counts: 4 and 9 tiles per block edge):
    plain and conjugate-transpose solves of a batch against SuperLU."""
    import torch
    from dataclasses import replace
    p = PROBLEMS[name]
    probs = [p, replace(p, widths=W.seeded_widths(len(p.widths), 77))]
    eps = [rcp.eps_from_widths(q, device="cuda") for q in probs]
    facs = rcp.factor_batch(probs, eps)
    s = oracle_setup(p)
    B = W.complex_normal((3, p.nx * p.ny), seed=12)
    X, _ = rcp.solve(facs[0], torch.from_numpy(B.reshape(3, p.nx, p.ny)).cuda())
    assert rel(X.cpu().numpy().reshape(3, -1), s.solve(B.T).T) < 1e-10
    Xc, _ = rcp.solve(facs[0], torch.from_numpy(B[:1].reshape(1, p.nx, p.ny)).cuda(),
                      conj_transpose=True)
    ref = np.conj(s.solve(np.conj(B[0])))
    assert rel(Xc.cpu().numpy().ravel(), ref) < 1e-10


@pytest.mark.parametrize("height,npml,focus", [(2, 4, 0.3), (3, 8, 1.0)], ids=["2-tiles", "3-tiles"])
def test_factor_batch_smallest_tile_counts(rcp, height, npml, focus):
    """Blocks of two and three 32-row tiles: the block-opening pass is followed at
    once by the last pass (two), or by a pass whose look-ahead forms the odd last
    panel for the one-panel final update (three).  Against the oracle and the
    one-panel-per-launch factorisation of each geometry."""
    from dataclasses import replace
    base = W.small_problem(3, height, seed=41, npml=npml, focus_height=focus)
    assert (base.ny + 31) // 32 == height
    probs = [replace(base, widths=W.seeded_widths(len(base.widths), 800 + g)) for g in range(3)]
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps)
    for p, e, f in zip(probs, eps, facs):
        Fb = rcp.reciprocal_average(f, p).item()
        Fs = rcp.reciprocal_average(rcp.Factors(p, e), p).item()
        assert abs(Fs - Fb) <= 1e-12 * abs(Fs)
        ref = ora.reciprocal(oracle_setup(p))
        assert abs(Fb - ref) / ref < 1e-10


@pytest.mark.parametrize("count", [3, 8])
def test_adjoint_batch_matches_single(rcp, count):
    """Batched adjoint (solves of all sets in the same launches) is bit-identical
    to one adjoint per factor set; mixed objectives and lights in one batch."""
    from dataclasses import replace
    base = PROBLEMS["conc_cone"]
    probs = [replace(base, widths=W.seeded_widths(len(base.widths), 500 + g),
                     c=base.c * (1.0 + 0.1 * g)) for g in range(count)]
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps)
    Fb, gb = rcp.adjoint_grad_batch(facs, probs)
    for g in range(count):
        F1, g1 = rcp.adjoint_grad(facs[g], probs[g])
        assert Fb[g].item() == F1.item()
        assert torch_equal(gb[g], g1)
    ref = ora.adjoint(oracle_setup(probs[-1]))
    assert abs(Fb[-1].item() - ref.F) / abs(ref.F) < 1e-10
    assert_grad_close(gb[-1].cpu().numpy(), ref.grad_eps, 1e-9)


def test_adjoint_batch_tile_once_product(rcp):
    """Batched solves on blocks of 22 tiles (the tile-once product, sixteen jobs
    per launch at eight sets) equal one adjoint per set bit for bit and match
    the oracle."""
    from dataclasses import replace
    base = PROBLEMS["conc_tile_once"]
    probs = [replace(base, widths=W.seeded_widths(len(base.widths), 700 + g)) for g in range(8)]
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps)
    Fb, gb = rcp.adjoint_grad_batch(facs, probs)
    for g in (0, 7):
        F1, g1 = rcp.adjoint_grad(facs[g], probs[g])
        assert Fb[g].item() == F1.item()
        assert torch_equal(gb[g], g1)
        ref = ora.adjoint(oracle_setup(probs[g]))
        assert abs(Fb[g].item() - ref.F) / abs(ref.F) < 1e-10
        assert_grad_close(gb[g].cpu().numpy(), ref.grad_eps, 1e-9)


def test_adjoint_batch_refined_fp32_falls_back_per_set(rcp):
    base = PROBLEMS["coll_annulus"]
    from dataclasses import replace
    probs = [replace(base, widths=W.seeded_widths(len(base.widths), 600 + g)) for g in range(2)]
    eps = [rcp.eps_from_widths(p, device="cuda") for p in probs]
    facs = rcp.factor_batch(probs, eps, rcp.RCP_FP32_REFINED)
    Fb, gb = rcp.adjoint_grad_batch(facs, probs)
    for g in range(2):
        F1, g1 = rcp.adjoint_grad(facs[g], probs[g])
        assert Fb[g].item() == F1.item()
        assert torch_equal(gb[g], g1)


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))
