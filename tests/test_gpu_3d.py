"""The 3D GPU path (Yee operator, block elimination over x-slices with sparse
couplings, one reciprocal solve per field component) against the 3D oracle."""
from functools import lru_cache

import numpy as np
import pytest

import workloads as W
from oracle import fdfd3d as F3

pytestmark = pytest.mark.gpu

CONC = W.metasurface3d("conc3d", 1, 1.5, 31, npml=4, focus_height=0.25, c_deg=20.0)
COLL = W.metasurface3d("coll3d", 1, 1.5, 32, npml=4, objective=W.COLLIMATOR, monitor_y=1.25,
                       c_deg=20.0, out_theta=0.2, out_azimuth=0.7)


@lru_cache(maxsize=None)
def oracle(p):
    return F3.Solved3D(p)


def to_slices(p, x):
    """Oracle ordering (component, i, j, k) -> slice ordering (i, component, j, k)."""
    return np.ascontiguousarray(np.asarray(x).reshape(3, p.nx, p.ny, p.nz).transpose(1, 0, 2, 3))


def gpu_factors(p):
    from paper_2207_10701_amd import maxwell3d as M
    eps = M.eps_from_pillars(p)
    return M, eps, M.Factors3D(p, eps)


def test_3d_permittivity_matches_oracle(rcp):
    from paper_2207_10701_amd import maxwell3d as M
    for p in (CONC, COLL):
        eps = M.eps_from_pillars(p).cpu().numpy()
        ref = to_slices(p, np.concatenate([e.ravel() for e in F3.permittivity(p)]))
        assert np.max(np.abs(eps - ref)) < 1e-13


@pytest.mark.parametrize("conj", [False, True])
def test_3d_solve_matches_superlu(rcp, conj):
    import torch
    p = CONC
    M, eps, fac = gpu_factors(p)
    s = oracle(p)
    N3 = 3 * p.n_cells
    b = W.complex_normal(N3, seed=9)
    x_ref = np.conj(s.solve(np.conj(b))) if conj else s.solve(b)
    x = M.solve(fac, torch.from_numpy(to_slices(p, b)).cuda(), conj_transpose=conj)
    xg = x.cpu().numpy()
    xr = to_slices(p, x_ref)
    assert np.linalg.norm(xg - xr) / np.linalg.norm(xr) < 1e-10


@pytest.mark.parametrize("p, solves", [(CONC, 3), (COLL, 2)], ids=["focal_spot", "output_mode"])
def test_3d_reciprocal_average_matches_oracle_and_brute_force(rcp, p, solves):
    """Three (two) reciprocal solves on the GPU give the oracle's sum_c v_c^dag W v_c
    and the GPU's own forward average over the same 18 directions and both
    polarisations (36 solves); per direction and polarisation the forward values
    match the oracle's."""
    M, eps, fac = gpu_factors(p)
    th, az, wt = W.cone_directions3d(p, 3, 6)
    dirs = M.directions(th, az, wt)
    F = M.reciprocal_average(fac, dirs).item()
    Fb, per = M.brute_force_average(fac, dirs, per=True)
    s = oracle(p)
    Fo = F3.reciprocal(s, F3.correlation_from_rule(p, th, az, wt))
    assert abs(F - Fo) / Fo < 1e-10
    assert abs(Fb.item() - F) / F < 1e-10
    B = F3.planewave_sources(p, th, az)
    E = s.solve(B)
    Wm = F3.objective_vectors(p)
    per_ref = (np.abs(Wm.conj().T @ E) ** 2).sum(axis=0)
    pg = per.cpu().numpy()
    assert np.linalg.norm(pg - per_ref) / np.linalg.norm(per_ref) < 1e-10


def test_3d_argument_errors(rcp):
    import torch
    from dataclasses import replace
    from paper_2207_10701_amd import RecipError
    from paper_2207_10701_amd import maxwell3d as M
    bad = replace(CONC, ny=2, nz=5)                      # 3 ny nz = 30: one tile
    with pytest.raises(RecipError):
        M.Factors3D(bad, torch.ones((bad.nx, 3, bad.ny, bad.nz), dtype=torch.float64, device="cuda"))
    M_, eps, fac = gpu_factors(CONC)
    th, az, wt = W.cone_directions3d(CONC, 2, 3)
    outside = replace(CONC, focus=(1, 1, 1))             # in the PML
    with pytest.raises(RecipError):
        M.reciprocal_average(fac, M.directions(th, az, wt), outside)


def test_3d_wrappers_on_a_side_stream(rcp):
    """Called with a stream outside any stream context, the 3D wrappers
    allocate their temporaries on that stream: the same F as on the default
    stream."""
    import torch
    from paper_2207_10701_amd import maxwell3d as M
    p = COLL
    th, az, wt = W.cone_directions3d(p, 2, 4)
    dirs = M.directions(th, az, wt)
    fac = M.Factors3D(p, M.eps_from_pillars(p))
    F0 = M.reciprocal_average(fac, dirs).item()
    s = torch.cuda.Stream()
    eps = M.eps_from_pillars(p, stream=s)
    fac2 = M.Factors3D(p, eps, stream=s)
    F = M.reciprocal_average(fac2, dirs, stream=s)
    s.synchronize()
    assert F.item() == F0
