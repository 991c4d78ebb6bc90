"""Pins of the 3D vector oracle (Sec. "Concluding remarks": in 3D the
reciprocal average takes one solve per field component the figure of merit
reads -- three for a focal spot, two for an output mode -- and the brute force
runs over two incidence angles and both polarisations).

Checked against what the mathematics fixes: the symmetry of the Yee operator
with its uniaxial PML and the reciprocity of its Green's function, the
three-solve (two-solve) reciprocal form equal to the forward average over a
rule of directions and both polarisations, the divergence-free displacement
field of the curl-curl operator, and the geometry of the polarisation vectors.
The absolute scale of the 3D sheet currents (unit power) has no pin of its
own here: parity unpinned (the 2D constant of the same derivation is pinned).""" 
import math
from dataclasses import replace
from functools import lru_cache

import numpy as np
import pytest

import workloads as W
from oracle import fdfd3d as F3

CONC = W.metasurface3d("conc3d", 1, 1.5, 31, npml=4, focus_height=0.25, c_deg=20.0)
COLL = W.metasurface3d("coll3d", 1, 1.5, 32, npml=4, objective=W.COLLIMATOR, monitor_y=1.25,
                       c_deg=20.0, out_theta=0.2, out_azimuth=0.7)


@lru_cache(maxsize=None)
def solved(p):
    return F3.Solved3D(p)


def test_3d_operator_is_symmetric_and_reciprocal():
    s = solved(CONC)
    assert abs(s.A - s.A.T).max() == 0.0
    n = s.A.shape[0]
    rng = np.random.default_rng(3)
    for _ in range(4):
        a, b = (int(x) for x in rng.integers(0, n, size=2))     # PML unknowns included
        ea = np.zeros(n, complex)
        eb = np.zeros(n, complex)
        ea[a] = 1.0
        eb[b] = 1.0
        gab = s.solve(ea)[b]
        gba = s.solve(eb)[a]
        assert abs(gab - gba) <= 1e-11 * max(abs(gab), 1e-30)


@pytest.mark.parametrize("p, solves", [(CONC, 3), (COLL, 2)], ids=["focal_spot", "output_mode"])
def test_3d_reciprocal_solves_equal_the_forward_average(p, solves):
    """sum_c v_c^dag W v_c with one solve per component (3 or 2) equals the
    forward average over 2 x 3 x 6 directions, both polarisations each, when W
    is built from the same rule; one polarisation or one component alone is not
    enough."""
    s = solved(p)
    th, az, wt = F3.cone_rule(p, 3, 6)
    Fb = F3.brute_force(s, th, az, wt)
    Wc = F3.correlation_from_rule(p, th, az, wt)
    Z = F3.reciprocal_fields(s)
    assert Z.shape[1] == solves
    Fr = F3.reciprocal(s, Wc)
    assert abs(Fr - Fb) < 1e-11 * Fb
    # the pieces: every component and both polarisations carry part of F
    V = Z[F3.plane_unknowns(p, p.source_k), :]
    parts = [complex(np.vdot(V[:, c], Wc @ V[:, c])).real for c in range(solves)]
    assert min(parts) > 1e-6 * Fb
    idx = F3.plane_unknowns(p, p.source_k)
    B = F3.planewave_sources(p, th, az)[idx, :]
    w_s = np.zeros(B.shape[1])
    w_s[0::2] = wt                       # s polarisation only
    Ws = (B * w_s[None, :]) @ B.conj().T
    Fs = sum(complex(np.vdot(V[:, c], Ws @ V[:, c])).real for c in range(solves))
    assert 0.05 * Fb < Fs < 0.95 * Fb


def test_3d_polarisation_vectors():
    for th, az in ((0.0, 0.3), (0.4, 1.1), (0.7, -2.0)):
        sdir, pdir = F3.polarisations(th, az)
        assert abs(np.dot(sdir, pdir)) < 1e-15
        assert abs(np.linalg.norm(sdir) - 1) < 1e-15 and abs(np.linalg.norm(pdir) - 1) < 1e-15
        assert sdir[2] == 0 and pdir[2] == 0
        # the s current is normal to the plane of incidence
        kpar = np.array([math.cos(az), math.sin(az), 0.0])
        assert abs(np.dot(sdir, kpar)) < 1e-15
    js, jp = F3.sheet_amplitudes(replace(CONC, n_source=1.7), 0.0)
    assert abs(js - jp) < 1e-15       # at normal incidence the two are the same wave
    js, jp = F3.sheet_amplitudes(replace(CONC, n_source=1.7), 0.5)
    assert abs(js * jp - 4 * 1.7) < 1e-12 and abs(jp / js - 1 / math.cos(0.5)) < 1e-12


def test_3d_field_is_divergence_free_away_from_the_source():
    """The Yee curl has no gradient in its range: with E = A^{-1} b,
    div(D_eps eps E) = -div(b) / k^2 cell by cell (backward differences of the
    edge values onto the grid nodes), so the stretched displacement field has
    no divergence wherever b has none -- to roundoff, inside the PML too.  A
    wrong sign or offset in one term of the curl breaks it."""
    p = CONC
    s = solved(p)
    rng = np.random.default_rng(7)
    N = p.n_cells
    b = np.zeros(3 * N, complex)
    hot = rng.choice(3 * N, 5, replace=False)
    b[hot] = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    E = s.solve(b)
    eps = F3.permittivity(p)
    D = [(F3.uniaxial(p, F3.component_positions(p, c), c) * eps[c]).ravel() * E[c * N:(c + 1) * N]
         for c in range(3)]
    Bc = [b[c * N:(c + 1) * N] for c in range(3)]

    def div(F):
        out = np.zeros((p.nx, p.ny, p.nz), complex)
        for c in range(3):
            f = F[c].reshape(p.nx, p.ny, p.nz)
            d = f.copy()
            sl = [slice(None)] * 3
            sl[c] = slice(1, None)
            lo = [slice(None)] * 3
            lo[c] = slice(None, -1)
            d[tuple(sl)] -= f[tuple(lo)]
            out += d / p.h
        return out

    lhs = div(D)
    rhs = -div(Bc) / F3.k0(p) ** 2
    scale = np.abs(lhs).max()
    assert np.abs(lhs - rhs).max() < 1e-9 * scale
    quiet = np.abs(rhs) == 0
    assert quiet.sum() > 0.9 * quiet.size
    assert np.abs(lhs[quiet]).max() < 1e-9 * scale
