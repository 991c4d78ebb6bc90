"""Pins of the 3D vector oracle (Sec. "Concluding remarks": in 3D the
reciprocal average takes one solve per field component the figure of merit
reads -- three for a focal spot, two for an output mode -- and the brute force
runs over two incidence angles and both polarisations).

Checked against what the mathematics fixes: the symmetry of the Yee operator
with its uniaxial PML and the reciprocity of its Green's function, the
three-solve (two-solve) reciprocal form equal to the forward average over a
rule of directions and both polarisations, the divergence-free displacement
field of the curl-curl operator, the geometry of the polarisation vectors, and the absolute scale of the sheet
currents: a full-width s or p sheet radiates one unit of power per unit area to
each side.""" 
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


def _medium(n, h):
    """Uniform index n; the incidence plane 4 cells above the lower PML, two
    physical columns each way (a full-width sheet makes one planewave, so the
    physical region need not be wide); a mild PML grading (R = 1e-3 over 8
    cells) keeps the continued sheet current in the lateral PML moderate."""
    npml = 8
    return W.Problem3D(name="medium3d", nx=2 * npml + 2, ny=2 * npml + 2, nz=2 * npml + 10,
                       npml=npml, h=h, pml_R=1e-3, eps_bg=n * n, eps_sub=n * n, eps_pillar=n * n,
                       sub_layers=0, pillar_k0=0, pillar_layers=0, n_source=n, source_k=npml + 4)


def _complex_coordinate(p, n_axis, xi):
    """h times the integral of the stretch s from the inner edge of the lower PML
    to xi (cell units): the coordinate in which a planewave continues through the
    PML, real on the physical cells."""
    m, L = p.pml_m, p.npml
    sigma = (m + 1) * math.log(1.0 / p.pml_R) / (2.0 * F3.k0(p) * L * p.h)
    lo = np.clip(xi, 0, L)
    hi = np.clip(xi, n_axis - L, n_axis)
    grow = (L / (m + 1)) * (((hi - (n_axis - L)) / L) ** (m + 1) - ((L - lo) / L) ** (m + 1))
    return p.h * (xi + 1j * sigma * grow)


def _full_width_sheet(p, theta, azimuth, pol):
    """The oracle's unit-power sheet current (sheet_amplitudes, polarisations) on
    every cell of the incidence plane, its phase continued through the lateral
    PML in complex coordinates.  In the uniaxial form A = C^T L^-1 C - k^2 eps L
    (L = det S / s_c^2) the unknown is S E and a physical current enters as
    i k (det S / s_c) J_c: s_y s_z for E_x, s_x s_z for E_y."""
    K = p.n_source * F3.k0(p)
    amp = F3.sheet_amplitudes(p, theta)[pol]
    e = F3.polarisations(theta, azimuth)[pol]
    kx, ky = K * math.sin(theta) * math.cos(azimuth), K * math.sin(theta) * math.sin(azimuth)
    I, J = np.meshgrid(np.arange(p.nx), np.arange(p.ny), indexing="ij")
    b = np.zeros(3 * p.n_cells, complex)
    for c in range(2):
        xi = I + (0.5 if c == 0 else 0.0)
        yi = J + (0.5 if c == 1 else 0.0)
        ph = np.exp(1j * (kx * _complex_coordinate(p, p.nx, xi) + ky * _complex_coordinate(p, p.ny, yi)))
        s_other = F3.stretch(p, p.ny, yi) if c == 0 else F3.stretch(p, p.nx, xi)   # s_z = 1 here
        b[F3.index(p, c, I, J, p.source_k).ravel()] = (1j * F3.k0(p) * amp * e[c] / p.h * s_other * ph).ravel()
    return b


def _z_flux(p, E, k):
    """Re(E x conj H)_z per unit area on the physical cells of layer k, H = C E / (i k)
    on the faces at k + 1/2: the term of the discrete energy identity that crosses
    the plane between layers k and k + 1 (E_x with H_y, E_y with H_x at the same x, y)."""
    H = (F3.curl(p) @ E) / (1j * F3.k0(p))
    a = np.arange(p.npml, p.nx - p.npml)
    I, J = np.meshgrid(a, np.arange(p.npml, p.ny - p.npml), indexing="ij")
    Ex, Ey = E[F3.index(p, 0, I, J, k)], E[F3.index(p, 1, I, J, k)]
    Hx, Hy = H[F3.index(p, 0, I, J, k)], H[F3.index(p, 1, I, J, k)]
    return np.real(Ex * np.conj(Hy) - Ey * np.conj(Hx))


def test_3d_sheet_currents_carry_unit_power():
    """Sec. "Reciprocal approach": the sources are unit-power planewaves.  The
    oracle's s and p sheet amplitudes (|J_s| = 2 sqrt(n cos theta), |J_p| =
    2 sqrt(n / cos theta)) on a full-width sheet must send a flux of 1 per unit
    area up and 1 down, in the normalisation of the scalar case, within the
    second-order error of the Yee stencil at K h = 0.24 (measured: 0.1-2.6%).
    A dropped cos theta gives 1.31 at 40 deg, s and p scalings swapped give
    cos^2 theta = 0.59, a dropped sqrt(n) gives 0.67 and a dropped 2 gives 0.25."""
    p = _medium(1.5, 0.025)
    s = F3.Solved3D(p)
    for deg in (0.0, 20.0, 40.0):
        for pol in (0, 1):
            E = s.solve(_full_width_sheet(p, math.radians(deg), 0.6, pol))
            up = _z_flux(p, E, p.source_k + 4)
            down = _z_flux(p, E, p.source_k - 3)
            assert np.ptp(up) < 0.01 * abs(up.mean())          # one planewave
            assert abs(up.mean() - 1.0) < 0.04, (deg, pol, up.mean())
            assert abs(down.mean() + 1.0) < 0.04, (deg, pol, down.mean())


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
