"""Pins of the FP64 CPU oracle to facts outside itself (no GPU).

Each test checks the oracle against something the paper or the mathematics
fixes: the reciprocity identity of Eq. 7 against the quadrature of Eq. 6, the
closed-form correlations against their defining integrals, the 2D Green's
function (i/4) H0(kr), source/receiver reciprocity, the discrete flux balance
of a lossless medium, the discrete planewave dispersion, the unit power of the
planewave sources and the output-mode amplitude of the collimator objective,
symmetry, limits and linearity in the light distribution, central finite
differences for the gradient, and the paper's Gauss-Legendre convergence numbers.
"""
import json
import math
from dataclasses import replace
from pathlib import Path

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sps

import workloads as W
from oracle import average as ora
from oracle import fdfd, light

GOLDEN = json.loads((Path(__file__).parent / "golden" / "paper_numbers.json").read_text())


def vacuum(width_wl, height_wl, h=0.05, npml=20):
    p = W.metasurface("vac", width_wl, height_wl, 0, npml=npml, h=h)
    return replace(p, eps_sub=1.0, eps_pillar=1.0, pillar_centers=(), widths=())


SMALL = W.small_problem(4, 4, seed=7)
SMALL_COLL = W.small_problem(5, 4, seed=8, objective=W.COLLIMATOR, light=W.ANNULUS,
                             th1_deg=6.0, th2_deg=25.0, monitor_y=3.0, phi=0.1)


# -- Eq. 7 vs Eq. 6 -------------------------------------------------------------

@pytest.mark.parametrize("p", [SMALL, SMALL_COLL], ids=["concentrator", "collimator"])
def test_P1_reciprocal_equals_brute_force_same_quadrature(p):
    """Eq. 7: v^dag T v with T built from an N-node rule equals the N-node Eq. 6 sum."""
    s = ora.setup(p)
    for n in (8, 16):
        th, wt = light.gauss_legendre(p, n)
        T = light.toeplitz_from_quadrature(p, th, wt)
        Fr = ora.reciprocal(s, T)
        Fb = ora.brute_force(s, n)
        assert abs(Fr - Fb) / Fb < 1e-12


def test_P1_config1_reciprocal_vs_converged_brute_force():
    """Config 1 (240 x 200): the exact-T reciprocal average is the N -> inf limit of Eq. 6."""
    p = W.config1()
    s = ora.setup(p)
    Fr = ora.reciprocal(s)
    assert abs(ora.brute_force(s, 32) - Fr) / Fr < 1e-12
    assert abs(ora.brute_force(s, 64) - Fr) / Fr < 1e-12


# -- correlation function ----------------------------------------------------------

@pytest.mark.parametrize("kind", ["cone", "annulus"])
def test_P2_closed_form_correlation_matches_integral(kind):
    p = SMALL if kind == "cone" else SMALL_COLL
    for d in (0.0, 0.05, 0.37, 1.3, 4.05):
        cf = float(light.correlation_closed_form(p, d))
        q = light.correlation_quad(p, d)
        assert abs(q.imag) < 1e-9 * abs(cf) + 1e-6
        assert abs(cf - q.real) <= 1e-10 * light.correlation_closed_form(p, 0.0)


def test_P3_total_power_zero_and_coherence_limit():
    p = W.with_light(SMALL, light=W.CONE, c=math.radians(20.0))
    k = fdfd.k0(p)
    K = p.n_source * k
    pref = 4 * k * k * p.n_source / p.h ** 2
    assert abs(light.correlation_closed_form(p, 0.0) - pref * math.sin(p.c) / p.c) < 1e-12 * pref
    d0 = math.pi / (K * math.sin(p.c))
    assert abs(light.correlation_closed_form(p, d0)) < 1e-10 * pref
    # as c -> 90 deg the first zero tends to half the wavelength in the medium
    lim = GOLDEN["coherence_width"]["limit_first_zero_over_wavelength_in_medium"]
    p90 = W.with_light(SMALL, light=W.CONE, c=math.radians(89.999))
    first_zero = math.pi / (K * math.sin(p90.c))
    assert abs(first_zero / (p.wavelength / p.n_source) - lim) < 1e-6


def test_cone_shape_is_the_printed_sinc_and_annulus_small_angle_limit():
    p = W.with_light(SMALL, light=W.CONE, c=math.radians(20.0))
    K = p.n_source * fdfd.k0(p)
    d = np.linspace(-3, 3, 61)
    shape = light.correlation_closed_form(p, d) / light.correlation_closed_form(p, 0.0)
    printed = light.sinc(d * K * math.sin(p.c))
    assert np.max(np.abs(shape - printed)) < 1e-14
    a = GOLDEN["annulus_correlation"]
    pa = W.with_light(SMALL, light=W.ANNULUS, th1=math.radians(a["theta1_deg"]),
                      th2=math.radians(a["theta2_deg"]))
    ours = light.correlation_closed_form(pa, d)
    paper = light.annulus_paper_printed(pa, d)
    rel = np.max(np.abs(ours - paper)) / np.max(np.abs(paper))
    assert 1e-4 < rel < 0.05       # differs, by the sin(theta) vs theta prefactors
    tiny = W.with_light(SMALL, light=W.ANNULUS, th1=1e-3, th2=2e-3)
    r2 = np.max(np.abs(light.correlation_closed_form(tiny, d) - light.annulus_paper_printed(tiny, d)))
    assert r2 / np.max(np.abs(light.annulus_paper_printed(tiny, d))) < 1e-5


def test_P15_toeplitz_hermitian_and_form_real_nonnegative():
    for p in (SMALL, SMALL_COLL):
        T = light.toeplitz_matrix(p)
        assert np.max(np.abs(T - T.conj().T)) == 0.0
        assert np.all(np.linalg.eigvalsh(T) > -1e-8 * np.abs(T).max())
        v = W.complex_normal(p.m_aperture, seed=3)
        f = ora.quadratic_form(v, T)
        assert abs(f.imag) < 1e-10 * abs(f.real) and f.real > 0


# -- operator ------------------------------------------------------------------------

def green_error(h):
    p = vacuum(8, 8, h=h)
    A = fdfd.operator(p)
    lu = fdfd.factor(A)
    ic, jc = p.nx // 2, p.ny // 2
    u = lu.solve(fdfd.point_source(p, ic, jc))
    k = fdfd.k0(p)
    errs = []
    for r in (1.0, 2.0, 3.0):
        di = int(round(r / h))
        G = 0.25j * sps.hankel1(0, k * di * h)
        errs.append(abs(u[fdfd.index(p, ic + di, jc)] - G) / abs(G))
    return np.array(errs)


def test_P4_green_function_matches_hankel():
    """Unit point source in vacuum vs (i/4) H0^(1)(k r): dispersion-limited, second order."""
    e20 = green_error(0.05)
    k, h = 2 * math.pi, 0.05
    bound = 1.2 * (k * h) ** 2 * k * np.array([1.0, 2.0, 3.0]) / 24 + 1e-3
    assert np.all(e20 <= bound), (e20, bound)
    e40 = green_error(0.025)
    ratio = e20 / e40
    assert np.all((ratio > 3.5) & (ratio < 4.5)), ratio


def test_P5_reciprocity_and_symmetry():
    p = SMALL
    A = fdfd.operator(p)
    assert abs(A - A.T).max() == 0.0
    lu = fdfd.factor(A)
    rng = np.random.default_rng(5)
    for _ in range(4):
        a = (int(rng.integers(0, p.nx)), int(rng.integers(0, p.ny)))   # PML cells included
        b = (int(rng.integers(0, p.nx)), int(rng.integers(0, p.ny)))
        ea = np.zeros(p.nx * p.ny, complex)
        eb = np.zeros(p.nx * p.ny, complex)
        ea[fdfd.index(p, *a)] = 1
        eb[fdfd.index(p, *b)] = 1
        gab = lu.solve(ea)[fdfd.index(p, *b)]
        gba = lu.solve(eb)[fdfd.index(p, *a)]
        assert abs(gab - gba) <= 1e-12 * max(abs(gab), 1e-30)


def test_P6_discrete_flux_balance_lossless():
    """Im sum_R conj(u) b = sum over edges leaving R of Im(conj(u_in) u_out) / h^2 (real eps)."""
    p = SMALL
    s = ora.setup(p)
    i0, j0 = p.npml + 30, p.npml + 30
    b = fdfd.point_source(p, i0, j0)
    u = s.solve(b).reshape(p.nx, p.ny)
    B = b.reshape(p.nx, p.ny)
    src = np.imag(np.conj(u[i0, j0]) * B[i0, j0])
    for (a0, a1, c0, c1) in [(i0 - 5, i0 + 6, j0 - 4, j0 + 9), (i0 - 20, i0 + 22, j0 - 25, j0 + 30)]:
        flux = 0.0
        for i in range(a0, a1):
            flux += np.imag(np.conj(u[i, c0]) * u[i, c0 - 1]) + np.imag(np.conj(u[i, c1 - 1]) * u[i, c1])
        for j in range(c0, c1):
            flux += np.imag(np.conj(u[a0, j]) * u[a0 - 1, j]) + np.imag(np.conj(u[a1 - 1, j]) * u[a1, j])
        flux /= p.h ** 2
        assert abs(flux - src) < 1e-11 * abs(src)


@pytest.mark.parametrize("deg,tol", [(0.0, 2e-4), (20.0, 5e-3)])
def test_P7_vacuum_planewave_phase(deg, tol):
    """A full-width line current (stretched phase in the x-PML) makes the discrete planewave."""
    p = vacuum(8, 8)
    A = fdfd.operator(p)
    lu = fdfd.factor(A)
    k, h = fdfd.k0(p), p.h
    kx = k * math.sin(math.radians(deg))
    _, sxf, _, _ = fdfd.stretches(p)
    # complex stretched coordinate at cell centres: integral of s_x from the left edge
    xt = np.concatenate([[0.0], np.cumsum(sxf[1:p.nx] * h)]) + (-p.npml + 0.5) * h
    js = p.npml + 20
    sxc, _, syc, _ = fdfd.stretches(p)
    b = np.zeros(p.nx * p.ny, complex)
    b[fdfd.index(p, np.arange(p.nx), js)] = -sxc * syc[js] * np.exp(1j * kx * xt)   # b = -s_x s_y f
    u = lu.solve(b).reshape(p.nx, p.ny)
    kyt = 2 / h * math.asin(math.sqrt(k ** 2 - 4 * math.sin(kx * h / 2) ** 2 / h ** 2) * h / 2)
    win = u[p.npml + 50:p.nx - p.npml - 50, js + 20:js + 80]
    rx = win[1:, :] / win[:-1, :]
    ry = win[:, 1:] / win[:, :-1]
    assert np.max(np.abs(rx - np.exp(1j * kx * h))) < tol
    assert np.max(np.abs(ry - np.exp(1j * kyt * h))) < tol


# -- absolute scale of the sources and of the collimator mode --------------------------

def uniform_medium(width_wl, height_wl, n, h):
    """A box of uniform index n (no pillars) whose incidence line sits mid-height."""
    p = W.metasurface("medium", width_wl, height_wl, 0, h=h)
    return replace(p, eps_bg=n * n, eps_sub=n * n, eps_pillar=n * n, pillar_centers=(),
                   widths=(), n_source=n, source_row=p.ny // 2)


def radiated_power_per_length(p, theta):
    """Power the aperture source b0(theta) radiates, per unit aperture length.

    By the discrete flux identity (P6) the power leaving every region that holds
    the source is Im sum_c conj(u_c) b_c; times h^2 it is the y-flux
    sum_i Im(conj u_ij u_i,j+1) of a line, and 1/k normalises it so that a
    planewave exp(i k_y y) of amplitude a carries |a|^2 k_y / k per unit length.
    """
    lu = fdfd.factor(fdfd.operator(p))
    b = fdfd.planewave_sources(p, [theta])[:, 0]
    u = lu.solve(b)
    P = p.h ** 2 / fdfd.k0(p) * float(np.sum(np.imag(np.conj(u) * b)))
    return P / (p.m_aperture * p.h)


def finite_aperture_factor(p, theta):
    """Power of a uniform sheet current of length L over that of the same current
    per unit length on an infinite line (continuum, both sides).

    A current J exp(i k_x x) on [0, L] has the spectrum J L sinc((k' - k_x) L / 2);
    each propagating component k' radiates |J(k')|^2 / (4 k k_y(k')) to each side,
    k_y = sqrt(K^2 - k'^2).  The infinite line gives |J|^2 L / (4 k k_y(k_x)) per
    side, so the factor is k_y(k_x) L / (2 pi) * int sinc^2 / k_y(k') dk'.
    """
    K = p.n_source * fdfd.k0(p)
    L = p.m_aperture * p.h
    kx = K * math.sin(theta)
    val, _ = si.quad(lambda kp: np.sinc((kp - kx) * L / (2 * math.pi)) ** 2, -K, K,
                     weight="alg", wvar=(-0.5, -0.5), limit=2000)
    return K * math.cos(theta) * L / (2 * math.pi) * val


@pytest.mark.parametrize("n", [1.5, 2.0])
def test_P16_planewave_sources_carry_unit_power(n):
    """Sec. "Reciprocal approach": the sources are unit-power incident planewaves.

    The aperture source b0(theta) must radiate one unit of power per unit length
    to each side of the incidence line (2 per unit length in all), up to the
    finite-aperture factor of the continuum and the second-order dispersion error
    of the 5-point stencil: |P/2 - factor| <= (K h)^2 / 4, and the error falls ~4x
    when h halves.  A lost factor 2 gives P/2 = 1/4, a lost sqrt(n) gives 1/n and a
    lost cos(theta) gives 1/cos(theta) (1.3 at 40 deg).
    """
    for deg in (0.0, 20.0, 40.0):
        th = math.radians(deg)
        errs = []
        for h in (0.05, 0.025):
            p = uniform_medium(8, 2, n, h)
            ratio = radiated_power_per_length(p, th) / 2.0 / finite_aperture_factor(p, th)
            K = n * fdfd.k0(p)
            assert abs(ratio - 1.0) <= (K * h) ** 2 / 4, (n, deg, h, ratio)
            errs.append(ratio - 1.0)
        assert 3.5 < errs[0] / errs[1] < 4.5, (n, deg, errs)


@pytest.mark.parametrize("sin_phi", [0.1875, 0.3125])
def test_P17_collimator_objective_is_the_output_mode_amplitude(sin_phi):
    """Sec. "Reciprocal approach": the collimator FOM is the overlap of the field
    with the output planewave mode at angle phi.

    A vacuum planewave exp(i k sin(phi) x) is driven by a full-width line current
    with stretched phase through the x-PML (as in P7).  On the monitor row w(phi)^dag u
    must equal the wave's amplitude there (the mean of |u| over the row), and the
    mode of the mirrored angle must not see it: sin(phi) is chosen so that the
    phase 2 k sin(phi) x runs through whole cycles over the aperture.  A flipped
    sign of phi makes |w(phi)^dag u| ~ 0; a lost h / L multiplies it by M.
    """
    phi = math.asin(sin_phi)
    p = W.metasurface("vac", 8, 6, 0, objective=W.COLLIMATOR, phi=phi, monitor_y=3.0)
    p = replace(p, eps_sub=1.0, eps_pillar=1.0, pillar_centers=(), widths=(), n_source=1.0)
    assert abs(2 * fdfd.k0(p) * sin_phi * p.m_aperture * p.h / (2 * math.pi)
               - round(2 * sin_phi * p.m_aperture * p.h)) < 1e-12
    lu = fdfd.factor(fdfd.operator(p))
    k, h = fdfd.k0(p), p.h
    kx = k * sin_phi
    sxc, sxf, syc, _ = fdfd.stretches(p)
    xt = np.concatenate([[0.0], np.cumsum(sxf[1:p.nx] * h)]) + (-p.npml + 0.5) * h
    js = p.npml + 20
    b = np.zeros(p.nx * p.ny, complex)
    b[fdfd.index(p, np.arange(p.nx), js)] = -sxc * syc[js] * np.exp(1j * kx * xt)
    u = lu.solve(b)
    i0, i1 = p.aperture
    amp = np.abs(u.reshape(p.nx, p.ny)[i0:i1, p.monitor_row]).mean()
    a_plus = abs(np.vdot(fdfd.objective_vector(p), u))
    a_minus = abs(np.vdot(fdfd.objective_vector(replace(p, phi=-phi)), u))
    assert abs(a_plus - amp) < 5e-3 * amp, (a_plus, amp)
    assert a_minus < 1e-2 * amp, (a_minus, amp)


# -- symmetry, limits, linearity -------------------------------------------------------

def test_P12_mirror_symmetry():
    p = W.small_problem(4, 4, seed=21)
    s = ora.setup(p)
    F = ora.reciprocal(s)
    pm = replace(p, widths=tuple(reversed(p.widths)), focus=(p.nx - 1 - p.focus[0], p.focus[1]))
    Fm = ora.reciprocal(ora.setup(pm))
    assert abs(F - Fm) / F < 1e-11


def test_P13_single_angle_limit():
    c = 1e-3
    p = W.with_light(SMALL, light=W.CONE, c=c)
    s = ora.setup(p)
    F = ora.reciprocal(s)
    F0 = float(ora.per_angle_fom(s, [0.0])[0])
    assert abs(F - F0) / F0 < 50 * c * c


def test_P14_linearity_in_the_distribution():
    t1, t2 = math.radians(7.0), math.radians(23.0)
    s = ora.setup(SMALL)
    Fa = ora.reciprocal(s, light.toeplitz_matrix(W.with_light(SMALL, light=W.ANNULUS, th1=t1, th2=t2)))
    F1 = ora.reciprocal(s, light.toeplitz_matrix(W.with_light(SMALL, light=W.CONE, c=t1)))
    F2 = ora.reciprocal(s, light.toeplitz_matrix(W.with_light(SMALL, light=W.CONE, c=t2)))
    assert abs((t2 - t1) * Fa - (t2 * F2 - t1 * F1)) < 1e-12 * t2 * F2


def test_P8_gl_convergence_config1():
    p = W.config1()
    s = ora.setup(p)
    Fr = ora.reciprocal(s)
    # converged once N exceeds about K c L / 2 (8.2 here)
    assert abs(ora.brute_force(s, 4) - Fr) / Fr > 1e-6
    assert abs(ora.brute_force(s, 24) - Fr) / Fr < 1e-11


def test_P8_paper_scale_gl_threshold():
    """Paper: 512 GL nodes do not resolve the +-20 deg average over 10^3 cells; 1024 do."""
    g = GOLDEN["gl_convergence"]
    n_s = math.sqrt(g["substrate_eps"])
    h = 0.1
    npml = 2
    nxp = int(round(g["aperture_wavelengths"] / h))
    p = replace(vacuum(1, 1, h=h, npml=npml), nx=nxp + 2 * npml, ny=2 * npml + 2,
                source_row=npml, n_source=n_s, light=W.CONE, c=math.radians(g["cone_deg"]))
    x = fdfd.x_centres(p)[p.npml:p.nx - p.npml]
    f = 0.5 * x[-1] / math.tan(math.asin(0.3))              # an NA 0.3 lens-like field
    v = np.exp(1j * n_s * fdfd.k0(p) * np.sqrt((x - x.mean()) ** 2 + f ** 2))
    line = fdfd.aperture_indices(p)

    def F(n):
        th, wt = light.gauss_legendre(p, n)
        tot = 0.0
        for a in range(0, n, 256):
            B = fdfd.planewave_sources(p, th[a:a + 256])[line, :]
            tot += np.sum(wt[a:a + 256] * light.alpha(p, th[a:a + 256]) * np.abs(v.conj() @ B) ** 2)
        return tot

    ref = F(3072)
    e_bad = abs(F(g["n_not_converged"]) - ref) / ref
    e_good = abs(F(g["n_converged"]) - ref) / ref
    assert e_good < g["threshold"] and e_good < 1e-9
    assert e_bad > 100 * e_good and e_bad > 1e-4


# -- gradient ----------------------------------------------------------------------------

def test_P11_adjoint_matches_central_differences():
    p = W.small_problem(3, 3, seed=31, npml=8)
    s = ora.setup(p)
    g = ora.adjoint(s)
    eps = s.eps
    rng = np.random.default_rng(1014)
    for _ in range(3):
        i = int(rng.integers(p.npml, p.nx - p.npml))
        j = int(rng.integers(p.pillar_row0, p.pillar_row0 + p.pillar_rows))
        d = 1e-4
        ep, em = eps.copy(), eps.copy()
        ep[i, j] += d
        em[i, j] -= d
        fd = (ora.reciprocal(ora.setup(p, ep)) - ora.reciprocal(ora.setup(p, em))) / (2 * d)
        assert abs(fd - g.grad_eps[i, j]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g.grad_eps).max())
    for k in range(len(p.widths)):
        d = 1e-6
        wp = list(p.widths)
        wm = list(p.widths)
        wp[k] += d
        wm[k] -= d
        fp = ora.reciprocal(ora.setup(replace(p, widths=tuple(wp))))
        fm = ora.reciprocal(ora.setup(replace(p, widths=tuple(wm))))
        fd = (fp - fm) / (2 * d)
        assert abs(fd - g.grad_widths[k]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g.grad_widths).max())


def test_permittivity_map_fill_fractions():
    p = W.small_problem(4, 4, seed=7)
    eps = fdfd.permittivity(p)
    rows = slice(p.pillar_row0, p.pillar_row0 + p.pillar_rows)
    # total pillar area per row equals the sum of widths (cells are fully inside the domain)
    fill = (eps[:, p.pillar_row0] - p.eps_bg) / (p.eps_pillar - p.eps_bg)
    assert abs(fill.sum() * p.h - sum(p.widths)) < 1e-12
    assert np.all(eps[:, :p.sub_rows] == p.eps_sub)
    assert np.all(eps[:, p.pillar_row0 + p.pillar_rows:] == p.eps_bg)
    assert np.all(np.ptp(eps[:, rows], axis=1) == 0)
