"""Pins of the oracle's general-correlation, many-output average (no GPU).

Eq. 7 for a correlation W that is not Toeplitz, and for several outputs on the
same factors, is pinned to facts outside the reciprocal code path:

* the forward (brute-force) form of Eq. 5 for a finite ensemble of correlated
  planewaves, one forward solve per planewave, with a complex Hermitian
  amplitude correlation (a transposed or conjugated C, W or v fails it);
* fully coherent light, where the average is the squared amplitude of one
  deterministic field (one forward solve of the superposed source);
* the uncorrelated limit, where the ensemble W of a Gauss-Legendre rule tends to
  the closed-form Toeplitz correlation (a different formula altogether);
* central finite differences of the summed average for the gradient.
"""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import average as ora
from oracle import fdfd, light

SMALL = W.small_problem(4, 4, seed=7)
SMALL_ANN = W.small_problem(5, 4, seed=8, objective=W.COLLIMATOR, light=W.ANNULUS,
                            th1_deg=6.0, th2_deg=25.0, monitor_y=3.0, phi=0.1)


def outputs_of(p, spots=3, modes=2, seed=3001):
    return W.output_set(p, spots, modes, seed=seed)


@pytest.mark.parametrize("p", [SMALL, SMALL_ANN], ids=["cone", "annulus"])
def test_dense_reciprocal_equals_correlated_brute_force(p):
    """Eq. 7 with the ensemble W equals the ensemble sum of Eq. 5 over forward solves."""
    s = ora.setup(p)
    outs = outputs_of(p)
    th = W.ensemble_angles(p, 24)
    C = W.gaussian_correlated_amplitudes(th, sigma_deg=3.0, tilt=4.0)
    assert np.abs(C - C.T).max() > 1e-3          # complex: C^T != C
    Wm = light.ensemble_correlation(p, th, C)
    assert np.abs(Wm.imag).max() > 1e-2 * np.abs(Wm).max()   # W^T != W as well
    F, V = ora.reciprocal_dense(s, outs, Wm)
    Fb = ora.brute_force_ensemble(s, outs, th, C)
    assert V.shape == (p.m_aperture, len(outs))
    np.testing.assert_allclose(F, Fb, rtol=1e-11, atol=0)
    # a transposed amplitude correlation gives a different average
    Fwrong = ora.brute_force_ensemble(s, outs, th, C.T)
    assert np.abs(Fwrong - Fb).max() > 1e-6 * np.abs(Fb).max()


def test_dense_coherent_light_is_one_deterministic_field():
    """C = a a^dag: the average is |w^dag A^{-1} sum_q a_q b0_q|^2."""
    p = SMALL
    s = ora.setup(p)
    outs = outputs_of(p, 2, 2, seed=3002)
    th = W.ensemble_angles(p, 16)
    a = W.coherent_amplitudes(16, seed=77)
    C = np.outer(a, a.conj())
    F, _ = ora.reciprocal_dense(s, outs, light.ensemble_correlation(p, th, C))
    np.testing.assert_allclose(F, ora.coherent_superposition(s, outs, th, a), rtol=1e-11)


@pytest.mark.parametrize("p", [SMALL, SMALL_ANN], ids=["cone", "annulus"])
def test_dense_uncorrelated_limit_is_the_closed_form_toeplitz(p):
    """Diagonal C on a Gauss-Legendre rule: W -> C(x_j - x_l) of Eq. 4 / the annulus form."""
    th, wt = light.gauss_legendre(p, 400)
    Wm = light.ensemble_correlation(p, th, np.diag(wt * light.alpha(p, th)))
    T = light.toeplitz_matrix(p)
    assert np.abs(Wm - T).max() < 1e-10 * np.abs(T).max()
    # and the many-output average then equals the single-output Toeplitz average
    s = ora.setup(p)
    F, _ = ora.reciprocal_dense(s, [p], T)
    assert abs(F[0] - ora.reciprocal(s)) <= 1e-12 * abs(F[0])


def test_dense_form_of_an_arbitrary_hermitian_matrix_is_real_and_additive():
    """Hermitian W: each v^dag W v is real; W = W1 + W2 splits the averages."""
    p = SMALL
    s = ora.setup(p)
    outs = outputs_of(p, 2, 1, seed=3003)
    W1 = W.random_hermitian(p.m_aperture, seed=91)
    W2 = W.random_hermitian(p.m_aperture, seed=92)
    F1, V = ora.reciprocal_dense(s, outs, W1)
    F2, _ = ora.reciprocal_dense(s, outs, W2)
    F12, _ = ora.reciprocal_dense(s, outs, W1 + W2)
    np.testing.assert_allclose(F12, F1 + F2, rtol=1e-10, atol=1e-12 * np.abs(F12).max())
    for k in range(len(outs)):
        q = np.vdot(V[:, k], W1 @ V[:, k])
        assert abs(q.imag) <= 1e-12 * abs(q)


def test_dense_adjoint_matches_central_differences():
    p = W.small_problem(3, 3, seed=31, npml=8)
    outs = outputs_of(p, 2, 1, seed=3004)
    th = W.ensemble_angles(p, 12)
    C = W.gaussian_correlated_amplitudes(th, sigma_deg=4.0, tilt=2.0)
    Wm = light.ensemble_correlation(p, th, C)
    s = ora.setup(p)
    g = ora.adjoint_dense(s, outs, Wm)
    F0, _ = ora.reciprocal_dense(s, outs, Wm)
    np.testing.assert_allclose(g.F, F0, rtol=1e-12)

    def total(eps):
        return ora.reciprocal_dense(ora.setup(p, eps), outs, Wm)[0].sum()

    rng = np.random.default_rng(1015)
    eps = s.eps
    for _ in range(3):
        i = int(rng.integers(p.npml, p.nx - p.npml))
        j = int(rng.integers(p.pillar_row0, p.pillar_row0 + p.pillar_rows))
        d = 1e-4
        ep, em = eps.copy(), eps.copy()
        ep[i, j] += d
        em[i, j] -= d
        fd = (total(ep) - total(em)) / (2 * d)
        assert abs(fd - g.grad_eps[i, j]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g.grad_eps).max())
    for k in range(len(p.widths)):
        d = 1e-6
        wp, wm = list(p.widths), list(p.widths)
        wp[k] += d
        wm[k] -= d
        fp = ora.reciprocal_dense(ora.setup(replace(p, widths=tuple(wp))), outs, Wm)[0].sum()
        fm = ora.reciprocal_dense(ora.setup(replace(p, widths=tuple(wm))), outs, Wm)[0].sum()
        fd = (fp - fm) / (2 * d)
        assert abs(fd - g.grad_widths[k]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g.grad_widths).max())
