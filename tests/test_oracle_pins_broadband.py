"""Pins of the oracle's broadband average (no GPU).

The broadband average is a weighted sum over a spectral rule of
single-wavelength reciprocal averages.  It is pinned to:

* the brute-force average of Eq. 6 at every wavelength of the rule (forward
  solves, converged Gauss-Legendre quadrature in angle), summed with the same
  weights: checks that k0 enters the operator, the sources, the objective and
  the correlation consistently at wavelengths other than 1;
* dimensional analysis: with every length measured in wavelengths, the problem
  at wavelength lambda on grid step h is the one at wavelength 1 on step
  h / lambda (operator and sources both scale by lambda^2, so the fields agree;
  the correlation scales by lambda^4 and the reciprocal field by lambda^-2), so
  the two averages are equal;
* a one-point rule, which gives the single-wavelength average;
* central differences of the weighted sum for its gradient.
"""
from dataclasses import replace

import numpy as np

import workloads as W
from oracle import average as ora

SMALL = W.small_problem(4, 4, seed=7)
SMALL_COLL = W.small_problem(5, 4, seed=8, objective=W.COLLIMATOR, light=W.ANNULUS,
                             th1_deg=6.0, th2_deg=25.0, monitor_y=3.0, phi=0.1)


def test_broadband_equals_brute_force_at_every_wavelength():
    for p in (SMALL, SMALL_COLL):
        lams, wts = W.spectral_rule(3, 0.85, 1.15)
        bb = ora.broadband(p, lams, wts)
        Fb = [ora.brute_force(ora.setup(ora.at_wavelength(p, lam)), 64) for lam in lams]
        np.testing.assert_allclose(bb.F, Fb, rtol=1e-10)
        assert abs(bb.total - float(np.dot(wts, Fb))) <= 1e-10 * abs(bb.total)
        # the average does depend on the wavelength
        assert np.ptp(bb.F) > 1e-3 * np.abs(bb.F).max()


def test_broadband_scale_invariance():
    """Wavelength lambda on grid h gives the average of wavelength 1 on grid h / lambda."""
    p = SMALL
    lam = 1.25
    a = ora.reciprocal(ora.setup(ora.at_wavelength(p, lam)))
    q = replace(p, h=p.h / lam, pillar_centers=tuple(c / lam for c in p.pillar_centers),
                widths=tuple(w / lam for w in p.widths))
    b = ora.reciprocal(ora.setup(q))
    assert abs(a - b) <= 1e-10 * abs(b)


def test_broadband_one_point_rule_is_the_single_wavelength_average():
    p = SMALL
    bb = ora.broadband(p, [1.0], [1.0])
    assert abs(bb.total - ora.reciprocal(ora.setup(p))) <= 1e-13 * abs(bb.total)


def test_broadband_gradient_matches_central_differences():
    p = W.small_problem(3, 3, seed=31, npml=8)
    lams, wts = W.spectral_rule(2, 0.9, 1.1)
    bb = ora.broadband(p, lams, wts)

    def total(widths):
        q = replace(p, widths=tuple(widths))
        return sum(w * ora.reciprocal(ora.setup(ora.at_wavelength(q, lam)))
                   for lam, w in zip(lams, wts))

    for k in range(len(p.widths)):
        d = 1e-6
        wp, wm = list(p.widths), list(p.widths)
        wp[k] += d
        wm[k] -= d
        fd = (total(wp) - total(wm)) / (2 * d)
        assert abs(fd - bb.grad_widths[k]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(bb.grad_widths).max())
