"""Oracle: statistics of the incoherent light.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Incoherent light": the incident light is a superposition of planewaves
with random amplitudes a(theta) (Eq. 1).  For translation-invariant
illumination the amplitudes at different angles are uncorrelated, so only the
mean-square amplitude alpha(theta) = <|a(theta)|^2> matters, and the equivalent
current on the incidence line has a cross-correlation that depends only on
x1 - x2 (Eq. 3 and the paragraph after it).

With the unit-power equivalent source b0(theta) of ``fdfd.planewave_sources``
(current amplitude J(theta) = -2 i k sqrt(n cos theta), spread over one cell of
height h), the discrete correlation matrix on the incidence line is

    T_jl = <b_j conj(b_l)> = C(x_j - x_l),
    C(Delta) = integral over I of alpha(theta) |J(theta)|^2 / h^2
               exp(i K Delta sin theta) d theta,        K = n k.

Readings (the paper's printed forms differ from the exact integrals):

* Eq. 4 prints W = sinc(Delta (2 pi / lambda) sin c) for light uniform in
  theta.  With alpha = 1/(2c) and the unit-power weight |J|^2 proportional to
  cos theta, the substitution sigma = sin theta makes the integral exactly
  sinc-shaped: C = (4 k^2 n / h^2) (sin c / c) sinc(K Delta sin c).  It differs
  from the printed form only by the constant factor sin(c)/c (and K = n k).
* The annulus formula of Sec. "Designs" carries prefactors theta_i; the exact
  integral over [-th2, -th1] u [th1, th2] with alpha = 1/(2 (th2 - th1)) has
  sin(theta_i):  C = (4 k^2 n / h^2) [sin th2 sinc(K D sin th2)
                                      - sin th1 sinc(K D sin th1)] / (th2 - th1).
  The printed form is its small-angle limit (``annulus_paper_printed``).
* Eq. 2 orders a*(theta) a(theta') and the text after Eq. 3 double-counts 1/2c;
  alpha(theta) = <|a|^2> with alpha = 1/(2c) on the cone is used, which keeps
  the total mean power fixed as c varies, as the text says.
* sinc z = sin z / z (unnormalised, sinc 0 = 1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate as si

from workloads import ANNULUS, CONE, Problem
from . import fdfd


def sinc(z):
    """Unnormalised sinc: sin z / z, 1 at z = 0 (numpy's sinc is sin(pi z)/(pi z))."""
    return np.sinc(np.asarray(z, dtype=np.float64) / math.pi)


def intervals(p: Problem):
    """Angular support I of the light as a list of (lo, hi) in radians."""
    if p.light == CONE:
        return [(-p.c, p.c)]
    if p.light == ANNULUS:
        return [(-p.th2, -p.th1), (p.th1, p.th2)]
    raise ValueError("unknown light kind")


def alpha(p: Problem, theta) -> np.ndarray:
    """Mean-square amplitude <|a(theta)|^2>, normalised to unit total."""
    theta = np.asarray(theta, dtype=np.float64)
    total = sum(hi - lo for lo, hi in intervals(p))
    inside = np.zeros(theta.shape, dtype=bool)
    for lo, hi in intervals(p):
        inside |= (theta >= lo) & (theta <= hi)
    return np.where(inside, 1.0 / total, 0.0)


def correlation_closed_form(p: Problem, delta) -> np.ndarray:
    """C(Delta) in closed form for the cone and the annulus (real, even)."""
    delta = np.asarray(delta, dtype=np.float64)
    k = fdfd.k0(p)
    K = p.n_source * k
    pref = 4.0 * k * k * p.n_source / (p.h * p.h)
    if p.light == CONE:
        return pref * (math.sin(p.c) / p.c) * sinc(K * delta * math.sin(p.c))
    if p.light == ANNULUS:
        s1, s2 = math.sin(p.th1), math.sin(p.th2)
        return pref * (s2 * sinc(K * delta * s2) - s1 * sinc(K * delta * s1)) / (p.th2 - p.th1)
    raise ValueError("unknown light kind")


def annulus_paper_printed(p: Problem, delta) -> np.ndarray:
    """The annulus correlation with the printed theta_i prefactors (comparison only)."""
    delta = np.asarray(delta, dtype=np.float64)
    k = fdfd.k0(p)
    K = p.n_source * k
    pref = 4.0 * k * k * p.n_source / (p.h * p.h)
    s1, s2 = math.sin(p.th1), math.sin(p.th2)
    return pref * (p.th2 * sinc(K * delta * s2) - p.th1 * sinc(K * delta * s1)) / (p.th2 - p.th1)


def correlation_quad(p: Problem, delta: float, epsabs: float = 1e-13) -> complex:
    """C(Delta) by adaptive quadrature of its defining integral (any alpha)."""
    k = fdfd.k0(p)
    K = p.n_source * k

    def weight(t):
        J = fdfd.source_amplitude(p, t)
        return float(alpha(p, t)) * abs(complex(J)) ** 2 / (p.h * p.h)

    re = im = 0.0
    for lo, hi in intervals(p):
        re += si.quad(lambda t: weight(t) * math.cos(K * delta * math.sin(t)), lo, hi,
                      epsabs=epsabs, epsrel=1e-13, limit=400)[0]
        im += si.quad(lambda t: weight(t) * math.sin(K * delta * math.sin(t)), lo, hi,
                      epsabs=epsabs, epsrel=1e-13, limit=400)[0]
    return complex(re, im)


def gauss_legendre(p: Problem, n: int):
    """Gauss-Legendre nodes and weights in theta over I (split evenly for an annulus)."""
    ivs = intervals(p)
    per = n // len(ivs)
    if per * len(ivs) != n or per < 1:
        raise ValueError("node count must split evenly over the intervals")
    xs, ws = np.polynomial.legendre.leggauss(per)
    th, wt = [], []
    for lo, hi in ivs:
        th.append(0.5 * (hi - lo) * xs + 0.5 * (hi + lo))
        wt.append(0.5 * (hi - lo) * ws)
    return np.concatenate(th), np.concatenate(wt)


def toeplitz_matrix(p: Problem) -> np.ndarray:
    """T_jl = C(x_j - x_l) on the incidence line (M x M, dense)."""
    i0, i1 = p.aperture
    x = fdfd.x_centres(p)[i0:i1]
    return correlation_closed_form(p, x[:, None] - x[None, :]).astype(np.complex128)


def toeplitz_from_quadrature(p: Problem, thetas, weights) -> np.ndarray:
    """T built from a quadrature rule: sum_q w_q alpha(theta_q) b0_q b0_q^dag on the line."""
    B = fdfd.planewave_line(p, thetas)
    wa = np.asarray(weights) * alpha(p, thetas)
    return (B * wa[None, :]) @ B.conj().T


def ensemble_correlation(p: Problem, thetas, C) -> np.ndarray:
    """W on the incidence line for a finite ensemble of planewaves (Eq. 1 and 3 as sums).

    Light made of planewaves at angles theta_q with random amplitudes a_q,
    C_qq' = <a_q conj(a_q')>, has the equivalent current b = sum_q a_q b0_q, so
    W = <b b^dag> = sum_qq' C_qq' b0_q b0_q'^dag: W_jl = (B C B^dag)_jl with
    column q of B the unit-power source b0(theta_q) on the line.  Any Hermitian
    C is allowed; for C diagonal this is the Toeplitz T of a quadrature rule.
    """
    B = fdfd.planewave_line(p, thetas)
    return B @ np.asarray(C, dtype=np.complex128) @ B.conj().T
