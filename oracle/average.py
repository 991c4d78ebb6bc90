"""Oracle: angle-averaged figure of merit, brute force and reciprocal, and its gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``brute_force``   Eq. 6: integral over theta of alpha(theta) |w^dag u(theta)|^2
                    with u(theta) = A^{-1} b0(theta), one forward solve per
                    Gauss-Legendre node.
* ``reciprocal``    Eq. 7: <|w^dag u|^2> = v^dag W v with v = A^{-dag} w on the
                    incidence line, evaluated as the plain double sum
                    sum_jl conj(v_j) C(x_j - x_l) v_l (no FFT).
* ``adjoint``       gradient of the reciprocal average with respect to the cell
                    permittivities and the pillar widths (Sec. "Reciprocal
                    approach": grad F = 2 Re(v^dag W grad v), with grad v from
                    one adjoint solve).  Reading: the printed
                    grad v = -A^{-dag} grad A^dag v differentiates the full
                    reciprocal field z = A^{-dag} w, then restricts it to the
                    line: grad v = -P A^{-dag} (grad A^dag) z.  With
                    lambda = A^{-1} P^T (W v) and dA = k^2 s_x s_y deps e_q e_q^T
                    this gives dF/deps_q = -2 k^2 Re(conj(lambda_q) conj(s_x s_y) z_q).
* ``reciprocal_dense`` / ``adjoint_dense``
                    Eq. 7 for any Hermitian W (plain dense product) and K outputs
                    w_k on the same factors, and the gradient of sum_k F_k.
* ``brute_force_ensemble``
                    Eq. 5 for a finite ensemble of planewaves with amplitude
                    correlation C_qq': one forward solve per planewave.
* ``broadband``     a weighted sum of single-wavelength averages over a
                    spectral rule, and its gradient.

Because A = A^T, A^{-dag} w = conj(A^{-1} conj(w)): the reciprocal problem is the
forward problem with the conjugated objective as its source (a point source at
the focus for a concentrator, a planewave from the output direction for a
collimator, Sec. "Reciprocal approach").
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from workloads import Problem
from . import fdfd, light


@dataclass
class Solved:
    """Factored operator of one problem (SuperLU) plus what the averages reuse."""

    p: Problem
    eps: np.ndarray
    A: object
    lu: object

    def solve(self, b):
        return self.lu.solve(np.ascontiguousarray(b, dtype=np.complex128))


def setup(p: Problem, eps=None) -> Solved:
    if eps is None:
        eps = fdfd.permittivity(p)
    A = fdfd.operator(p, eps)
    return Solved(p=p, eps=eps, A=A, lu=fdfd.factor(A))


def forward_fields(s: Solved, thetas) -> np.ndarray:
    """u(theta) = A^{-1} b0(theta) for each angle (N x Q)."""
    return s.solve(fdfd.planewave_sources(s.p, thetas))


def per_angle_fom(s: Solved, thetas) -> np.ndarray:
    """|w^dag u(theta)|^2 for each angle (one forward solve per angle)."""
    w = fdfd.objective_vector(s.p)
    U = forward_fields(s, thetas)
    return np.abs(w.conj() @ U) ** 2


def brute_force(s: Solved, n_nodes: int) -> float:
    """Eq. 6 by n-node Gauss-Legendre quadrature in theta over I."""
    th, wt = light.gauss_legendre(s.p, n_nodes)
    return float(np.sum(wt * light.alpha(s.p, th) * per_angle_fom(s, th)))


def reciprocal_field(s: Solved) -> np.ndarray:
    """z = A^{-dag} w = conj(A^{-1} conj(w)) on the whole grid."""
    w = fdfd.objective_vector(s.p)
    return np.conj(s.solve(np.conj(w)))


def line_field(s: Solved, z=None) -> np.ndarray:
    """v = z restricted to the incidence line (physical columns of the source row)."""
    if z is None:
        z = reciprocal_field(s)
    return z[fdfd.aperture_indices(s.p)]


def quadratic_form(v: np.ndarray, T: np.ndarray) -> complex:
    """v^dag T v as the plain double sum."""
    return complex(np.sum(np.conj(v)[:, None] * T * v[None, :]))


def reciprocal(s: Solved, T=None) -> float:
    """Eq. 7 with the closed-form correlation (or a given T): one reciprocal solve."""
    v = line_field(s)
    if T is None:
        T = light.toeplitz_matrix(s.p)
    return quadratic_form(v, T).real


@dataclass
class Gradient:
    F: float
    z: np.ndarray               # reciprocal field, N
    Tv: np.ndarray              # W v on the line, M
    lam: np.ndarray             # adjoint field A^{-1} P^T (W v), N
    grad_eps: np.ndarray        # dF/deps, nx x ny
    grad_widths: np.ndarray     # dF/dw_p, one per pillar


def adjoint(s: Solved) -> Gradient:
    p = s.p
    z = reciprocal_field(s)
    v = line_field(s, z)
    T = light.toeplitz_matrix(p)
    Tv = T @ v
    F = complex(np.vdot(v, Tv)).real
    rhs = np.zeros(p.nx * p.ny, dtype=np.complex128)
    rhs[fdfd.aperture_indices(p)] = Tv
    lam = s.solve(rhs)
    sxc, _, syc, _ = fdfd.stretches(p)
    sxsy = (sxc[:, None] * syc[None, :]).ravel()
    k2 = fdfd.k0(p) ** 2
    g = -2.0 * k2 * np.real(np.conj(lam) * np.conj(sxsy) * z)
    grad_eps = g.reshape(p.nx, p.ny)
    return Gradient(F=F, z=z, Tv=Tv, lam=lam, grad_eps=grad_eps,
                    grad_widths=width_gradient(p, grad_eps))


def edge_cells(p: Problem, centre: float, width: float):
    """Columns holding the left and right pillar edges (half-open cells)."""
    x0 = (0.0 - p.npml) * p.h          # left face of column 0 in physical x
    left = int(np.floor((centre - width / 2 - x0) / p.h))
    right = int(np.floor((centre + width / 2 - x0) / p.h))
    return left, right


def width_gradient(p: Problem, grad_eps: np.ndarray, widths=None) -> np.ndarray:
    """Chain rule eps(widths): each edge moves by dw/2, changing one cell's fill by dw/(2h)."""
    widths = p.widths if widths is None else widths
    rows = slice(p.pillar_row0, p.pillar_row0 + p.pillar_rows)
    d = (p.eps_pillar - p.eps_bg) / (2.0 * p.h)
    out = np.zeros(len(widths))
    for k, (xc, w) in enumerate(zip(p.pillar_centers, widths)):
        il, ir = edge_cells(p, xc, w)
        out[k] = d * (grad_eps[il, rows].sum() + grad_eps[ir, rows].sum())
    return out


# ---------------------------------------------------------------------------
# Any correlation W and many outputs
#
# Eq. 7 holds for any current correlation W (Sec. "Incoherent light": the
# reciprocal technique also covers arbitrarily correlated light), with W v a
# dense product when W is not Toeplitz.  Several outputs w_k (focal spots or
# output modes, Sec. "Concluding remarks": averages over many spots or modes)
# take one reciprocal solve each on the same factors; their averages add up to
# the trace form sum_k v_k^dag W v_k = Tr(V^dag W V).
# ---------------------------------------------------------------------------

def reciprocal_fields(s: Solved, outputs) -> np.ndarray:
    """z_k = A^{-dag} w_k for each output (N x K), one reciprocal solve each."""
    Wo = np.stack([fdfd.objective_vector(o) for o in outputs], axis=1)
    return np.conj(s.solve(np.conj(Wo)))


def reciprocal_dense(s: Solved, outputs, W: np.ndarray):
    """F_k = v_k^dag W v_k (real part; W Hermitian), v_k = z_k on the line.

    Returns (F, V): F has the K per-output averages, V is M x K.
    """
    Z = reciprocal_fields(s, outputs)
    V = Z[fdfd.aperture_indices(s.p), :]
    F = np.array([quadratic_form(V[:, k], W).real for k in range(V.shape[1])])
    return F, V


def brute_force_ensemble(s: Solved, outputs, thetas, C) -> np.ndarray:
    """Eq. 5 for a finite ensemble: F_k = sum_qq' C_qq' (w_k^dag u_q) conj(w_k^dag u_q').

    One forward solve u_q = A^{-1} b0(theta_q) per planewave of the ensemble.
    """
    U = forward_fields(s, thetas)
    C = np.asarray(C, dtype=np.complex128)
    F = []
    for o in outputs:
        g = fdfd.objective_vector(o).conj() @ U
        F.append(np.sum(C * g[:, None] * np.conj(g)[None, :]).real)
    return np.array(F)


def coherent_superposition(s: Solved, outputs, thetas, a) -> np.ndarray:
    """|w_k^dag u|^2 for the deterministic field u = A^{-1} sum_q a_q b0(theta_q)."""
    b = fdfd.planewave_sources(s.p, thetas) @ np.asarray(a, dtype=np.complex128)
    u = s.solve(b)
    return np.array([abs(np.vdot(fdfd.objective_vector(o), u)) ** 2 for o in outputs])


@dataclass
class DenseGradient:
    F: np.ndarray               # per-output averages, K
    V: np.ndarray               # reciprocal fields on the line, M x K
    Y: np.ndarray               # W V, M x K
    grad_eps: np.ndarray        # d(sum_k F_k)/deps, nx x ny
    grad_widths: np.ndarray


def adjoint_dense(s: Solved, outputs, W: np.ndarray) -> DenseGradient:
    """Gradient of sum_k F_k: the single-output adjoint summed over the outputs.

    Per output lambda_k = A^{-1} P^T (W v_k) and
    dF_k/deps_q = -2 k^2 Re(conj(lambda_kq) conj(s_x s_y)_q z_kq).
    """
    p = s.p
    Z = reciprocal_fields(s, outputs)
    idx = fdfd.aperture_indices(p)
    V = Z[idx, :]
    Y = W @ V
    F = np.array([complex(np.vdot(V[:, k], Y[:, k])).real for k in range(V.shape[1])])
    rhs = np.zeros((p.nx * p.ny, V.shape[1]), dtype=np.complex128)
    rhs[idx, :] = Y
    Lam = s.solve(rhs)
    sxc, _, syc, _ = fdfd.stretches(p)
    sxsy = (sxc[:, None] * syc[None, :]).ravel()
    k2 = fdfd.k0(p) ** 2
    g = np.zeros(p.nx * p.ny)
    for k in range(V.shape[1]):
        g += -2.0 * k2 * np.real(np.conj(Lam[:, k]) * np.conj(sxsy) * Z[:, k])
    grad_eps = g.reshape(p.nx, p.ny)
    return DenseGradient(F=F, V=V, Y=Y, grad_eps=grad_eps,
                         grad_widths=width_gradient(p, grad_eps))


# ---------------------------------------------------------------------------
# Broadband
#
# Sec. "Method" notes that the single-wavelength calculation can be repeated at
# several wavelengths for broadband problems, and Sec. "Concluding remarks" that
# the frequency integral is a weighted quadrature over the spectrum.  With a
# rule (lambda_l, w_l) the broadband average is sum_l w_l F(lambda_l), each term
# the reciprocal average of Eq. 7 at that wavelength (k0 = 2 pi / lambda_l in
# the operator, the PML, the sources and the correlation; permittivities do not
# depend on the wavelength), and its gradient is sum_l w_l dF(lambda_l)/deps.
# ---------------------------------------------------------------------------

def at_wavelength(p: Problem, lam: float) -> Problem:
    return replace(p, wavelength=float(lam))


@dataclass
class Broadband:
    F: np.ndarray            # per-wavelength averages
    total: float             # sum_l w_l F_l
    grad_eps: np.ndarray     # sum_l w_l dF_l/deps
    grad_widths: np.ndarray


def broadband(p: Problem, wavelengths, weights) -> Broadband:
    F, g = [], np.zeros((p.nx, p.ny))
    for lam, w in zip(wavelengths, weights):
        gl = adjoint(setup(at_wavelength(p, lam)))
        F.append(gl.F)
        g += w * gl.grad_eps
    F = np.array(F)
    return Broadband(F=F, total=float(np.dot(weights, F)), grad_eps=g,
                     grad_widths=width_gradient(p, g))
