"""Oracle: FDFD discretisation of the 2D scalar Helmholtz problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper writes the scattered field as u = A^{-1} b, with A "the Maxwell's
equations operator" and b a current source, and notes that A may be a matrix
from a finite-difference discretisation (Sec. "Reciprocal approach").  The
paper's own solver is an approximate locally-periodic one; here A is the
finite-difference operator of the continuous equation

    (1/s_x) d/dx (1/s_x du/dx) + (1/s_y) d/dy (1/s_y du/dy) + k^2 eps u = -f

(time dependence exp(-i omega t), outgoing waves exp(+i k r)), multiplied
through by s_x s_y so that the discrete matrix is complex *symmetric*:

    A u = b,   b = -s_x s_y f.

Every function follows that definition directly; nothing is blocked or fused.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import COLLIMATOR, CONCENTRATOR, Problem


def k0(p: Problem) -> float:
    return 2.0 * math.pi / p.wavelength


def x_centres(p: Problem) -> np.ndarray:
    """x of cell centres, origin at the left edge of the physical region."""
    return (np.arange(p.nx) - p.npml + 0.5) * p.h


def y_centres(p: Problem) -> np.ndarray:
    return (np.arange(p.ny) - p.npml + 0.5) * p.h


def pml_stretch(p: Problem, n_axis: int, xi: np.ndarray) -> np.ndarray:
    """Stretch factor s(xi) = 1 + i sigma (d/L)^m at grid positions xi (cell units).

    d is the depth into the PML (0 in the interior), L = npml h its thickness
    and sigma = (m+1) ln(1/R) / (2 k L) gives a normal-incidence round-trip
    reflection R for the continuous profile.
    """
    L = p.npml * p.h
    depth = np.maximum(np.maximum(p.npml - xi, xi - (n_axis - p.npml)), 0.0) * p.h
    sigma = (p.pml_m + 1) * math.log(1.0 / p.pml_R) / (2.0 * k0(p) * L)
    return 1.0 + 1j * sigma * (depth / L) ** p.pml_m


def stretches(p: Problem):
    """(s_x at centres, s_x at faces 0..nx, s_y at centres, s_y at faces 0..ny)."""
    sxc = pml_stretch(p, p.nx, np.arange(p.nx) + 0.5)
    sxf = pml_stretch(p, p.nx, np.arange(p.nx + 1).astype(float))
    syc = pml_stretch(p, p.ny, np.arange(p.ny) + 0.5)
    syf = pml_stretch(p, p.ny, np.arange(p.ny + 1).astype(float))
    return sxc, sxf, syc, syf


def overlap_fraction(p: Problem, centre: float, width: float) -> np.ndarray:
    """Fraction of each cell [x_i - h/2, x_i + h/2) covered by [centre -/+ width/2]."""
    x = x_centres(p)
    lo = np.maximum(x - p.h / 2, centre - width / 2)
    hi = np.minimum(x + p.h / 2, centre + width / 2)
    return np.clip(hi - lo, 0.0, None) / p.h


def permittivity(p: Problem, widths=None) -> np.ndarray:
    """Cell permittivity eps[i, j] (nx x ny, float64).

    Background eps_bg everywhere, substrate eps_sub in rows j < sub_rows (all x),
    and in the pillar-layer rows the arithmetic mean of eps over each cell's x
    extent (the exact cell average for the TM field, which is tangential to the
    vertical pillar walls).
    """
    widths = p.widths if widths is None else widths
    eps = np.full((p.nx, p.ny), p.eps_bg, dtype=np.float64)
    eps[:, : p.sub_rows] = p.eps_sub
    frac = np.zeros(p.nx)
    for xc, w in zip(p.pillar_centers, widths):
        frac += overlap_fraction(p, xc, w)
    rows = slice(p.pillar_row0, p.pillar_row0 + p.pillar_rows)
    eps[:, rows] = p.eps_bg + (p.eps_pillar - p.eps_bg) * frac[:, None]
    return eps


def index(p: Problem, i, j):
    """Unknown index q = i * ny + j (x-major: column i is a contiguous block)."""
    return np.asarray(i) * p.ny + np.asarray(j)


def operator(p: Problem, eps=None) -> sp.csc_matrix:
    """The symmetric 5-point PML operator A (N x N complex128, CSC).

    Row q = (i, j):
      coupling to (i+-1, j) = s_y(j) / (s_x(face between the two cells) h^2)
      coupling to (i, j+-1) = s_x(i) / (s_y(face between the two cells) h^2)
      diagonal              = -(sum of the four couplings, boundary faces
                               included) + k^2 eps_ij s_x(i) s_y(j)
    Neighbours outside the grid are dropped (u = 0 there).
    """
    if eps is None:
        eps = permittivity(p)
    sxc, sxf, syc, syf = stretches(p)
    h2 = p.h * p.h
    I, J = np.meshgrid(np.arange(p.nx), np.arange(p.ny), indexing="ij")
    cxm = syc[J] / (sxf[I] * h2)          # to (i-1, j) through face i
    cxp = syc[J] / (sxf[I + 1] * h2)      # to (i+1, j) through face i+1
    cym = sxc[I] / (syf[J] * h2)          # to (i, j-1) through face j
    cyp = sxc[I] / (syf[J + 1] * h2)      # to (i, j+1) through face j+1
    diag = -(cxm + cxp + cym + cyp) + k0(p) ** 2 * eps * sxc[I] * syc[J]

    q = index(p, I, J)
    rows = [q.ravel()]
    cols = [q.ravel()]
    vals = [diag.ravel()]
    m = I > 0
    rows.append(q[m]); cols.append(index(p, I[m] - 1, J[m])); vals.append(cxm[m])
    m = I < p.nx - 1
    rows.append(q[m]); cols.append(index(p, I[m] + 1, J[m])); vals.append(cxp[m])
    m = J > 0
    rows.append(q[m]); cols.append(index(p, I[m], J[m] - 1)); vals.append(cym[m])
    m = J < p.ny - 1
    rows.append(q[m]); cols.append(index(p, I[m], J[m] + 1)); vals.append(cyp[m])
    N = p.nx * p.ny
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N), dtype=np.complex128)
    return A.tocsc()


def factor(A: sp.spmatrix):
    """SuperLU factorisation of A with partial pivoting and a COLAMD column ordering
    (the minimum-degree ordering of A + A^T fills these tall grids far more)."""
    return spla.splu(sp.csc_matrix(A), permc_spec="COLAMD")


def point_source(p: Problem, i: int, j: int) -> np.ndarray:
    """b for a unit point source f = delta(r - r_ij) (discretised as e_q / h^2)."""
    sxc, _, syc, _ = stretches(p)
    b = np.zeros(p.nx * p.ny, dtype=np.complex128)
    b[index(p, i, j)] = -sxc[i] * syc[j] / (p.h * p.h)
    return b


def source_amplitude(p: Problem, theta) -> np.ndarray:
    """Sheet-current amplitude J(theta) of the unit-power equivalent source.

    A line current J delta(y - y_s) exp(i K sin(theta) x) in a medium of index n
    (K = n k) radiates planewaves of amplitude i J / (2 K cos theta) on each side.
    A planewave of unit power through a horizontal plane has amplitude
    1/sqrt(n cos theta), hence J = -2 i k sqrt(n cos theta).
    """
    theta = np.asarray(theta, dtype=np.float64)
    return -2j * k0(p) * np.sqrt(p.n_source * np.cos(theta))


def planewave_line(p: Problem, thetas) -> np.ndarray:
    """b0(theta) on the incidence line only: M x len(thetas).

    theta is measured in the source-plane medium (index n_source); the current
    sits on row source_row over the physical columns, and b = -f there (the
    stretch factors are 1 outside the PML).
    """
    thetas = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    i0, i1 = p.aperture
    x = x_centres(p)[i0:i1]
    K = p.n_source * k0(p)
    J = source_amplitude(p, thetas)                                # (Q,)
    f_line = (J[None, :] / p.h) * np.exp(1j * K * np.outer(x, np.sin(thetas)))
    return -f_line


def planewave_sources(p: Problem, thetas) -> np.ndarray:
    """b0(theta) for each angle: N x len(thetas), nonzero on the incidence line."""
    thetas = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    i0, i1 = p.aperture
    B = np.zeros((p.nx * p.ny, thetas.size), dtype=np.complex128)
    B[index(p, np.arange(i0, i1), p.source_row), :] = planewave_line(p, thetas)
    return B


def objective_vector(p: Problem) -> np.ndarray:
    """w with w^dag u = focal field (concentrator) or output-mode amplitude (collimator)."""
    w = np.zeros(p.nx * p.ny, dtype=np.complex128)
    if p.objective == CONCENTRATOR:
        w[index(p, *p.focus)] = 1.0
    elif p.objective == COLLIMATOR:
        i0, i1 = p.aperture
        x = x_centres(p)[i0:i1]
        Lm = (i1 - i0) * p.h
        w[index(p, np.arange(i0, i1), p.monitor_row)] = (p.h / Lm) * np.exp(
            1j * k0(p) * p.n_monitor * math.sin(p.phi) * x)
    else:
        raise ValueError("unknown objective")
    return w


def aperture_indices(p: Problem) -> np.ndarray:
    """Unknown indices of the incidence line (the plane where W acts)."""
    i0, i1 = p.aperture
    return index(p, np.arange(i0, i1), p.source_row)
