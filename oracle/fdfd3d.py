"""Oracle: 3D vector frequency-domain Maxwell solve on a Yee grid, and the
reciprocal angle-and-polarisation average of Sec. "Concluding remarks".

TEST INFRASTRUCTURE ONLY (see the package docstring).

In 3D the field is a vector and incoherent light varies over two incidence
angles and two polarisations.  The paper notes that the reciprocal method then
needs one solve per field component that the figure of merit reads: three for
the intensity |E|^2 at a focal spot, two for the power in an output planewave
mode (one per output polarisation).  With E = A^{-1} b,

    <sum_c |w_c^dag E|^2> = sum_c v_c^dag W v_c,   v_c = A^{-dag} w_c on the
                                                    incidence plane,
    W = < b b^dag > = sum over angles and both polarisations of alpha b b^dag,

the 3D form of Eq. 6 = Eq. 7 (this module computes both sides by their plain
definitions; W is built from the same quadrature rule as the forward average).

Discretisation (time dependence exp(-i omega t), vacuum wavelength 1, mu = 1):
curl curl E - k^2 eps E = i k J on a Yee grid -- E_x at ((i+1/2)h, j h, k h),
E_y at (i h, (j+1/2)h, k h), E_z at (i h, j h, (k+1/2)h) -- with tangential E
zero beyond the arrays.  The PML is the uniaxial form of stretched coordinates,

    A = C^T D_mu^{-1} C - k^2 D_eps eps,
    D = diag(s_y s_z / s_x, s_x s_z / s_y, s_x s_y / s_z) at each component,

with C the forward-difference curl (E on edges -> H on faces) and C^T the
backward one; A is complex symmetric (A = A^T), so reciprocity holds inside the
PML too.  Same stretch profile as the 2D operator (m = 3, R = 1e-8).

Index of component c at cell (i, j, k): c N + (i ny + j) nz + k, N = nx ny nz.

Pinned (tests/test_oracle_pins_3d.py): A = A^T and reciprocity of its inverse;
the reciprocal form with one solve per component equal to the forward average
over directions and both polarisations; the divergence-free displacement field
of the curl-curl operator; the polarisation vectors; the absolute scale of the
unit-power sheet currents (``sheet_amplitudes``): a full-width s or p sheet
sends a flux of 1 per unit area to each side at 0, 20 and 40 degrees.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import COLLIMATOR, CONCENTRATOR, Problem3D


def k0(p: Problem3D) -> float:
    return 2.0 * math.pi / p.wavelength


def stretch(p: Problem3D, n_axis: int, xi: np.ndarray) -> np.ndarray:
    """s(xi) = 1 + i sigma (d/L)^m at positions xi (cell units) along an axis of n_axis cells."""
    L = p.npml * p.h
    depth = np.maximum(np.maximum(p.npml - xi, xi - (n_axis - p.npml)), 0.0) * p.h
    sigma = (p.pml_m + 1) * math.log(1.0 / p.pml_R) / (2.0 * k0(p) * L)
    return 1.0 + 1j * sigma * (depth / L) ** p.pml_m


def _grids(p: Problem3D):
    return np.meshgrid(np.arange(p.nx), np.arange(p.ny), np.arange(p.nz), indexing="ij")


def component_positions(p: Problem3D, c: int):
    """(x, y, z) in cell units (0 = lower grid edge) of component c on every cell."""
    I, J, K = _grids(p)
    pos = [I.astype(float), J.astype(float), K.astype(float)]
    pos[c] = pos[c] + 0.5
    return pos


def face_positions(p: Problem3D, c: int):
    """(x, y, z) in cell units of H component c (faces normal to axis c)."""
    I, J, K = _grids(p)
    pos = [I + 0.5, J + 0.5, K + 0.5]
    pos[c] = pos[c] - 0.5
    return [a.astype(float) for a in pos]


def uniaxial(p: Problem3D, pos, c: int) -> np.ndarray:
    """s_a s_b / s_c for component c at positions pos (a, b the other two axes)."""
    s = [stretch(p, p.nx, pos[0]), stretch(p, p.ny, pos[1]), stretch(p, p.nz, pos[2])]
    a, b = [d for d in range(3) if d != c]
    return s[a] * s[b] / s[c]


def permittivity(p: Problem3D, widths=None):
    """eps at the position of each E component: three (nx, ny, nz) arrays.

    Background eps_bg, substrate below sub_layers (all x, y), and in the pillar
    layers the mean of eps over the h x h square around the component's (x, y)
    (square pillars of side w centred on the lattice points)."""
    widths = p.widths if widths is None else widths
    out = []
    for c in range(3):
        pos = component_positions(p, c)
        x = (pos[0] - p.npml) * p.h
        y = (pos[1] - p.npml) * p.h
        z = pos[2]
        frac = np.zeros(x.shape)
        for (xc, yc), w in zip(p.pillar_centers, widths):
            fx = np.clip(np.minimum(x + p.h / 2, xc + w / 2) - np.maximum(x - p.h / 2, xc - w / 2),
                         0.0, None) / p.h
            fy = np.clip(np.minimum(y + p.h / 2, yc + w / 2) - np.maximum(y - p.h / 2, yc - w / 2),
                         0.0, None) / p.h
            frac += fx * fy
        eps = np.full(x.shape, p.eps_bg)
        eps[z < p.sub_layers] = p.eps_sub
        layer = (z >= p.pillar_k0) & (z < p.pillar_k0 + p.pillar_layers)
        eps[layer] = p.eps_bg + (p.eps_pillar - p.eps_bg) * frac[layer]
        out.append(eps)
    return out


def index(p: Problem3D, c: int, i, j, k):
    N = p.n_cells
    return c * N + (np.asarray(i) * p.ny + np.asarray(j)) * p.nz + np.asarray(k)


def curl(p: Problem3D) -> sp.csr_matrix:
    """Forward-difference curl C: E (3N) -> H (3N), H_c on the faces normal to c.

    H_x = dE_z/dy - dE_y/dz, H_y = dE_x/dz - dE_z/dx, H_z = dE_y/dx - dE_x/dy,
    each difference (E(. + 1) - E(.)) / h with E = 0 beyond the arrays."""
    N = p.n_cells
    n = (p.nx, p.ny, p.nz)
    I, J, K = _grids(p)
    rows, cols, vals = [], [], []

    def diff(hc, ec, axis, sign):
        # + sign (E_ec(cell + e_axis) - E_ec(cell)) / h into H_hc(cell)
        r = index(p, hc, I, J, K).ravel()
        rows.append(r)
        cols.append(index(p, ec, I, J, K).ravel())
        vals.append(np.full(r.size, -sign / p.h))
        idx = [I, J, K]
        m = (idx[axis] + 1 < n[axis]).ravel()
        nb = [I, J, K]
        nb = [a + (1 if d == axis else 0) for d, a in enumerate(nb)]
        rows.append(r[m])
        cols.append(index(p, ec, *[a.ravel()[m] for a in nb]))
        vals.append(np.full(int(m.sum()), sign / p.h))

    diff(0, 2, 1, +1.0)
    diff(0, 1, 2, -1.0)
    diff(1, 0, 2, +1.0)
    diff(1, 2, 0, -1.0)
    diff(2, 1, 0, +1.0)
    diff(2, 0, 1, -1.0)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * N, 3 * N)).tocsr()


def operator(p: Problem3D, eps=None) -> sp.csc_matrix:
    """A = C^T D_mu^{-1} C - k^2 D_eps eps (3N x 3N complex128, symmetric)."""
    if eps is None:
        eps = permittivity(p)
    C = curl(p)
    dmu = np.concatenate([uniaxial(p, face_positions(p, c), c).ravel() for c in range(3)])
    deps = np.concatenate([(uniaxial(p, component_positions(p, c), c) * eps[c]).ravel()
                           for c in range(3)])
    A = C.T @ sp.diags(1.0 / dmu) @ C - k0(p) ** 2 * sp.diags(deps)
    return sp.csc_matrix(A, dtype=np.complex128)


def factor(A):
    return spla.splu(sp.csc_matrix(A), permc_spec="COLAMD")


# -- sources and objectives -----------------------------------------------------------

def polarisations(theta: float, azimuth: float):
    """Unit sheet-current directions (in the x-y plane) of the s and p waves of
    the incidence direction (theta, azimuth): s is normal to the plane of
    incidence, p lies along the tangential wavevector."""
    kp = np.array([math.cos(azimuth), math.sin(azimuth), 0.0])
    s = np.array([-kp[1], kp[0], 0.0])
    return s, kp


def sheet_amplitudes(p: Problem3D, theta: float):
    """Magnitudes |J| of the unit-power sheet currents of the s and p waves.

    A tangential sheet current J on the plane radiates a planewave to each side;
    for the s wave its tangential E is k |J| / (2 k_z), for the p wave its
    tangential H is |J| / 2.  A unit-power wave (power flux 1 per unit area
    through a plane z = const, in the normalisation (1/k) Im(conj E . dE/dz) of
    the scalar case) has |E| = 1 / sqrt(n cos theta) (s) and |H| = sqrt(n / cos
    theta) (p), so |J_s| = 2 sqrt(n cos theta) and |J_p| = 2 sqrt(n / cos theta)."""
    n = p.n_source
    ct = math.cos(theta)
    return 2.0 * math.sqrt(n * ct), 2.0 * math.sqrt(n / ct)


def plane_unknowns(p: Problem3D, kplane: int):
    """Indices of the tangential components (E_x, E_y) on plane k = kplane over
    the physical cells: the incidence (or monitor) plane."""
    a = np.arange(p.npml, p.nx - p.npml)
    b = np.arange(p.npml, p.ny - p.npml)
    I, J = np.meshgrid(a, b, indexing="ij")
    ix = index(p, 0, I, J, kplane).ravel()
    iy = index(p, 1, I, J, kplane).ravel()
    return np.concatenate([ix, iy])


def planewave_sources(p: Problem3D, thetas, azimuths):
    """b = i k J for the unit-power s and p sheet currents of each direction,
    on the incidence plane's physical cells: 3N x (2 Q), columns (q, s), (q, p).
    theta, azimuth are measured in the source medium; the current carries the
    tangential phase exp(i K sin theta (cos az x + sin az y)), K = n k, with x, y
    of each component's own position."""
    thetas = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    azimuths = np.atleast_1d(np.asarray(azimuths, dtype=np.float64))
    N = p.n_cells
    K = p.n_source * k0(p)
    a = np.arange(p.npml, p.nx - p.npml)
    b = np.arange(p.npml, p.ny - p.npml)
    I, J = np.meshgrid(a, b, indexing="ij")
    ks = p.source_k
    B = np.zeros((3 * N, 2 * thetas.size), dtype=np.complex128)
    for q, (th, az) in enumerate(zip(thetas, azimuths)):
        js, jp = sheet_amplitudes(p, th)
        sdir, pdir = polarisations(th, az)
        kx, ky = K * math.sin(th) * math.cos(az), K * math.sin(th) * math.sin(az)
        for c in range(2):
            x = ((I + (0.5 if c == 0 else 0.0)) - p.npml) * p.h
            y = ((J + (0.5 if c == 1 else 0.0)) - p.npml) * p.h
            ph = np.exp(1j * (kx * x + ky * y)).ravel()
            idx = index(p, c, I, J, ks).ravel()
            # a sheet current spread over one cell height: J / h per edge
            B[idx, 2 * q] = 1j * k0(p) * js * sdir[c] / p.h * ph
            B[idx, 2 * q + 1] = 1j * k0(p) * jp * pdir[c] / p.h * ph
    return B


def objective_vectors(p: Problem3D):
    """The w_c the figure of merit reads, as columns of a 3N x m matrix.

    Concentrator: the three field components at the focus cell (m = 3), so that
    sum_c |w_c^dag E|^2 = |E(focus)|^2.  Collimator: the amplitudes of the two
    polarisations of the output planewave mode in direction (out_theta,
    out_azimuth) on the monitor plane (m = 2): w = (h^2 / A) e_pol
    exp(i k sin theta (cos az x + sin az y)) on the tangential components, A the
    monitor area."""
    N = p.n_cells
    if p.objective == CONCENTRATOR:
        Wm = np.zeros((3 * N, 3), dtype=np.complex128)
        for c in range(3):
            Wm[index(p, c, *p.focus), c] = 1.0
        return Wm
    if p.objective == COLLIMATOR:
        a = np.arange(p.npml, p.nx - p.npml)
        b = np.arange(p.npml, p.ny - p.npml)
        I, J = np.meshgrid(a, b, indexing="ij")
        area = (a.size * p.h) * (b.size * p.h)
        kk = k0(p) * math.sin(p.out_theta)
        sdir, pdir = polarisations(p.out_theta, p.out_azimuth)
        Wm = np.zeros((3 * N, 2), dtype=np.complex128)
        for m, e in enumerate((sdir, pdir)):
            for c in range(2):
                x = ((I + (0.5 if c == 0 else 0.0)) - p.npml) * p.h
                y = ((J + (0.5 if c == 1 else 0.0)) - p.npml) * p.h
                ph = np.exp(1j * kk * (math.cos(p.out_azimuth) * x + math.sin(p.out_azimuth) * y))
                Wm[index(p, c, I, J, p.monitor_k).ravel(), m] = (p.h ** 2 / area) * e[c] * ph.ravel()
        return Wm
    raise ValueError("unknown objective")


# -- light and the two averages ------------------------------------------------------------

def cone_rule(p: Problem3D, n_theta: int, n_az: int):
    """Quadrature over the cone theta <= c with the uniform angular density
    alpha = 1 / Omega, Omega = 2 pi (1 - cos c): Gauss-Legendre in theta (with
    the sin theta of the solid angle) times the trapezoid rule in the azimuth.
    Returns (thetas, azimuths, weights) with weights including alpha."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    th = 0.5 * p.c * (x + 1.0)
    wt = 0.5 * p.c * w * np.sin(th)
    az = 2.0 * math.pi * np.arange(n_az) / n_az
    T, A = np.meshgrid(th, az, indexing="ij")
    Wt = np.outer(wt, np.full(n_az, 2.0 * math.pi / n_az))
    omega = 2.0 * math.pi * (1.0 - math.cos(p.c))
    return T.ravel(), A.ravel(), Wt.ravel() / omega


class Solved3D:
    def __init__(self, p: Problem3D, eps=None):
        self.p = p
        self.A = operator(p, eps)
        self.lu = factor(self.A)

    def solve(self, B):
        return self.lu.solve(np.ascontiguousarray(B, dtype=np.complex128))


def brute_force(s: Solved3D, thetas, azimuths, weights) -> float:
    """The forward average: one solve per direction and polarisation,
    F = sum_q weight_q sum_pol sum_c |w_c^dag E_(q,pol)|^2."""
    B = planewave_sources(s.p, thetas, azimuths)
    E = s.solve(B)
    Wm = objective_vectors(s.p)
    amp = np.abs(Wm.conj().T @ E) ** 2               # (m, 2Q)
    per = amp.sum(axis=0).reshape(-1, 2).sum(axis=1)  # per direction, both polarisations
    return float(np.sum(np.asarray(weights) * per))


def reciprocal_fields(s: Solved3D) -> np.ndarray:
    """v_c = A^{-dag} w_c = conj(A^{-1} conj(w_c)) on the whole grid (3N x m)."""
    Wm = objective_vectors(s.p)
    return np.conj(s.solve(np.conj(Wm)))


def correlation_from_rule(p: Problem3D, thetas, azimuths, weights) -> np.ndarray:
    """W = sum_q weight_q sum_pol b b^dag on the incidence-plane unknowns."""
    idx = plane_unknowns(p, p.source_k)
    B = planewave_sources(p, thetas, azimuths)[idx, :]
    wq = np.repeat(np.asarray(weights), 2)
    return (B * wq[None, :]) @ B.conj().T


def reciprocal(s: Solved3D, Wc: np.ndarray) -> float:
    """sum_c v_c^dag W v_c with one reciprocal solve per component the FOM reads."""
    Z = reciprocal_fields(s)
    V = Z[plane_unknowns(s.p, s.p.source_k), :]
    F = sum(complex(np.vdot(V[:, c], Wc @ V[:, c])) for c in range(V.shape[1]))
    return F.real
