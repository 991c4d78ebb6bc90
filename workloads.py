"""Seeded synthetic workloads shared by the oracle and the GPU path.

This module holds only *inputs*: grid sizes, cell indices of rows and points,
pillar centres and seeded widths, light-distribution parameters and seeded
request streams.  It contains none of the method's arithmetic (no permittivity
map, no PML, no operator, no sources, no current correlations W); each side
computes those from these numbers on its own.  The amplitude statistics of a
light ensemble (which angles, how their random amplitudes correlate) are inputs.

The shapes follow the paper's setting (Sec. "Designs": a single layer of
dielectric pillars of sub-wavelength period on a substrate, concentrator /
collimator objectives, light uniform in a cone or an annulus of angles), scaled
to the synthetic configurations below:

* ``config1``  10 x 8 wavelengths, 10 pillars, cone +-10 deg, concentrator
                (240 x 200 cells with a 20-cell PML on every side).
* ``config2``  100 x 52 wavelengths, 100 pillars, cone +-20 deg, concentrator
                with focal distance 50 (2040 x 1080 cells).
* ``config3``  200 x 20 wavelengths, 200 pillars, annulus 10-30 deg and its
                mirror, collimator at output angle 0 (4040 x 440 cells).
* ``config4_large`` 100 x 20 wavelengths, 100 pillars, cone +-10 deg,
                concentrator 5 wavelengths above a 100 x 10 design region
                (2040 x 440 cells).
* ``serving_stream`` Poisson arrivals of concentrator / collimator requests of
                random width and depth.
* ``output_set`` / ``ensemble_angles`` / ``gaussian_correlated_amplitudes``
                many outputs of one evaluation (focal spots and output modes)
                and a finite ensemble of planewaves with correlated amplitudes
                (light that is not translation invariant).
* ``spectral_rule`` a flat spectrum sampled at n wavelengths (broadband).

Units: vacuum wavelength 1, grid step h = 1/20.  Cell (i, j) has its centre at
x = (i - npml + 1/2) h, y = (j - npml + 1/2) h, origin at the lower-left corner
of the physical (non-PML) region.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

CONCENTRATOR = 0
COLLIMATOR = 1
CONE = 0
ANNULUS = 1


@dataclass(frozen=True)
class Problem:
    """One metasurface evaluation: geometry, objective and light statistics."""

    name: str
    nx: int                      # cells along x (long axis, block index)
    ny: int                      # cells along y (block size n)
    npml: int = 20
    h: float = 0.05
    wavelength: float = 1.0
    pml_R: float = 1e-8          # target normal-incidence PML reflection
    pml_m: int = 3               # PML grading exponent
    eps_bg: float = 1.0
    eps_sub: float = 2.25
    eps_pillar: float = 5.76
    sub_rows: int = 40           # rows j < sub_rows hold substrate (y < 1), PML included
    pillar_row0: int = 40        # first pillar-layer row (y = 1)
    pillar_rows: int = 10        # pillar height 0.5 = 10 rows
    pillar_centers: Tuple[float, ...] = ()
    widths: Tuple[float, ...] = ()
    objective: int = CONCENTRATOR
    focus: Tuple[int, int] = (0, 0)          # concentrator: focus cell (i, j)
    monitor_row: int = 0                     # collimator: monitor row j_m
    phi: float = 0.0                         # collimator output angle (rad, in air)
    n_monitor: float = 1.0
    source_row: int = 30                     # incidence line (equivalent source plane) j_s
    n_source: float = 1.5                    # index of the source-plane medium (substrate)
    light: int = CONE
    c: float = 0.0                           # cone half-angle (rad)
    th1: float = 0.0                         # annulus inner edge (rad)
    th2: float = 0.0                         # annulus outer edge (rad)

    # derived, integer-only helpers (no physics)
    @property
    def n_cells(self) -> int:
        return self.nx * self.ny

    @property
    def aperture(self) -> Tuple[int, int]:
        """Physical columns [i0, i1) of the incidence line / monitor row."""
        return self.npml, self.nx - self.npml

    @property
    def m_aperture(self) -> int:
        i0, i1 = self.aperture
        return i1 - i0


def seeded_widths(n: int, seed: int, lo: float = 0.1, hi: float = 0.9) -> Tuple[float, ...]:
    rng = np.random.default_rng(seed)
    return tuple(float(w) for w in rng.uniform(lo, hi, size=n))


def _pillars(n: int, period: float = 1.0) -> Tuple[float, ...]:
    return tuple((p + 0.5) * period for p in range(n))


def metasurface(name: str, width_wl: int, height_wl: int, seed: int, *,
                objective: int = CONCENTRATOR, focus_height: float = 5.0,
                light: int = CONE, c_deg: float = 10.0, th1_deg: float = 0.0,
                th2_deg: float = 0.0, phi: float = 0.0, monitor_y: float = 11.5,
                npml: int = 20, h: float = 0.05) -> Problem:
    """A physical region width_wl x height_wl wavelengths, pillars of period 1."""
    per = int(round(1.0 / h))
    nxp, nyp = width_wl * per, height_wl * per
    nx, ny = nxp + 2 * npml, nyp + 2 * npml
    sub_rows = npml + per          # substrate y < 1
    pillar_row0 = npml + per       # pillars y in [1, 1.5)
    pillar_rows = per // 2
    top = pillar_row0 + pillar_rows           # first row above the pillars
    fj = top + int(round(focus_height * per))  # focus row: focus_height above pillar tops
    fi = npml + nxp // 2
    mj = npml + int(round((monitor_y - 0.5 * h) / h))
    return Problem(name=name, nx=nx, ny=ny, npml=npml, h=h,
                   sub_rows=sub_rows, pillar_row0=pillar_row0, pillar_rows=pillar_rows,
                   pillar_centers=_pillars(width_wl), widths=seeded_widths(width_wl, seed),
                   objective=objective, focus=(fi, fj), monitor_row=mj, phi=phi,
                   source_row=npml + per // 2, light=light,
                   c=math.radians(c_deg), th1=math.radians(th1_deg), th2=math.radians(th2_deg))


def config1(seed: int = 1001) -> Problem:
    """Plain FP64 concentrator, 10 x 8 wavelengths (240 x 200 cells)."""
    return metasurface("config1", 10, 8, seed, focus_height=5.0, c_deg=10.0)


def config2(seed: int = 1002) -> Problem:
    """Concentrator 100 wavelengths wide, focal distance 50 (2040 x 1080 cells)."""
    # 52 wavelengths of physical height: substrate (1) + pillars (0.5) + 50 to the
    # focus + 0.5 clearance below the top PML.
    return metasurface("config2", 100, 52, seed, focus_height=50.0, c_deg=20.0)


def config3(seed: int = 1003) -> Problem:
    """Collimator 200 x 20 wavelengths, annulus 10-30 deg + mirror (4040 x 440)."""
    return metasurface("config3", 200, 20, seed, objective=COLLIMATOR, light=ANNULUS,
                       th1_deg=10.0, th2_deg=30.0, phi=0.0, monitor_y=11.5)


def config4_large(seed: int = 1004) -> Problem:
    """Adjoint step at scale: 100 x 20 wavelengths, cone +-10 deg (2040 x 440)."""
    return metasurface("config4_large", 100, 20, seed, focus_height=5.0 + 9.5, c_deg=10.0)


def small_problem(width_wl: int = 4, height_wl: int = 4, seed: int = 7, *,
                  objective: int = CONCENTRATOR, light: int = CONE, c_deg: float = 15.0,
                  th1_deg: float = 5.0, th2_deg: float = 20.0, npml: int = 10,
                  focus_height: float = 2.0, monitor_y: float = 3.0,
                  phi: float = 0.0) -> Problem:
    """A tiny problem the oracle factors in well under a second."""
    return metasurface(f"small{width_wl}x{height_wl}", width_wl, height_wl, seed,
                       objective=objective, light=light, c_deg=c_deg, th1_deg=th1_deg,
                       th2_deg=th2_deg, npml=npml, focus_height=focus_height,
                       monitor_y=monitor_y, phi=phi)


def with_light(p: Problem, *, light: int, c: float = 0.0, th1: float = 0.0,
               th2: float = 0.0) -> Problem:
    return replace(p, light=light, c=c, th1=th1, th2=th2)


def pixel_patch(p: Problem, width_cells: int, height_cells: int) -> Tuple[int, int, int, int]:
    """Central patch of the pillar layer [i0, i1) x [j0, j1) for per-pixel gradients."""
    ic = p.npml + (p.nx - 2 * p.npml) // 2
    i0 = ic - width_cells // 2
    return i0, i0 + width_cells, p.pillar_row0, p.pillar_row0 + height_cells


def seeded_cells(p: Problem, count: int, seed: int,
                 region: Optional[Tuple[int, int, int, int]] = None) -> np.ndarray:
    """Distinct seeded cell indices q = i*ny + j inside region (default: physical)."""
    rng = np.random.default_rng(seed)
    if region is None:
        region = (p.npml, p.nx - p.npml, p.npml, p.ny - p.npml)
    i0, i1, j0, j1 = region
    qs = set()
    while len(qs) < count:
        i = int(rng.integers(i0, i1))
        j = int(rng.integers(j0, j1))
        qs.add(i * p.ny + j)
    return np.array(sorted(qs), dtype=np.int64)


def complex_normal(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


# ----------------------------------------------------------------------------
# Many outputs and correlated light (inputs only)
# ----------------------------------------------------------------------------

def output_set(p: Problem, n_spots: int, n_modes: int = 0, seed: int = 3001) -> List[Problem]:
    """Outputs of one evaluation: copies of p that differ only in the objective.

    ``n_spots`` focal spots at distinct seeded columns of p's focal row (middle
    half of the physical width), then ``n_modes`` planewave output modes on p's
    monitor row at seeded angles U[-20, 20] deg.
    """
    rng = np.random.default_rng(seed)
    nxp = p.nx - 2 * p.npml
    lo, hi = p.npml + nxp // 4, p.npml + (3 * nxp) // 4
    if n_spots > hi - lo:
        raise ValueError("more focal spots than columns in the middle half")
    cols = rng.choice(np.arange(lo, hi), size=n_spots, replace=False)
    fj = p.focus[1]
    out = [replace(p, objective=CONCENTRATOR, focus=(int(i), fj)) for i in cols]
    for _ in range(n_modes):
        phi = math.radians(float(rng.uniform(-20.0, 20.0)))
        out.append(replace(p, objective=COLLIMATOR, phi=phi))
    return out


def ensemble_angles(p: Problem, n: int) -> np.ndarray:
    """n evenly spaced incidence angles (cell midpoints) over the light's support.

    Cone: n cells of [-c, c]; annulus: n/2 cells on each of [-th2, -th1] and
    [th1, th2] (n even).
    """
    if p.light == CONE:
        ivs = [(-p.c, p.c)]
    else:
        ivs = [(-p.th2, -p.th1), (p.th1, p.th2)]
    per = n // len(ivs)
    if per * len(ivs) != n or per < 1:
        raise ValueError("angle count must split evenly over the intervals")
    th = [lo + (np.arange(per) + 0.5) * (hi - lo) / per for lo, hi in ivs]
    return np.concatenate(th)


def gaussian_correlated_amplitudes(thetas: np.ndarray, sigma_deg: float = 2.0,
                                   tilt: float = 3.0, skew: float = 2.0) -> np.ndarray:
    """Amplitude correlation <a_q conj(a_q')> of a partially coherent ensemble.

    sqrt(s_q s_q') exp(-(th_q - th_q')^2 / (2 sigma^2)) exp(i tilt (th_q - th_q')) / n
    with mean-square weight s_q = exp(skew th_q): angles closer than about sigma
    are correlated (a beam of finite width), the phase tilt makes the matrix
    complex and the skew makes the light brighter on one side, so that the
    current correlation it implies is complex as well.  Hermitian and positive
    semi-definite.
    """
    th = np.asarray(thetas, dtype=np.float64)
    d = th[:, None] - th[None, :]
    s = math.radians(sigma_deg)
    amp = np.exp(0.5 * skew * th)
    return (amp[:, None] * amp[None, :] * np.exp(-d * d / (2 * s * s)) * np.exp(1j * tilt * d)
            / th.size).astype(np.complex128)


def coherent_amplitudes(n: int, seed: int) -> np.ndarray:
    """Seeded complex amplitudes a_q of a fully coherent superposition."""
    return complex_normal(n, seed) / math.sqrt(n)


def spectral_rule(n: int, lam_lo: float = 0.9, lam_hi: float = 1.1):
    """A flat spectrum over vacuum wavelengths [lam_lo, lam_hi] as n frequency samples.

    Midpoints of n equal cells in frequency 1/lam, each of weight 1/n (the
    weights sum to one).  Returns (wavelengths, weights), longest wavelength
    first.
    """
    f_lo, f_hi = 1.0 / lam_hi, 1.0 / lam_lo
    f = f_lo + (np.arange(n) + 0.5) * (f_hi - f_lo) / n
    return 1.0 / f, np.full(n, 1.0 / n)


def random_hermitian(m: int, seed: int) -> np.ndarray:
    """A seeded dense Hermitian m x m matrix (X + X^dag) / 2, X complex normal."""
    x = complex_normal((m, m), seed)
    return 0.5 * (x + x.conj().T)


# ----------------------------------------------------------------------------
# Serving mix: Poisson request stream
# ----------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float               # seconds since stream start
    problem: Problem
    adjoint: bool


def serving_stream(n_requests: int, rate: float = 200.0, seed: int = 5001, *,
                   width_range=(20, 300), depth_range=(10, 60), adjoint_frac: float = 0.2,
                   geometry_pool: int = 0, geom_seed: int = 5002,
                   scale: float = 1.0) -> List[Request]:
    """Seeded Poisson stream of concentrator / collimator evaluations.

    Widths are uniform in width_range wavelengths, depths in depth_range; cone
    half-angles are U[5, 40] deg, annuli have inner edge U[5, 20] deg and width
    U[5, 40] deg.  ``scale`` shrinks widths and depths (for tests).  With
    ``geometry_pool`` > 0 the geometries are drawn from a seeded pool of that
    many, so that requests can share factors.
    """
    rng = np.random.default_rng(seed)
    grng = np.random.default_rng(geom_seed)

    def draw_geom(k: int):
        w = int(round(grng.uniform(*width_range) * scale))
        d = int(round(grng.uniform(*depth_range) * scale))
        return max(w, 2), max(d, 4), 10_000 + k

    pool = [draw_geom(k) for k in range(geometry_pool)] if geometry_pool > 0 else None
    t = 0.0
    out: List[Request] = []
    for r in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        if pool is not None:
            w, d, gseed = pool[int(rng.integers(0, len(pool)))]
        else:
            w, d, gseed = draw_geom(100 + r)
        collim = bool(rng.uniform() < 0.5)
        annulus = bool(rng.uniform() < 0.5)
        adj = bool(rng.uniform() < adjoint_frac)
        if annulus:
            th1 = float(rng.uniform(5.0, 20.0))
            th2 = th1 + float(rng.uniform(5.0, 40.0))
            light = dict(light=ANNULUS, th1_deg=th1, th2_deg=th2)
        else:
            light = dict(light=CONE, c_deg=float(rng.uniform(5.0, 40.0)))
        fh = min(5.0, d - 2.5)
        p = metasurface(f"req{r}", w, d, gseed,
                        objective=COLLIMATOR if collim else CONCENTRATOR,
                        focus_height=fh, monitor_y=min(d - 1.0, 1.5 + fh), **light)
        out.append(Request(rid=r, arrival=t, problem=p, adjoint=adj))
    return out


# ----------------------------------------------------------------------------
# 3D metasurfaces (vector fields on a Yee grid; inputs only)
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Problem3D:
    """One 3D evaluation: a lattice of square pillars on a substrate, the
    incidence plane below them, a focus (or a monitor plane) above.

    Cells (i, j, k) have their centres at x = (i - npml + 1/2) h, likewise y and
    z, origin at the lower corner of the physical region.  Incident light is
    measured in the substrate (index n_source) by its polar angle theta from +z
    and its azimuth; a cone of half-angle c around +z.
    """

    name: str
    nx: int
    ny: int
    nz: int
    npml: int = 6
    h: float = 0.125
    wavelength: float = 1.0
    pml_R: float = 1e-8
    pml_m: int = 3
    eps_bg: float = 1.0
    eps_sub: float = 2.25
    eps_pillar: float = 5.76
    sub_layers: int = 14          # z-cells k < sub_layers hold substrate
    pillar_k0: int = 14           # first pillar layer
    pillar_layers: int = 4        # pillar height 0.5
    pillar_centers: Tuple[Tuple[float, float], ...] = ()
    widths: Tuple[float, ...] = ()
    objective: int = CONCENTRATOR
    focus: Tuple[int, int, int] = (0, 0, 0)
    monitor_k: int = 0            # collimator: monitor plane
    out_theta: float = 0.0        # collimator output direction (rad, in air)
    out_azimuth: float = 0.0
    source_k: int = 10            # incidence plane
    n_source: float = 1.5
    c: float = 0.0                # cone half-angle (rad)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz


def metasurface3d(name: str, width_wl: int, height_wl: float, seed: int, *,
                  h: float = 0.125, npml: int = 6, objective: int = CONCENTRATOR,
                  focus_height: float = 1.0, monitor_y: float = 1.5, c_deg: float = 15.0,
                  out_theta: float = 0.0, out_azimuth: float = 0.0) -> Problem3D:
    """width_wl x width_wl pillars of period 1 (seeded widths U[0.1, 0.9]) on a
    substrate 0.5 thick, pillar height 0.5; height_wl of physical depth."""
    per = int(round(1.0 / h))
    nxp = width_wl * per
    nzp = int(round(height_wl * per))
    sub = npml + per // 2
    pk = sub
    top = pk + per // 2
    centers = tuple(((a + 0.5), (b + 0.5)) for a in range(width_wl) for b in range(width_wl))
    fk = top + int(round(focus_height * per))
    mk = npml + int(round(monitor_y * per))
    what, k = ("focus", fk) if objective == CONCENTRATOR else ("monitor plane", mk)
    if not npml <= k < nzp + npml:
        raise ValueError(f"{what} at z cell {k} lies outside the physical cells "
                         f"[{npml}, {nzp + npml})")
    return Problem3D(name=name, nx=nxp + 2 * npml, ny=nxp + 2 * npml, nz=nzp + 2 * npml,
                     npml=npml, h=h, sub_layers=sub, pillar_k0=pk, pillar_layers=per // 2,
                     pillar_centers=centers, widths=seeded_widths(len(centers), seed),
                     objective=objective,
                     focus=(npml + nxp // 2, npml + nxp // 2, fk),
                     monitor_k=mk, out_theta=out_theta,
                     out_azimuth=out_azimuth, source_k=npml + per // 4,
                     c=math.radians(c_deg))


def cone_directions3d(p: Problem3D, n_theta: int, n_az: int):
    """The incident light of a 3D cone as sampled directions: polar angles at the
    Gauss-Legendre nodes of [0, c] (weighted by sin theta, the solid angle),
    azimuths evenly spaced over the circle; each weight includes the uniform
    mean-square amplitude 1 / Omega, Omega = 2 pi (1 - cos c).  Returns
    (thetas, azimuths, weights) of n_theta * n_az directions."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    th = 0.5 * p.c * (x + 1.0)
    wt = 0.5 * p.c * w * np.sin(th)
    az = 2.0 * math.pi * np.arange(n_az) / n_az
    T, A = np.meshgrid(th, az, indexing="ij")
    Wt = np.outer(wt, np.full(n_az, 2.0 * math.pi / n_az))
    omega = 2.0 * math.pi * (1.0 - math.cos(p.c))
    return T.ravel(), A.ravel(), Wt.ravel() / omega
