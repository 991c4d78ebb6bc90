"""3D vector problems (Sec. "Concluding remarks") through librecip's rcp_*3d calls.

Fields and permittivities are torch tensors in the library's slice order: shape
(nx, 3, ny, nz) -- x-slice, component (E_x, E_y, E_z), y, z.  Every step runs in
the library's kernels; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import torch

from workloads import CONCENTRATOR, Problem3D
from . import _lib, _on_stream
from ._lib import RCP_COLLIMATOR, RCP_CONCENTRATOR, RecipError, check, lib


def _stream(stream=None) -> int:
    return (stream if stream is not None else torch.cuda.current_stream()).cuda_stream


def k0_of(p: Problem3D) -> float:
    return 2.0 * math.pi / p.wavelength


def grid_struct(p: Problem3D, eps: Optional[torch.Tensor] = None) -> _lib.Grid3D:
    return _lib.Grid3D(p.nx, p.ny, p.nz, p.npml, p.h, k0_of(p), p.pml_R, p.pml_m,
                       eps.data_ptr() if eps is not None else None)


@_on_stream
def eps_from_pillars(p: Problem3D, device="cuda", stream=None) -> torch.Tensor:
    """Permittivity at the E positions, (nx, 3, ny, nz) float64."""
    centers = torch.tensor([c for xy in p.pillar_centers for c in xy] or [0.0],
                           dtype=torch.float64, device=device)
    widths = torch.tensor(list(p.widths) or [0.0], dtype=torch.float64, device=device)
    pil = _lib.Pillars3D(len(p.pillar_centers), centers.data_ptr(), widths.data_ptr(), p.eps_bg,
                         p.eps_sub, p.eps_pillar, p.sub_layers, p.pillar_k0, p.pillar_layers)
    eps = torch.empty((p.nx, 3, p.ny, p.nz), dtype=torch.float64, device=device)
    g = grid_struct(p)
    check(lib.rcp_eps3d_from_pillars(C.byref(g), C.byref(pil), eps.data_ptr(), _stream(stream)))
    return eps


class Factors3D:
    """Factored 3D operator of one geometry; owns its device buffer."""

    def __init__(self, p: Problem3D, eps: torch.Tensor, stream=None):
        if stream is not None:   # temporaries belong to the stream the kernels run on
            with torch.cuda.stream(stream):
                self._init(p, eps, stream)
        else:
            self._init(p, eps, None)

    def _init(self, p: Problem3D, eps: torch.Tensor, stream):
        self.problem = p
        eps = eps.to(torch.float64).contiguous()
        g = grid_struct(p, eps)
        self.nbytes = int(lib.rcp_factor3d_bytes(C.byref(g)))
        if self.nbytes == 0:
            raise RecipError(_lib.RCP_EINVAL, "invalid 3D grid")
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=eps.device)
        h = C.c_void_p()
        check(lib.rcp_factor3d(C.byref(g), self.buf.data_ptr(), self.nbytes, _stream(stream),
                               C.byref(h)))
        self.handle = h

    def release(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.rcp_factors_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


@_on_stream
def solve(fac: Factors3D, b: torch.Tensor, conj_transpose: bool = False, stream=None):
    b = b.to(torch.complex128).contiguous()
    x = torch.empty_like(b)
    check(lib.rcp_solve3d(fac.handle, b.data_ptr(), x.data_ptr(), 1 if conj_transpose else 0,
                          _stream(stream)))
    return x


def objective_struct(p: Problem3D) -> _lib.Objective3D:
    kind = RCP_CONCENTRATOR if p.objective == CONCENTRATOR else RCP_COLLIMATOR
    return _lib.Objective3D(kind, p.focus[0], p.focus[1], p.focus[2], p.monitor_k, p.out_theta,
                            p.out_azimuth, 1.0)


def _light(p: Problem3D, dirs: torch.Tensor) -> _lib.Light3D:
    return _lib.Light3D(p.source_k, p.n_source, dirs.shape[0], dirs.data_ptr())


def directions(thetas, azimuths, weights, device="cuda") -> torch.Tensor:
    """A (ndir, 3) device table of (theta, azimuth, weight)."""
    import numpy as np
    d = np.stack([np.asarray(thetas, float), np.asarray(azimuths, float),
                  np.asarray(weights, float)], axis=1)
    return torch.from_numpy(np.ascontiguousarray(d)).to(device)


def _work(fac, o, lt, device):
    need = int(lib.rcp_average3d_work_bytes(fac.handle, C.byref(o), C.byref(lt)))
    if need == 0:
        raise RecipError(_lib.RCP_EINVAL, "invalid 3D objective or light")
    return torch.empty(need, dtype=torch.uint8, device=device), need


@_on_stream
def reciprocal_average(fac: Factors3D, dirs: torch.Tensor, p: Optional[Problem3D] = None,
                       stream=None) -> torch.Tensor:
    """Eq. 7 in 3D: one reciprocal solve per component the objective reads."""
    p = p or fac.problem
    dirs = dirs.to(torch.float64).contiguous()
    o, lt = objective_struct(p), _light(p, dirs)
    work, need = _work(fac, o, lt, dirs.device)
    F = torch.empty((), dtype=torch.float64, device=dirs.device)
    check(lib.rcp_reciprocal_average3d(fac.handle, C.byref(o), C.byref(lt), F.data_ptr(),
                                       work.data_ptr(), need, _stream(stream)))
    return F


@_on_stream
def brute_force_average(fac: Factors3D, dirs: torch.Tensor, p: Optional[Problem3D] = None,
                        per: bool = False, stream=None):
    """Eq. 6 in 3D: one forward solve per direction and polarisation."""
    p = p or fac.problem
    dirs = dirs.to(torch.float64).contiguous()
    o, lt = objective_struct(p), _light(p, dirs)
    work, need = _work(fac, o, lt, dirs.device)
    F = torch.empty((), dtype=torch.float64, device=dirs.device)
    pv = torch.empty(2 * dirs.shape[0], dtype=torch.float64, device=dirs.device) if per else None
    check(lib.rcp_brute_force_average3d(fac.handle, C.byref(o), C.byref(lt), F.data_ptr(),
                                        pv.data_ptr() if pv is not None else None,
                                        work.data_ptr(), need, _stream(stream)))
    return (F, pv) if per else F
