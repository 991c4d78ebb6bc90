"""Reciprocal angle average of incoherent light through 2D metasurfaces on MI355X.

Python front end of librecip (include/recip.h).  PyTorch provides device
memory and streams; every step of the computation runs in librecip's HIP
kernels.  Method: Pestourie, Yao, Kante, Johnson, "Efficient inverse design of
large-area metasurfaces for incoherent light" -- one reciprocal solve
v = A^{-dag} w followed by the Toeplitz form v^dag W v (Eq. 7) instead of an
angle quadrature over forward solves (Eq. 6).
"""
from __future__ import annotations

import ctypes as C
import functools
import inspect
import math
from typing import Optional, Tuple

import torch

from workloads import ANNULUS, COLLIMATOR, CONCENTRATOR, CONE, Problem
from . import _lib
from ._lib import (RCP_ANNULUS, RCP_COLLIMATOR, RCP_CONCENTRATOR, RCP_CONE, RCP_FP32_REFINED,
                   RCP_FP64, RCP_SYMBOL_TABLE, RecipError, check, lib)

__all__ = ["Factors", "factor_batch", "FactorEngine", "factor_bytes", "eps_from_widths", "reciprocal_average",
           "brute_force_average", "adjoint_grad", "adjoint_grad_batch", "width_grad", "solve",
           "IncoherentFOM", "correlation_matrix", "reciprocal_average_dense",
           "adjoint_grad_dense", "broadband_grad",
           "RCP_FP64", "RCP_FP32_REFINED", "RecipError"]


def _stream(stream: Optional[torch.cuda.Stream] = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _on_stream(fn):
    """Run a wrapper that takes ``stream`` with that stream current, so that the
    device temporaries it allocates (argument copies, workspaces, outputs) belong
    to the stream its kernels run on and are not reused before they finish."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)
    return wrapper


def k0_of(p: Problem) -> float:
    return 2.0 * math.pi / p.wavelength


def grid_struct(p: Problem, eps: Optional[torch.Tensor] = None) -> _lib.Grid:
    return _lib.Grid(p.nx, p.ny, p.npml, p.h, k0_of(p), p.pml_R, p.pml_m,
                     eps.data_ptr() if eps is not None else None)


def objective_struct(p: Problem) -> _lib.Objective:
    i0, i1 = p.aperture
    kind = RCP_CONCENTRATOR if p.objective == CONCENTRATOR else RCP_COLLIMATOR
    return _lib.Objective(kind, p.focus[0], p.focus[1], p.monitor_row, i0, i1, p.phi, p.n_monitor)


def light_struct(p: Problem, symbol: Optional[torch.Tensor] = None) -> _lib.Light:
    i0, i1 = p.aperture
    if symbol is not None:
        return _lib.Light(p.source_row, i0, i1, p.n_source, RCP_SYMBOL_TABLE, 0.0, 0.0, 0.0,
                          symbol.data_ptr())
    kind = RCP_CONE if p.light == CONE else RCP_ANNULUS
    return _lib.Light(p.source_row, i0, i1, p.n_source, kind, p.c, p.th1, p.th2, None)


class _PillarArgs:
    """Keeps the device copies of pillar centres and widths alive with the struct."""

    def __init__(self, p: Problem, widths: Optional[torch.Tensor], device):
        self.centers = torch.tensor(p.pillar_centers, dtype=torch.float64, device=device)
        if widths is None:
            widths = torch.tensor(p.widths, dtype=torch.float64, device=device)
        self.widths = widths.detach().to(device=device, dtype=torch.float64).contiguous()
        self.struct = _lib.Pillars(len(p.pillar_centers), self.centers.data_ptr(),
                                   self.widths.data_ptr(), p.eps_bg, p.eps_sub, p.eps_pillar,
                                   p.sub_rows, p.pillar_row0, p.pillar_rows)


@_on_stream
def eps_from_widths(p: Problem, widths: Optional[torch.Tensor] = None, device="cuda",
                    stream=None) -> torch.Tensor:
    """Cell permittivity map (nx x ny float64) of the pillar layer (kernel a1)."""
    pa = _PillarArgs(p, widths, device)
    eps = torch.empty((p.nx, p.ny), dtype=torch.float64, device=device)
    g = grid_struct(p)
    check(lib.rcp_eps_from_widths(C.byref(g), C.byref(pa.struct), eps.data_ptr(), _stream(stream)))
    return eps


def factor_bytes(p: Problem, precision: int = RCP_FP64) -> int:
    g = grid_struct(p)
    n = lib.rcp_factor_bytes(C.byref(g), precision)
    if n == 0:
        raise RecipError(_lib.RCP_EINVAL, "invalid grid for factor_bytes")
    return int(n)


class Factors:
    """Factored operator of one geometry; owns its device buffer (a torch tensor)."""

    @_on_stream
    def __init__(self, p: Problem, eps: torch.Tensor, precision: int = RCP_FP64, stream=None,
                 buffer: Optional[torch.Tensor] = None):
        self.problem = p
        self.precision = precision
        self.nbytes = factor_bytes(p, precision)
        if buffer is None:
            buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=eps.device)
        if buffer.numel() < self.nbytes:
            raise RecipError(_lib.RCP_ENOMEM, "factor buffer too small")
        self.buf = buffer
        eps = eps.to(dtype=torch.float64).contiguous()
        g = grid_struct(p, eps)
        h = C.c_void_p()
        check(lib.rcp_factor(C.byref(g), precision, buffer.data_ptr(), self.nbytes,
                             _stream(stream), C.byref(h)))
        self.handle = h

    @classmethod
    def _wrap(cls, p: Problem, precision: int, buffer: torch.Tensor, handle: C.c_void_p):
        obj = cls.__new__(cls)
        obj.problem = p
        obj.precision = precision
        obj.nbytes = factor_bytes(p, precision)
        obj.buf = buffer
        obj.handle = handle
        return obj

    def release(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.rcp_factors_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def status(self, stream=None) -> None:
        """The pivot check of this set (waits for the stream; raises RecipError
        with RCP_ESINGULAR when a pivot failed)."""
        check(lib.rcp_factors_status(self.handle, _stream(stream)))

    def status_dev(self) -> int:
        """Device address of the set's int32 status word (0: every pivot passed)."""
        return int(lib.rcp_factors_status_dev(self.handle) or 0)

    def last_solve_stats(self) -> Tuple[int, float]:
        st = _lib.SolveStats()
        check(lib.rcp_last_solve_stats(self.handle, C.byref(st)))
        return int(st.iters), float(st.rel_residual)


@_on_stream
def factor_batch(problems, eps_list, precision: int = RCP_FP64, buffers=None, stream=None,
                 wait: bool = True):
    """Factor 1-16 same-grid geometries in the same kernel launches (chains side by side;
    above 8 as two groups on two library streams, side by side).

    wait=False enqueues only (rcp_factor_batch_async): the pivot check stays on
    the device until status() or status_dev() of a returned Factors reads it."""
    B = len(problems)
    if B < 1 or B > 16 or len(eps_list) != B:
        raise ValueError("factor_batch takes 1 to 16 problems with one eps map each")
    nbytes = factor_bytes(problems[0], precision)
    dev = eps_list[0].device
    if buffers is None:
        buffers = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(B)]
    eps_c = [e.to(dtype=torch.float64).contiguous() for e in eps_list]
    grids = (_lib.Grid * B)(*[grid_struct(p, e) for p, e in zip(problems, eps_c)])
    bufs = (C.c_void_p * B)(*[b.data_ptr() for b in buffers])
    outs = (C.c_void_p * B)()
    fn = lib.rcp_factor_batch if wait else lib.rcp_factor_batch_async
    check(fn(B, grids, precision, bufs, nbytes, _stream(stream), outs))
    return [Factors._wrap(p, precision, b, C.c_void_p(h)) for p, b, h in zip(problems, buffers, outs)]


class FactorEngine:
    """Factorisation engine (rcp_engine_*): geometries of any grid size factored
    in shared kernel launches, admitted while others are in progress.

    add() admits a geometry (its eps map, a caller buffer or a new one) and
    returns its Factors, usable once step() reports it done; step() enqueues
    rounds on the engine's stream and returns the Factors completed.  One host
    thread drives an engine."""

    def __init__(self, precision: int = RCP_FP64, stream: Optional[torch.cuda.Stream] = None):
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        check(lib.rcp_engine_create(precision, C.byref(h)))
        self.handle = h
        self.inflight = {}           # handle value -> (Factors, eps kept alive)

    def __len__(self) -> int:
        return len(self.inflight)

    def add(self, p: Problem, eps: torch.Tensor, buffer: Optional[torch.Tensor] = None) -> Factors:
        if len(self.inflight) >= 8:
            raise RecipError(_lib.RCP_EINVAL, "engine full: 8 geometries in flight")
        nbytes = factor_bytes(p, self.precision)
        with torch.cuda.stream(self.stream):
            if buffer is None:
                buffer = torch.empty(nbytes, dtype=torch.uint8, device=eps.device)
            if buffer.numel() < nbytes:
                raise RecipError(_lib.RCP_ENOMEM, "factor buffer too small")
            eps = eps.to(dtype=torch.float64).contiguous()
            g = grid_struct(p, eps)
            h = C.c_void_p()
            check(lib.rcp_engine_add(self.handle, C.byref(g), buffer.data_ptr(), nbytes,
                                     self.stream.cuda_stream, C.byref(h)))
        fac = Factors._wrap(p, self.precision, buffer, h)
        self.inflight[h.value] = (fac, eps)
        return fac

    def step(self, rounds: int = 1 << 30):
        """Enqueue up to `rounds` rounds; returns [(Factors, error or None)] of the
        geometries completed (a failed one is released)."""
        done = (C.c_void_p * 8)()
        status = (C.c_int32 * 8)()
        nd, na = C.c_int32(0), C.c_int32(0)
        with torch.cuda.stream(self.stream):
            check(lib.rcp_engine_step(self.handle, int(rounds), self.stream.cuda_stream, done,
                                      status, 8, C.byref(nd), C.byref(na)))
        out = []
        for i in range(nd.value):
            fac, _ = self.inflight.pop(done[i])
            err = None
            if status[i] != _lib.RCP_OK:
                err = RecipError(status[i], lib.rcp_last_error().decode())
                fac.release()
            out.append((fac, err))
        return out

    def run(self):
        """Drive every geometry in flight to completion; returns what step() does."""
        out = []
        while self.inflight:
            out += self.step()
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.rcp_engine_destroy(self.handle)
            self.handle = None
            for fac, _ in self.inflight.values():
                fac.release()
            self.inflight.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@_on_stream
def reciprocal_average(fac: Factors, p: Optional[Problem] = None, want_v: bool = False,
                       want_z: bool = False, symbol: Optional[torch.Tensor] = None, stream=None,
                       out: Optional[torch.Tensor] = None):
    """F = v^dag W v (Eq. 7) on device; returns F (0-d float64 tensor) [, v] [, z]."""
    p = p or fac.problem
    dev = fac.buf.device
    F = out if out is not None else torch.empty((), dtype=torch.float64, device=dev)
    v = torch.empty(p.m_aperture, dtype=torch.complex128, device=dev) if want_v else None
    z = torch.empty((p.nx, p.ny), dtype=torch.complex128, device=dev) if want_z else None
    o, lt = objective_struct(p), light_struct(p, symbol)
    check(lib.rcp_reciprocal_average(fac.handle, C.byref(o), C.byref(lt), F.data_ptr(),
                                     v.data_ptr() if v is not None else None,
                                     z.data_ptr() if z is not None else None, _stream(stream)))
    res = [F]
    if want_v:
        res.append(v)
    if want_z:
        res.append(z)
    return res[0] if len(res) == 1 else tuple(res)


@_on_stream
def brute_force_average(fac: Factors, nangles: int, p: Optional[Problem] = None,
                        rhs_chunk: Optional[int] = None, per_angle: bool = False, stream=None,
                        work: Optional[torch.Tensor] = None):
    """Eq. 6 by nangles-node Gauss-Legendre quadrature over forward solves."""
    p = p or fac.problem
    dev = fac.buf.device
    rhs_chunk = rhs_chunk or min(nangles, 256)
    need = int(lib.rcp_brute_force_work_bytes(fac.handle, nangles, rhs_chunk))
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    F = torch.empty((), dtype=torch.float64, device=dev)
    pa = torch.empty(nangles, dtype=torch.float64, device=dev) if per_angle else None
    o, lt = objective_struct(p), light_struct(p)
    check(lib.rcp_brute_force_average(fac.handle, C.byref(o), C.byref(lt), nangles, rhs_chunk,
                                      work.data_ptr(), need, F.data_ptr(),
                                      pa.data_ptr() if pa is not None else None, _stream(stream)))
    return (F, pa) if per_angle else F


@_on_stream
def adjoint_grad(fac: Factors, p: Optional[Problem] = None, stream=None):
    """(F, dF/deps) with dF/deps an nx x ny float64 map, from one extra solve."""
    p = p or fac.problem
    dev = fac.buf.device
    F = torch.empty((), dtype=torch.float64, device=dev)
    g = torch.empty((p.nx, p.ny), dtype=torch.float64, device=dev)
    o, lt = objective_struct(p), light_struct(p)
    check(lib.rcp_adjoint_grad(fac.handle, C.byref(o), C.byref(lt), F.data_ptr(), g.data_ptr(),
                               _stream(stream)))
    return F, g


@_on_stream
def adjoint_grad_batch(facs, problems=None, stream=None):
    """adjoint_grad for 1-8 factor sets of one grid (e.g. from factor_batch), their
    two solves advancing in the same kernel launches.  Returns (F of shape (B,),
    list of nx x ny dF/deps maps); each bit-identical to adjoint_grad."""
    B = len(facs)
    problems = problems or [f.problem for f in facs]
    if B < 1 or B > 8 or len(problems) != B:
        raise ValueError("adjoint_grad_batch takes 1 to 8 factor sets with one problem each")
    dev = facs[0].buf.device
    F = torch.empty(B, dtype=torch.float64, device=dev)
    grads = [torch.empty((p.nx, p.ny), dtype=torch.float64, device=dev) for p in problems]
    handles = (C.c_void_p * B)(*[f.handle.value for f in facs])
    objs = (_lib.Objective * B)(*[objective_struct(p) for p in problems])
    lights = (_lib.Light * B)(*[light_struct(p) for p in problems])
    gptr = (C.c_void_p * B)(*[g.data_ptr() for g in grads])
    check(lib.rcp_adjoint_grad_batch(B, handles, objs, lights, F.data_ptr(), gptr,
                                     _stream(stream)))
    return F, grads


@_on_stream
def reciprocal_average_many(fac: Factors, problems, stream=None,
                            work: Optional[torch.Tensor] = None) -> torch.Tensor:
    """F for several requests on the same factors (problems of this geometry with
    their own objectives and lights): one multi-RHS reciprocal sweep for all of
    them, then each one's Toeplitz form.  Returns F of shape (len(problems),)."""
    K = len(problems)
    if K < 1 or K > 64:
        raise ValueError("reciprocal_average_many takes 1 to 64 problems")
    dev = fac.buf.device
    need = int(lib.rcp_reciprocal_many_work_bytes(fac.handle, K))
    work = _work(need, dev, work)
    F = torch.empty(K, dtype=torch.float64, device=dev)
    objs = (_lib.Objective * K)(*[objective_struct(p) for p in problems])
    lights = (_lib.Light * K)(*[light_struct(p) for p in problems])
    check(lib.rcp_reciprocal_average_many(fac.handle, K, objs, lights, F.data_ptr(),
                                          work.data_ptr(), need, _stream(stream)))
    return F


@_on_stream
def broadband_grad(facs, weights, problems=None, stream=None):
    """Weighted sum over 1-8 factor sets (one geometry at the wavelengths of a
    spectral rule, e.g. from factor_batch): returns (F of shape (B + 1,) with the
    per-wavelength averages then the weighted sum, d(sum)/deps as nx x ny)."""
    B = len(facs)
    problems = problems or [f.problem for f in facs]
    if B < 1 or B > 8 or len(problems) != B or len(weights) != B:
        raise ValueError("broadband_grad takes 1 to 8 factor sets with one problem and weight each")
    dev = facs[0].buf.device
    p = problems[0]
    F = torch.empty(B + 1, dtype=torch.float64, device=dev)
    g = torch.empty((p.nx, p.ny), dtype=torch.float64, device=dev)
    handles = (C.c_void_p * B)(*[f.handle.value for f in facs])
    objs = (_lib.Objective * B)(*[objective_struct(q) for q in problems])
    lights = (_lib.Light * B)(*[light_struct(q) for q in problems])
    w = (C.c_double * B)(*[float(x) for x in weights])
    check(lib.rcp_broadband_grad(B, handles, objs, lights, w, F.data_ptr(), g.data_ptr(),
                                 _stream(stream)))
    return F, g


def _work(need: int, device, work: Optional[torch.Tensor]) -> torch.Tensor:
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=device)
    return work


@_on_stream
def correlation_matrix(p: Problem, thetas: torch.Tensor, C_amp: torch.Tensor, stream=None,
                       work: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Line correlation W = G C G^dag (M x M complex128) of a finite ensemble of
    planewaves at angles thetas with amplitude correlation C_amp (N x N)."""
    dev = C_amp.device
    th = thetas.to(device=dev, dtype=torch.float64).contiguous()
    Ca = C_amp.to(torch.complex128).contiguous()
    N = th.numel()
    if Ca.shape != (N, N):
        raise ValueError("C_amp must be N x N for N angles")
    M = p.m_aperture
    need = int(lib.rcp_correlation_work_bytes(M, N))
    if need == 0:
        raise RecipError(_lib.RCP_EINVAL, "invalid sizes for correlation_matrix")
    work = _work(need, dev, work)
    Wm = torch.empty((M, M), dtype=torch.complex128, device=dev)
    g, lt = grid_struct(p), light_struct(p)
    check(lib.rcp_correlation_matrix(C.byref(g), C.byref(lt), N, th.data_ptr(), Ca.data_ptr(),
                                     Wm.data_ptr(), work.data_ptr(), need, _stream(stream)))
    return Wm


def _dense_args(fac: Factors, outputs, W: torch.Tensor, p: Optional[Problem]):
    p = p or fac.problem
    K = len(outputs)
    Wc = W.to(torch.complex128).contiguous()
    if Wc.shape != (p.m_aperture, p.m_aperture):
        raise ValueError("W must be M x M on the incidence line")
    objs = (_lib.Objective * K)(*[objective_struct(o) for o in outputs])
    need = int(lib.rcp_dense_work_bytes(fac.handle, K, p.m_aperture))
    if need == 0:
        raise RecipError(_lib.RCP_EINVAL, "invalid sizes for the dense form")
    return p, K, Wc, objs, light_struct(p), need


@_on_stream
def reciprocal_average_dense(fac: Factors, outputs, W: torch.Tensor, p: Optional[Problem] = None,
                             want_v: bool = False, stream=None,
                             work: Optional[torch.Tensor] = None):
    """F_k = v_k^dag W v_k for each output (a list of problems that differ in the
    objective) and their sum: returns F of shape (K + 1,) [, V of shape (K, M)]."""
    p, K, Wc, objs, lt, need = _dense_args(fac, outputs, W, p)
    dev = fac.buf.device
    work = _work(need, dev, work)
    F = torch.empty(K + 1, dtype=torch.float64, device=dev)
    V = torch.empty((K, p.m_aperture), dtype=torch.complex128, device=dev) if want_v else None
    check(lib.rcp_reciprocal_average_dense(fac.handle, K, objs, C.byref(lt), Wc.data_ptr(),
                                           F.data_ptr(), V.data_ptr() if V is not None else None,
                                           work.data_ptr(), need, _stream(stream)))
    return (F, V) if want_v else F


@_on_stream
def adjoint_grad_dense(fac: Factors, outputs, W: torch.Tensor, p: Optional[Problem] = None,
                       stream=None, work: Optional[torch.Tensor] = None):
    """(F of shape (K + 1,), d(sum_k F_k)/deps as an nx x ny map)."""
    p, K, Wc, objs, lt, need = _dense_args(fac, outputs, W, p)
    dev = fac.buf.device
    work = _work(need, dev, work)
    F = torch.empty(K + 1, dtype=torch.float64, device=dev)
    g = torch.empty((p.nx, p.ny), dtype=torch.float64, device=dev)
    check(lib.rcp_adjoint_grad_dense(fac.handle, K, objs, C.byref(lt), Wc.data_ptr(), F.data_ptr(),
                                     g.data_ptr(), work.data_ptr(), need, _stream(stream)))
    return F, g


@_on_stream
def width_grad(p: Problem, grad_eps: torch.Tensor, widths: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
    """Chain rule dF/deps -> dF/dwidths (kernel, backward of eps_from_widths)."""
    dev = grad_eps.device
    pa = _PillarArgs(p, widths, dev)
    out = torch.empty(len(p.pillar_centers), dtype=torch.float64, device=dev)
    g = grid_struct(p)
    check(lib.rcp_width_grad(C.byref(g), C.byref(pa.struct), grad_eps.contiguous().data_ptr(),
                             out.data_ptr(), _stream(stream)))
    return out


@_on_stream
def solve(fac: Factors, B: torch.Tensor, conj_transpose: bool = False, tol: float = 1e-12,
          max_refine: int = 10, stream=None):
    """X = A^{-1} B (or A^{-dag} B) for B of shape (R, nx, ny) complex128."""
    B = B.to(torch.complex128).contiguous()
    if B.dim() == 2:
        B = B.unsqueeze(0)
    X = torch.empty_like(B)
    st = _lib.SolveStats()
    check(lib.rcp_solve_multi_rhs(fac.handle, B.shape[0], B.data_ptr(), X.data_ptr(),
                                  1 if conj_transpose else 0, tol, max_refine, _stream(stream),
                                  C.byref(st)))
    return X, (int(st.iters), float(st.rel_residual))


class IncoherentFOM(torch.autograd.Function):
    """Angle-averaged FOM as a differentiable function of the pillar widths or of
    the per-pixel permittivity.

    x is either the widths (1-D, one per pillar of the problem) or a permittivity
    map (nx x ny float64).
    forward: [widths -> eps (kernel)] -> factor -> F = v^dag W v
    backward: dF/deps from the adjoint solve (Sec. "Reciprocal approach"), and for
    widths the eps(widths) chain rule.
    """

    @staticmethod
    def forward(ctx, x: torch.Tensor, problem: Problem, precision: int = RCP_FP64):
        if x.dim() == 2:
            if tuple(x.shape) != (problem.nx, problem.ny):
                raise ValueError("a permittivity map must be nx x ny")
            eps = x.detach()
        elif x.dim() == 1:
            if x.numel() != len(problem.pillar_centers):
                raise ValueError("widths must hold one value per pillar")
            eps = eps_from_widths(problem, x, device=x.device)
        else:
            raise ValueError("x must be the widths (1-D) or a permittivity map (nx x ny)")
        fac = Factors(problem, eps, precision)
        if x.requires_grad:
            F, g = adjoint_grad(fac, problem)
            ctx.save_for_backward(g if x.dim() == 2 else width_grad(problem, g, x))
        else:
            F = reciprocal_average(fac, problem)
            ctx.save_for_backward(None)
        fac.release()
        return F

    @staticmethod
    def backward(ctx, grad_out):
        (gw,) = ctx.saved_tensors
        return (grad_out * gw if gw is not None else None), None, None


def kernel_timing_start(sample_every: int = 1) -> None:
    """Bracket every sample_every-th launch of each kernel class with HIP events."""
    check(lib.rcp_timing_start(int(sample_every)))


def kernel_timing_stop() -> dict:
    """Per kernel class: launches, timed samples, their total ms and algorithmic work."""
    arr = (_lib.KernelStat * _lib.NKCLASS)()
    check(lib.rcp_timing_stop(arr, _lib.NKCLASS))
    out = {}
    for name, st in zip(_lib.KCLASS_NAMES, arr):
        out[name] = dict(launches=int(st.launches), samples=int(st.samples), ms=float(st.ms),
                         work=float(st.work))
    return out
