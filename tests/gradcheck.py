"""Gradient comparison used by the GPU parity tests.

Two criteria, both required: the relative 2-norm of the difference, and a
per-component bound |g_i - r_i| <= tol * max(|r_i|, 1e-3 ||r||_inf), so that an
error confined to a few cells (pillar edges, PML rows) cannot hide under a norm
that the large components near the focus control.
"""
import numpy as np


def grad_errors(g, ref):
    g = np.asarray(g).ravel()
    ref = np.asarray(ref).ravel()
    d = np.abs(g - ref)
    norm = float(np.linalg.norm(d) / np.linalg.norm(ref))
    floor = 1e-3 * np.abs(ref).max()
    comp = float(np.max(d / np.maximum(np.abs(ref), floor)))
    return norm, comp


def assert_grad_close(g, ref, norm_tol, comp_tol=1e-5):
    norm, comp = grad_errors(g, ref)
    assert norm < norm_tol, f"gradient 2-norm error {norm:.3e} >= {norm_tol:.1e}"
    assert comp < comp_tol, f"gradient per-component error {comp:.3e} >= {comp_tol:.1e}"
