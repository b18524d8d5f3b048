"""Basis functions of the regularised adjoint-source estimate (Section 3.3).

The adjoint source is known only at the few frequencies omega_k, while the
stepping engine needs a time series.  The paper estimates it by minimising
    Psi = || s(omega) - B s(t') ||^2 + gamma || s(t') ||^2      (eq. B)
with the real 2Nw x Nt matrix B whose rows are the damped cosines and sines
of the transform (eq. dft) split into real and imaginary parts.  The
solution is s(t) = B+ s(omega), B+ = (B^T B + gamma I)^{-1} B^T
(eq. mpinv), and the columns b_k of B+ are the basis functions: the time
series for any receiver is sum_k Re s(omega_k) b_k + Im s(omega_k) b_{k+Nw}
(eq. basis).

Reading of the time grid: the rows of B are sampled at the times the
engine injects J', t_n = (n+1/2) dt, n = 0..Nt-1, so that the transform of
the injected series at z_k is exactly B s(t).

B+ has a plain definition, so the oracle evaluates that definition (the
paper reaches it iteratively with CGNR; the HIP library does, and is checked
against this).  Numerically it is computed from the thin SVD B = U S V^T as
B+ = V diag(S / (S^2 + gamma)) U^T, which is the same matrix.
"""
from __future__ import annotations

import numpy as np


def basis_matrix(a: np.ndarray, dt: float, nt: int) -> np.ndarray:
    """B [2Nw][Nt]: rows exp(-a_k t_n) cos(a_k t_n), then exp(-a_k t_n)
    sin(a_k t_n), a_k = sqrt(omega_k omega0), t_n = (n+1/2) dt (eq. B)."""
    t = (np.arange(nt) + 0.5) * dt
    at = np.outer(a, t)
    damp = np.exp(-at)
    return np.vstack([damp * np.cos(at), damp * np.sin(at)])


def gamma_from_rel(B: np.ndarray, gamma_rel: float) -> float:
    """Regularisation weight relative to the energy of B:
    gamma = gamma_rel * ||B||_F^2.  (Reading: the paper quotes an absolute
    gamma = 1e-3 for one Nt and dt; its scale follows ||B||^2, which grows
    with Nt and shrinks with dt.)"""
    return float(gamma_rel * np.sum(B * B))


def basis_pinv(B: np.ndarray, gamma: float) -> np.ndarray:
    """Rows are the 2Nw basis functions b_k (columns of B+, eq. mpinv)."""
    U, S, Vt = np.linalg.svd(B, full_matrices=False)
    filt = S / (S * S + gamma)
    Bp = (Vt.T * filt) @ U.T          # Nt x 2Nw
    return np.ascontiguousarray(Bp.T)


def synthesize(spec: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Time series from complex spectra spec[..., Nw] with the basis b
    [2Nw][Nt] (eq. basis)."""
    c = np.concatenate([spec.real, spec.imag], axis=-1)
    return c @ b
