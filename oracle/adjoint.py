"""Adjoint run and gradient with respect to ln(rho) (Section 3).

Misfit (eq. phid): phi = 1/2 || W (d - R u) ||^2.  The adjoint field obeys
A^T conj(v) = conj(R^T W^T W (d - R u)) (eq. adj1), which the same stepping
engine solves because A^T = A.  Reading of eq. adj2: the electric residual
is an electric current source, placed in the J' slot with the factor
sqrt(-i omega / 2 omega0), the same map that turns J into J' in the forward
problem (the printed equation puts it on the curl E row; only this reading
matches the gradient formula eq. gradsigmaij and the finite-difference
check).  The adjoint spectrum at each receiver is turned into a time series
with the basis functions (eq. basis) and injected there.

Magnetic data (receiver components 3-5, weighted by W2 in eq. phid) follow
from the same reading: the magnetic residual is a magnetic current source in
the M' slot.  The forward field is H = u_H / W_k (M' = M and H' = sqrt(-i
w/2w0) H leave no factor), so its adjoint spectrum is conj(resid) alone
against the electric sqrt(-i w/2w0) conj(resid) (the common 1/W_k is
carried by the normalised forward field in the gradient).  M' acts at n dt
while the basis functions are built on the injection times (n+1/2) dt of
J': a series with sum_n b^n z^{n+1/2} = c has sum_n b^n z^n = c z^{-1/2},
so the magnetic coefficients are conj(resid) z^{1/2}.  The node weights are
w / (dual volume of the H node), the weights under which the discrete
Faraday and Ampere rows form a symmetric system.

Gradient (eq. gradsigmaij, isotropic case; cell volume scaling as the text
after eq. adj0 allows): on every E edge
    d phi / d sigma_e = - Re sum_s sum_k (Omega_k / w'_k) conj(E_adj)_e E_e dV_e
where conj(E_adj) is what the engine computes and the factor
Omega_k / w'_k = sin(w'_k dt/2) / (w'_k dt/2) turns the continuous-time
expression into the derivative of the discrete stepped system (reading:
the paper's formula is its dt -> 0 limit).  Edge values are mapped to cells
by the transpose of the conductivity averaging, and the ln(rho) chain rule
(Section 3.5) gives d phi / d ln rho = - sigma d phi / d sigma.
"""
from __future__ import annotations

import numpy as np

from .basis import basis_matrix, basis_pinv, gamma_from_rel, synthesize
from .discretization import Setup, cell_gradient, dual_volumes, edge_sigma_transpose, h_volumes
from .stepping import point_entries, run_stepping


def misfit(E: np.ndarray, d: np.ndarray, W: np.ndarray | float = 1.0) -> float:
    """phi_d = 1/2 sum |W (d - E)|^2 (eq. phid, over whichever electric and
    magnetic components the data hold)."""
    return 0.5 * float(np.sum(np.abs(W * (d - E)) ** 2))


def source_factors(s: Setup, rec_comp) -> np.ndarray:
    """Per component and frequency, the factor between conj(resid) and the
    coefficients handed to the basis functions [ncomp][nf]: sqrt(-i w/2w0)
    for E (the J' slot), z^{1/2} for H (the M' slot, acting at n dt)."""
    magnetic = np.asarray(rec_comp) >= 3
    fac_e = np.sqrt(-1j * s.omega / (2.0 * s.omega0))
    fac_h = np.exp(0.5j * s.wprime * s.dt)
    return np.where(magnetic[:, None], fac_h[None, :], fac_e[None, :])


def adjoint_sources(s: Setup, rec_pos, rec_comp, resid_s: np.ndarray,
                    b: np.ndarray):
    """Injection entries and time series of the adjoint sources of one
    forward source.  resid_s [nr][ncomp][nf] is the weighted residual
    W^2 (d - E).  Returns (entries, series [nr * ncomp][nt], coefficients
    [nr][ncomp][nf] handed to the basis functions)."""
    spec = source_factors(s, rec_comp)[None] * np.conj(resid_s)
    ts = synthesize(spec, b)                    # [nr][ncomp][nt]
    vols = dual_volumes(s) + h_volumes(s)
    inj = []
    ncomp = len(rec_comp)
    for r, pos in enumerate(rec_pos):
        for ci, c in enumerate(rec_comp):
            row = r * ncomp + ci
            for (k, j, i, w) in point_entries(s, c, pos):
                inj.append((c, k, j, i, w / vols[c][k, j, i], row))
    return inj, ts.reshape(len(rec_pos) * ncomp, -1), spec


def adjoint_gradient(p, fwd: dict, resid: np.ndarray, gamma_rel: float = 1e-12,
                     gamma_abs: float = 0.0, probe_nodes: list | None = None):
    """Gradient of phi_d with respect to ln(rho) for every cell.

    fwd    output of ``stepping.forward(p, want_volume=True)``; its volume
           transform may be decimated (stepping.run_stepping), the adjoint
           transform never is: the adjoint sources built from the basis
           functions start at full amplitude and fall within a few steps,
           so a decimated adjoint transform would alias
    resid  weighted residual W^2 (d - E) [ns][nr][ncomp][nf]
    Returns dict(grad [nz][ny][nx], grad_edges (gx, gy, gz), basis, fit,
    probe [ns][len(probe_nodes)][nf] raw adjoint transforms at probe_nodes)."""
    s: Setup = fwd["setup"]
    B = basis_matrix(s.a, s.dt, s.nt)
    gamma = gamma_abs if gamma_abs > 0.0 else gamma_from_rel(B, gamma_rel)
    b = basis_pinv(B, gamma)
    fit = float(np.max(np.abs(B @ b.T - np.eye(B.shape[0]))))
    vols = dual_volumes(s)
    corr = s.Omega / s.wprime                    # discrete-time factor
    gx = np.zeros(vols[0].shape)
    gy = np.zeros(vols[1].shape)
    gz = np.zeros(vols[2].shape)
    probes = []
    for si in range(len(p.src_pos)):
        inj, ts, _ = adjoint_sources(s, p.rec_pos, p.rec_comp, resid[si], b)
        acc, v = run_stepping(s, inj, ts, probe_nodes or [], True)
        probes.append(acc)
        E = fwd["vol"][si]
        for c, g in enumerate((gx, gy, gz)):
            prod = np.einsum("k,k...->...", corr, v[c] * E[c])
            g -= np.real(prod) * vols[c]
    g_sigma = edge_sigma_transpose(gx, gy, gz, s.hx, s.hy, s.hz)
    # capped cells do not see rho; in VTI the x, y edges give rho_h, the z
    # edges rho_v (Section 3.1); grad = d / d ln rho with rho_h, rho_v scaled
    # together
    grad_h, grad_v = cell_gradient(s, gx, gy, gz)
    return {"grad": grad_h + grad_v, "grad_h": grad_h, "grad_v": grad_v,
            "grad_sigma": g_sigma, "grad_edges": (gx, gy, gz),
            "basis": b, "B": B, "gamma": gamma, "fit": fit,
            "probe": np.array(probes)}
