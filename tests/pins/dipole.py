"""Closed-form field of an electric dipole in a homogeneous conductive
whole space (quasi-static, e^{-i omega t}); a pin for the oracle that shares
nothing with it.

With the paper's convention (eq. freq: curl H - sigma E = J, d/dt <-> -i w)
the electric field obeys curl curl E - k^2 E = i w mu J with k^2 = i w mu
sigma, Im k > 0.  For J = p delta(x) its solution is
    E = (1/sigma) (k^2 I + grad grad) G p,   G = e^{ikr} / (4 pi r),
which written out is
    E_i = G/(sigma r^2) [ (x_i x_j / r^2)(3 - 3ikr - k^2 r^2)
                          + delta_ij (ikr - 1 + k^2 r^2) ] p_j.
The magnetic field is H = curl (G p) = G'(r) (r_hat x p) with
G' = (ik - 1/r) G; then curl E = (k^2 / sigma) H = i omega mu H, the
Faraday row of eq. freq with M = 0.
"""
from __future__ import annotations

import numpy as np

MU0 = 4.0e-7 * np.pi


def wavenumber(omega, sigma, mu=MU0):
    """k = sqrt(i omega mu sigma) on the branch with Im k > 0."""
    k = np.sqrt(1j * omega * mu * sigma + 0j)
    return np.where(np.imag(k) < 0, -k, k)


def dipole_field(r_vec, p, k, sigma):
    """E at offsets ``r_vec`` [..., 3] from a dipole of moment ``p`` [3] in a
    whole space of conductivity ``sigma`` with wavenumber ``k``."""
    r_vec = np.asarray(r_vec, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    r = np.linalg.norm(r_vec, axis=-1)
    G = np.exp(1j * k * r) / (4.0 * np.pi * r)
    kr = k * r
    rp = np.einsum("...i,i->...", r_vec, p)
    a = (3.0 - 3.0j * kr - kr * kr) / r ** 2
    b = 1j * kr - 1.0 + kr * kr
    return (G / (sigma * r * r))[..., None] * (a[..., None] * rp[..., None] * r_vec
                                               + b[..., None] * p)


def dipole_field_discrete_time(r_vec, p, sigma, omega, omega0, Omega, mu=MU0):
    """The same closed form with the temporal discretisation of the leapfrog
    folded in: the stepped system at complex frequency Omega obeys
    curl curl E - (Omega^2 mu sigma / 2 omega0) E = i Omega mu J' with
    J' = sqrt(-i omega / 2 omega0) J, so the whole-space solution is the
    formula above with k^2 = Omega^2 mu sigma / (2 omega0) and an overall
    factor w'/Omega, w' = (1+i) sqrt(omega omega0)."""
    k = np.sqrt(Omega ** 2 * mu * sigma / (2.0 * omega0) + 0j)
    k = np.where(np.imag(k) < 0, -k, k)
    wp = (1.0 + 1.0j) * np.sqrt(omega * omega0)
    return (wp / Omega) * dipole_field(r_vec, p, k, sigma)


def magnetic_field(r_vec, p, k):
    """H at offsets ``r_vec`` [..., 3] from an electric dipole of moment
    ``p`` [3] with wavenumber ``k``: (ik - 1/r) G (r_hat x p)."""
    r_vec = np.asarray(r_vec, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    r = np.linalg.norm(r_vec, axis=-1)
    G = np.exp(1j * k * r) / (4.0 * np.pi * r)
    dG = (1j * k - 1.0 / r) * G
    return (dG / r)[..., None] * np.cross(r_vec, p)


def magnetic_field_discrete_time(r_vec, p, sigma, omega0, Omega, mu=MU0):
    """H of the stepped system at complex frequency Omega.  The Faraday row
    of the stepped system gives H' = curl E' / (i Omega mu); with E' from
    dipole_field_discrete_time and H = H' / sqrt(-i omega / 2 omega0) every
    factor cancels: H is the closed form above at k^2 = Omega^2 mu sigma /
    (2 omega0)."""
    k = np.sqrt(Omega ** 2 * mu * sigma / (2.0 * omega0) + 0j)
    k = np.where(np.imag(k) < 0, -k, k)
    return magnetic_field(r_vec, p, k)


def magnetic_dipole_e(r_vec, m, k):
    """E at offsets ``r_vec`` [..., 3] from a magnetic dipole of moment ``m``
    [3] (M = m delta(x) in the Faraday row of eq. freq).  Taking the curl of
    that row, curl curl E - k^2 E = curl M; E is divergence-free, so
    (lap + k^2) E = -curl M and E = curl (G m) = grad G x m =
    (ik - 1/r) G (r_hat x m)."""
    r_vec = np.asarray(r_vec, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    r = np.linalg.norm(r_vec, axis=-1)
    G = np.exp(1j * k * r) / (4.0 * np.pi * r)
    dG = (1j * k - 1.0 / r) * G
    return (dG / r)[..., None] * np.cross(r_vec, m)


def magnetic_dipole_h(r_vec, m, k, sigma, omega, mu=MU0):
    """H of the same magnetic dipole away from it: from the Faraday row,
    i omega mu H = curl E = curl curl (G m) = (k^2 + grad div) (G m), which is
    sigma times the electric dipole's E of moment m (dipole_field)."""
    return sigma / (1j * omega * mu) * dipole_field(r_vec, m, k, sigma)


def magnetic_dipole_discrete_time(r_vec, m, sigma, omega, omega0, Omega, mu=MU0):
    """(E, H) of a magnetic dipole in the stepped system at complex frequency
    Omega.  Its transformed rows are curl E^ - i Omega mu H^ = M^ and
    curl H^ + i Omega eps E^ = J^ (eps = sigma / 2 omega0); with M' = M and
    J = 0, E^ solves curl curl E^ - (Omega^2 mu sigma / 2 omega0) E^ = curl M^,
    the closed form above with k^2 = Omega^2 mu sigma / (2 omega0) and no
    other factor.  H' = H^ = sigma dipole_field(m) / (i Omega mu) away from
    the source, and H = H' / sqrt(-i omega / 2 omega0)."""
    k = np.sqrt(Omega ** 2 * mu * sigma / (2.0 * omega0) + 0j)
    k = np.where(np.imag(k) < 0, -k, k)
    E = magnetic_dipole_e(r_vec, m, k)
    Hp = sigma / (1j * Omega * mu) * dipole_field(r_vec, m, k, sigma)
    return E, Hp / np.sqrt(-1j * omega / (2.0 * omega0))
