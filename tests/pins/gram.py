"""Closed form of the Gram matrix B B^T of the adjoint-source estimate, a pin
that does not build B.

The rows of B (eq. B) are Re q_k^{t_n/dt} and Im q_k^{t_n/dt} with
q_k = exp((-a_k + i a_k) dt), t_n = (n+1/2) dt.  With u = q_j^{n+1/2},
v = q_k^{n+1/2}:
    Re u Re v = (Re(uv) + Re(u conj v)) / 2
    Im u Im v = (Re(u conj v) - Re(uv)) / 2
    Re u Im v = (Im(uv) - Im(u conj v)) / 2
and each sum over n is a geometric sum
    S(zeta) = sum_{n=0}^{Nt-1} zeta^{n+1/2} = zeta^{1/2} (1 - zeta^Nt)/(1 - zeta).
"""
from __future__ import annotations

import numpy as np


def geometric(zeta, nt):
    return np.sqrt(zeta) * (1.0 - zeta ** nt) / (1.0 - zeta)


def gram(a, dt, nt):
    a = np.asarray(a, dtype=np.float64)
    nf = len(a)
    q = np.exp((-a + 1j * a) * dt)
    G = np.zeros((2 * nf, 2 * nf))
    for j in range(nf):
        for k in range(nf):
            s1 = geometric(q[j] * q[k], nt)
            s2 = geometric(q[j] * np.conj(q[k]), nt)
            G[j, k] = 0.5 * (s1.real + s2.real)                  # cos . cos
            G[nf + j, nf + k] = 0.5 * (s2.real - s1.real)        # sin . sin
            G[j, nf + k] = 0.5 * (s1.imag - s2.imag)             # cos_j . sin_k
            G[nf + k, j] = G[j, nf + k]
    return G
