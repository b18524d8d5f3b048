"""Pins of the oracle's inversion driver (Section 3.5) and the host-side
agreement of the library's driver with it.

The oracle's regularisation is pinned by the closed form of a linear ramp
(phi_m = 1/2 sum_d alpha_d^2 c_d^2 n_faces_d, gradient only on the first and
last cell of each line), by an explicit loop over faces and by central
differences; its dense BFGS matrix by the secant condition, symmetry and
positive definiteness; the optimiser by the known minimisers of bounded and
regularised quadratics (the latter solved densely with a face-loop
Laplacian) and by the restart rule.  The library's driver (two-loop
recursion, no dense matrix) then has to follow the same iterates.
"""
import numpy as np
import pytest

from oracle import inversion as oinv
from paper_2211_16665_amd import inversion as inv


def test_roughness_of_a_linear_ramp():
    nz, ny, nx = 4, 5, 6
    c = (0.3, -0.7, 1.1)                           # slope per cell along x, y, z
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = c[0] * i + c[1] * j + c[2] * k
    alpha = (1.0, 0.5, 0.2)
    val, g = oinv.roughness(m, np.zeros_like(m), alpha)
    faces = ((nx - 1) * ny * nz, nx * (ny - 1) * nz, nx * ny * (nz - 1))
    assert np.isclose(val, 0.5 * sum(a * a * s * s * f for a, s, f in zip(alpha, c, faces)),
                      rtol=1e-13)
    ref = np.zeros_like(m)
    ref[:, :, 0] -= alpha[0] ** 2 * c[0]
    ref[:, :, -1] += alpha[0] ** 2 * c[0]
    ref[:, 0, :] -= alpha[1] ** 2 * c[1]
    ref[:, -1, :] += alpha[1] ** 2 * c[1]
    ref[0] -= alpha[2] ** 2 * c[2]
    ref[-1] += alpha[2] ** 2 * c[2]
    assert np.allclose(g, ref, atol=1e-13)


def _face_loop_laplacian(shape, alpha):
    nz, ny, nx = shape
    n = nz * ny * nx
    L = np.zeros((n, n))
    lin = lambda k, j, i: (k * ny + j) * nx + i           # noqa: E731
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for a, (dk, dj, di) in ((alpha[0], (0, 0, 1)), (alpha[1], (0, 1, 0)),
                                        (alpha[2], (1, 0, 0))):
                    if k + dk < nz and j + dj < ny and i + di < nx:
                        p, q = lin(k, j, i), lin(k + dk, j + dj, i + di)
                        w = a * a
                        L[p, p] += w
                        L[q, q] += w
                        L[p, q] -= w
                        L[q, p] -= w
    return L


def test_roughness_against_face_loops_and_finite_differences():
    rng = np.random.default_rng(5)
    shape = (3, 4, 5)
    m, mref = rng.standard_normal(shape), rng.standard_normal(shape)
    alpha = (0.9, 1.3, 0.4)
    L = _face_loop_laplacian(shape, alpha)
    u = (m - mref).ravel()
    val, g = oinv.roughness(m, mref, alpha)
    assert np.isclose(val, 0.5 * u @ L @ u, rtol=1e-13)
    assert np.allclose(g.ravel(), L @ u, atol=1e-13)
    h = 1e-6
    for c in [(0, 0, 0), (1, 2, 3), (2, 3, 4)]:
        mp, mm = m.copy(), m.copy()
        mp[c] += h
        mm[c] -= h
        fd = (oinv.roughness(mp, mref, alpha)[0] - oinv.roughness(mm, mref, alpha)[0]) / (2 * h)
        assert abs(fd - g[c]) < 1e-7 * max(1.0, abs(fd))
    # two parameters are regularised independently
    v2, g2 = oinv.roughness(np.stack([m, m]), np.stack([mref, mref]), alpha)
    assert np.isclose(v2, 2 * val) and np.allclose(g2[0], g) and np.allclose(g2[1], g)


@pytest.mark.parametrize("with_d", [False, True])
def test_bfgs_matrix_secant_symmetry_definiteness(with_d):
    rng = np.random.default_rng(6)
    n = 15
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(5)]
    Y = [A @ s for s in S]
    D = rng.uniform(0.5, 3.0, n) if with_d else None
    H = oinv.bfgs_inverse_hessian(S, Y, D)
    assert np.allclose(H @ Y[-1], S[-1], rtol=1e-11, atol=1e-12)      # secant condition
    assert np.allclose(H, H.T, atol=1e-13)
    assert np.linalg.eigvalsh(H).min() > 0.0
    # one pair: H0 = gamma diag(D), with gamma = s'y / y'D y
    d = np.ones(n) if D is None else D
    H1 = oinv.bfgs_inverse_hessian(S[-1:], Y[-1:], D)
    s, y = S[-1], Y[-1]
    gamma = (s @ y) / (y @ (d * y))
    # on vectors z with s'z = 0 and y'D z = 0 the update leaves H0 alone
    M = np.stack([s, d * y], axis=1)
    z = rng.standard_normal(n)
    z -= M @ np.linalg.lstsq(M, z, rcond=None)[0]
    assert abs(s @ z) < 1e-12 and abs(y @ (d * z)) < 1e-10
    assert np.allclose(H1 @ z, gamma * d * z, rtol=1e-11, atol=1e-12)
    assert np.allclose(H1 @ y, s, rtol=1e-11, atol=1e-12)


def _quad(A, b):
    def term(m):
        x = m.ravel()
        return 0.5 * x @ A @ x - b @ x, (A @ x - b).reshape(m.shape)
    return term


def test_oracle_driver_reaches_known_minimisers():
    rng = np.random.default_rng(7)
    shape = (2, 3, 4)
    n = 24
    d = rng.uniform(1.0, 3.0, n)
    target = rng.uniform(-2.0, 2.0, n)
    A = np.diag(d)
    b = d * target
    act = np.ones(shape, bool)
    r = oinv.invert(_quad(A, b), np.zeros(shape), act, np.zeros(n), beta=0.0, max_iter=80,
                    m_min=-1.0, m_max=1.0, first_step=0.5)
    assert np.allclose(r["x"], np.clip(target, -1, 1), atol=1e-5)
    beta, alpha = 0.3, (1.0, 0.5, 0.2)
    xs = np.linalg.solve(A + beta * _face_loop_laplacian(shape, alpha), b)
    r = oinv.invert(_quad(A, b), np.zeros(shape), act, np.zeros(n), alpha=alpha, beta=beta,
                    max_iter=80, first_step=0.5)
    assert np.allclose(r["x"], xs, atol=1e-6)
    phis = [h["phi"] for h in r["history"]]
    assert all(q <= p + 1e-15 for p, q in zip(phis, phis[1:]))


def test_oracle_restart_rule():
    n = 10
    A = np.diag(np.linspace(1.0, 4.0, n))
    quad = _quad(A, np.ones(n))
    calls = {"n": 0}

    def wrong_late(m):
        calls["n"] += 1
        f, g = quad(m)
        return f, (-g if calls["n"] > 4 else g)
    r = oinv.invert(wrong_late, np.zeros((1, 1, n)), np.ones((1, 1, n), bool), np.zeros(n),
                    max_iter=20, first_step=0.2, max_backtracks=4)
    assert r["restarts"] == 1
    assert sum(1 for h in r["history"] if h["restart"]) == 1
    assert len(r["history"]) < 20


@pytest.mark.parametrize("case", ["plain", "bounds+cooling", "precond+partial"])
def test_library_driver_follows_the_oracle(case):
    """The library's driver (two-loop, host vectors) takes the same steps as
    the dense oracle on a nonlinear objective: every history entry and the
    final model agree to rounding."""
    rng = np.random.default_rng(8)
    shape = (3, 4, 5)
    n_all = 60
    Q = rng.standard_normal((n_all, n_all))
    A = Q @ Q.T / n_all + np.eye(n_all)
    b = rng.standard_normal(n_all)

    def term(m):                                   # quadratic plus a quartic bump
        x = m.ravel()
        f = 0.5 * x @ A @ x - b @ x + 0.05 * np.sum(x ** 4)
        return f, (A @ x - b + 0.2 * x ** 3).reshape(m.shape)
    mref = 0.1 * rng.standard_normal(shape)
    act = np.ones(shape, bool)
    kw = dict(max_iter=12, memory=4, first_step=0.4)
    if case == "bounds+cooling":
        kw.update(m_min=-0.5, m_max=0.6, cooling=0.7)
    if case == "precond+partial":
        act[0] = False
        D = inv.depth_preconditioner(np.arange(4.0) * 100.0, shape, depth0=100.0)[act]
        kw["precond"] = D
    n = int(act.sum())
    x0 = np.zeros(n)
    obj = inv.Objective(term, mref, active=act, alpha=(1.0, 0.8, 0.3), beta=0.2)
    res = inv.lbfgs(obj, x0, **kw)
    ref = oinv.invert(term, mref, act, x0, alpha=(1.0, 0.8, 0.3), beta=0.2, **kw)
    assert len(res.history) == len(ref["history"])
    for h, o in zip(res.history, ref["history"]):
        assert h["step"] == o["step"] and h["restart"] == o["restart"]
        assert np.isclose(h["phi"], o["phi"], rtol=1e-11, atol=1e-13)
    assert np.allclose(res.m, ref["m"], rtol=1e-9, atol=1e-11)
    assert res.evaluations == ref["evaluations"]
