"""Pins of the inversion driver (Section 3.5) on the CPU.

The regularisation is checked against a brute-force sum over faces and
central differences; the l-BFGS two-loop recursion against the explicit
dense BFGS inverse-Hessian update of the same pairs; the optimiser against
the known minimiser of bounded quadratics; the restart rule (steepest
descent after the first line-search failure, stop after the second) with an
objective whose gradient turns wrong.
"""
import numpy as np

from paper_2211_16665_amd import inversion as inv


def test_roughness_against_brute_force_and_finite_differences():
    rng = np.random.default_rng(0)
    m = rng.standard_normal((4, 5, 6))
    mref = rng.standard_normal((4, 5, 6))
    alpha = (1.0, 0.7, 0.1)
    val, g = inv.roughness(m, mref, alpha)
    u = m - mref
    ref = 0.0
    nz, ny, nx = u.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if i + 1 < nx:
                    ref += 0.5 * alpha[0] ** 2 * (u[k, j, i + 1] - u[k, j, i]) ** 2
                if j + 1 < ny:
                    ref += 0.5 * alpha[1] ** 2 * (u[k, j + 1, i] - u[k, j, i]) ** 2
                if k + 1 < nz:
                    ref += 0.5 * alpha[2] ** 2 * (u[k + 1, j, i] - u[k, j, i]) ** 2
    assert np.isclose(val, ref, rtol=1e-13)
    h = 1e-6
    for c in [(0, 0, 0), (2, 3, 4), (3, 4, 5), (1, 2, 0)]:
        mp, mm = m.copy(), m.copy()
        mp[c] += h
        mm[c] -= h
        fd = (inv.roughness(mp, mref, alpha)[0] - inv.roughness(mm, mref, alpha)[0]) / (2 * h)
        assert abs(fd - g[c]) < 1e-7 * max(1.0, abs(fd))
    # two parameters (VTI) are regularised independently
    val2, g2 = inv.roughness(np.stack([m, 2 * m]), np.stack([mref, 2 * mref]), alpha)
    assert np.isclose(val2, 5 * val) and np.allclose(g2[1], 2 * g)


def test_two_loop_equals_dense_bfgs():
    """For the same pairs, the two-loop recursion applies exactly the BFGS
    inverse-Hessian built by the dense update H <- (I - r s y') H (I - r y s')
    + r s s' from H0 = gamma I."""
    rng = np.random.default_rng(1)
    n, k = 12, 5
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(k)]
    Y = [A @ s for s in S]
    g = rng.standard_normal(n)
    gamma = S[-1] @ Y[-1] / (Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    I = np.eye(n)
    for s, y in zip(S, Y):
        r = 1.0 / (y @ s)
        H = (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)
    assert np.allclose(inv.two_loop(g, S, Y), H @ g, rtol=1e-11, atol=1e-12)


def _quadratic(A, b):
    def term(m):
        x = m.ravel()
        return 0.5 * x @ A @ x - b @ x, (A @ x - b).reshape(m.shape)
    return term


def test_lbfgs_reaches_the_minimiser_of_a_quadratic():
    rng = np.random.default_rng(2)
    n = 3 * 4 * 5
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T / n + np.eye(n)
    b = rng.standard_normal(n)
    obj = inv.Objective(_quadratic(A, b), np.zeros((3, 4, 5)), beta=0.0)
    res = inv.lbfgs(obj, np.zeros(n), max_iter=60, memory=8, first_step=0.5)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(res.m.ravel() - xs) < 1e-6 * np.linalg.norm(xs)
    phis = [h["phi"] for h in res.history]
    assert all(b2 <= a2 + 1e-15 for a2, b2 in zip(phis, phis[1:]))   # monotone


def test_lbfgs_with_bounds_and_regularisation():
    """A diagonal quadratic whose minimiser lies partly outside the bounds:
    the projected iteration ends at the clipped minimiser; with beta > 0 the
    minimiser of phi_d + beta phi_m (solved densely) is reached."""
    rng = np.random.default_rng(3)
    shape = (2, 3, 4)
    n = 24
    d = rng.uniform(1.0, 3.0, n)
    target = rng.uniform(-2.0, 2.0, n)
    A = np.diag(d)
    b = d * target
    obj = inv.Objective(_quadratic(A, b), np.zeros(shape), beta=0.0)
    res = inv.lbfgs(obj, np.zeros(n), max_iter=80, m_min=-1.0, m_max=1.0, first_step=0.5)
    assert np.allclose(res.m.ravel(), np.clip(target, -1, 1), atol=1e-5)
    # regularised, unbounded: (A + beta L) x = b with L the roughness Hessian
    beta, alpha = 0.3, (1.0, 0.5, 0.2)
    L = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        L[:, i] = inv.roughness(e.reshape(shape), np.zeros(shape), alpha)[1].ravel()
    xs = np.linalg.solve(A + beta * L, b)
    obj = inv.Objective(_quadratic(A, b), np.zeros(shape), alpha=alpha, beta=beta)
    res = inv.lbfgs(obj, np.zeros(n), max_iter=80, first_step=0.5)
    assert np.allclose(res.m.ravel(), xs, atol=1e-6)


def test_restart_after_the_first_line_search_failure():
    """The gradient turns wrong (sign flipped) after a few evaluations: the
    l-BFGS step fails its line search, the driver restarts once from the
    steepest-descent direction of the (wrong) gradient, fails again and
    stops; the misfit never increases."""
    n = 10
    A = np.diag(np.linspace(1.0, 4.0, n))
    b = np.ones(n)
    calls = {"n": 0}
    quad = _quadratic(A, b)

    def wrong_late(m):
        calls["n"] += 1
        f, g = quad(m)
        return f, (-g if calls["n"] > 4 else g)
    obj = inv.Objective(wrong_late, np.zeros((1, 1, n)), beta=0.0)
    res = inv.lbfgs(obj, np.zeros(n), max_iter=20, first_step=0.2, max_backtracks=4)
    assert res.restarts == 1
    assert sum(1 for h in res.history if h["restart"]) == 1
    phis = [h["phi"] for h in res.history]
    assert all(b2 <= a2 + 1e-15 for a2, b2 in zip(phis, phis[1:]))
    assert len(res.history) < 20


def test_preconditioned_lbfgs_keeps_the_minimiser():
    """A diagonal initial inverse Hessian changes the path, not the
    minimiser; the two-loop with D equals dense BFGS from H0 = gamma D."""
    rng = np.random.default_rng(4)
    n = 30
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T / n + np.diag(np.linspace(1.0, 20.0, n))
    b = rng.standard_normal(n)
    D = np.linspace(1.0, 10.0, n)
    obj = inv.Objective(_quadratic(A, b), np.zeros((1, 1, n)), beta=0.0)
    res = inv.lbfgs(obj, np.zeros(n), max_iter=80, memory=6, first_step=0.3, precond=D)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(res.m.ravel() - xs) < 1e-6 * np.linalg.norm(xs)
    S = [rng.standard_normal(n) for _ in range(4)]
    Y = [A @ s for s in S]
    g = rng.standard_normal(n)
    H = (S[-1] @ Y[-1] / (Y[-1] @ (D * Y[-1]))) * np.diag(D)
    I = np.eye(n)
    for s, y in zip(S, Y):
        r = 1.0 / (y @ s)
        H = (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)
    assert np.allclose(inv.two_loop(g, S, Y, D), H @ g, rtol=1e-11, atol=1e-12)


def test_depth_preconditioner():
    z = np.array([-200.0, -100.0, 0.0, 100.0, 300.0])
    P = inv.depth_preconditioner(z, (2, 4, 3, 2), depth0=100.0, power=2.0)
    f = (1.0 + np.maximum(np.array([-150.0, -50.0, 50.0, 200.0]), 0.0) / 100.0) ** 2
    assert P.shape == (2, 4, 3, 2)
    assert np.allclose(P[1, :, 2, 1], f) and np.allclose(P[0, :, 0, 0], f)
