"""Pins of the reference gradient (constant-rank pseudoinverse derivative)."""
import numpy as np
import pytest

from oracle import adjoint_ref as G


def _problem(seed, n, m, r):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, r)) @ rng.standard_normal((r, m))
    Y = rng.standard_normal(n)
    xt = rng.standard_normal(m)
    return A, Y, xt


@pytest.mark.parametrize("seed,n,m,r", [(0, 12, 8, 3), (1, 9, 9, 4), (2, 6, 10, 2), (3, 15, 5, 5)])
def test_closed_form_vs_fd_entries(seed, n, m, r):
    """Every entry of dL/dA and dL/dY against central FD through the
    rank-r truncated SVD solve, for L = 0.5 ||x - x_t||^2."""
    A, Y, xt = _problem(seed, n, m, r)
    loss = lambda x: 0.5 * float(np.sum((x - xt) ** 2))
    x = G.solve_rank(A, Y, r)
    dA, dY = G.grad_closed_form(A, Y, x - xt, r)
    ent = [(i, j) for i in range(n) for j in range(m)]
    fd = G.grad_fd(A, Y, loss, r, entries=ent).reshape(n, m)
    assert np.abs(fd - dA).max() <= 1e-6 * max(1.0, np.abs(dA).max())
    fdy = G.grad_fd_y(A, Y, loss, r)
    assert np.abs(fdy - dY).max() <= 1e-6 * max(1.0, np.abs(dY).max())


def test_full_rank_reduces_to_normal_equation_gradient():
    """Full column rank: x = (A^T A)^-1 A^T Y, and with S = (A^T A)^-1 g the
    textbook gradient is dL/dY = A S, dL/dA = (Y - A x) S^T - (A S) x^T."""
    A, Y, xt = _problem(7, 14, 6, 6)
    x = np.linalg.solve(A.T @ A, A.T @ Y)
    g = x - xt
    S = np.linalg.solve(A.T @ A, g)
    dA, dY = G.grad_closed_form(A, Y, g, 6)
    assert np.allclose(dY, A @ S, rtol=1e-10, atol=1e-12)
    assert np.allclose(dA, np.outer(Y - A @ x, S) - np.outer(A @ S, x), rtol=1e-9, atol=1e-11)


def test_dy_is_linear():
    """x is linear in Y, so dL/dY for a linear loss c^T x is exactly A^+T c."""
    A, Y, _ = _problem(8, 10, 7, 3)
    c = np.arange(7.0)
    _, dY = G.grad_closed_form(A, Y, c, 3)
    _, dY2 = G.grad_closed_form(A, 5.0 * Y - 2.0, c, 3)
    assert np.allclose(dY, dY2, rtol=1e-12, atol=1e-12)
    assert np.allclose(dY, G.pinv_rank(A, 3).T @ c, rtol=1e-12, atol=1e-12)


def test_directional_derivatives():
    A, Y, xt = _problem(9, 20, 12, 4)
    loss = lambda x: 0.5 * float(np.sum((x - xt) ** 2))
    x = G.solve_rank(A, Y, 4)
    dA, dY = G.grad_closed_form(A, Y, x - xt, 4)
    rng = np.random.default_rng(3)
    dirs = [(rng.standard_normal(A.shape), rng.standard_normal(Y.shape)) for _ in range(8)]
    fd = G.grad_fd(A, Y, loss, 4, directions=dirs)
    an = np.array([np.sum(dA * d) + np.sum(dY * e) for d, e in dirs])
    assert np.abs(fd - an).max() <= 1e-6 * max(1.0, np.abs(an).max())
