"""Reference gradients of x = A^+ Y at constant rank (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper does not differentiate the solve.  The reading used here: the
derivative is the one of the rank-r truncated pseudoinverse, i.e. the rank is
held fixed (Golub and Pereyra, 1973):

  dA^+ = -A^+ dA A^+ + A^+ A^+T dA^T (I - A A^+) + (I - A^+ A) dA^T A^+T A^+.

For a loss L(x) with g = dL/dx and x = A^+ Y this gives

  dL/dY = A^+T g
  dL/dA = -(A^+T g) x^T + rho (A^+ A^+T g)^T + (A^+T x) ((I - A^+ A) g)^T,

with rho = Y - A x.  ``grad_closed_form`` evaluates these with A^+ from a
truncated SVD.  ``grad_fd`` is the plain definition: central differences of
L(A^+_r Y) where A^+_r is the rank-r truncated SVD pseudoinverse.
"""
import numpy as np


def pinv_rank(A, rank):
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    return (Vt[:rank].T / s[:rank]) @ U[:, :rank].T


def solve_rank(A, Y, rank):
    return pinv_rank(A, rank) @ np.asarray(Y, dtype=np.float64)


def grad_closed_form(A, Y, g, rank):
    """(dL/dA, dL/dY) for the given upstream gradient g = dL/dx."""
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    Ap = pinv_rank(A, rank)
    x = Ap @ Y
    rho = Y - A @ x
    a = Ap.T @ g
    s = Ap @ a
    p = g - Ap @ (A @ g)
    t = Ap.T @ x
    dA = -np.outer(a, x) + np.outer(rho, s) + np.outer(t, p)
    return dA, a


def grad_fd(A, Y, loss, rank, h=1e-6, entries=None, directions=None):
    """Central finite differences of loss(A^+_r Y).

    entries: list of (i, j) entries of A to perturb (returns dL/dA there), or
    directions: list of (dA, dY) pairs (returns the directional derivatives).
    """
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    f = lambda A_, Y_: loss(solve_rank(A_, Y_, rank))
    if directions is not None:
        return np.array([(f(A + h * dA, Y + h * dY) - f(A - h * dA, Y - h * dY)) / (2 * h)
                         for dA, dY in directions])
    out = []
    for (i, j) in entries:
        E = np.zeros_like(A)
        E[i, j] = h
        out.append((f(A + E, Y) - f(A - E, Y)) / (2 * h))
    return np.array(out)


def grad_fd_y(A, Y, loss, rank, h=1e-6):
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty_like(Y)
    for i in range(Y.shape[0]):
        e = np.zeros_like(Y)
        e[i] = h
        out[i] = (loss(solve_rank(A, Y + e, rank)) - loss(solve_rank(A, Y - e, rank))) / (2 * h)
    return out
