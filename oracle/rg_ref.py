"""Plain reference implementation of rank-Greville (Staub & Steinmann).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything here is written for a reader to check against the paper by eye:
Python lists of scalars, explicit loops, no blocking and no reordering.  The
scalar type is generic: ``fractions.Fraction`` gives exact rational runs (the
paper notes in Section 3 that the non-orthogonal scheme only uses operations
defined on rationals), ``float`` gives an IEEE double run.

Notation follows the paper: Gamma (new observation row, length m), y (its
target), X (least-squares solution, length m), C (r x m, rows = the accepted
raw observations), Ct (C tilde, the dual basis (C C^T)^-1 C, r x m), Pinv
(P^-1 = (B^T B)^-1, r x r), gamma = Ct Gamma, Gamma_r = Gamma - C^T gamma
(rejection), zeta = Pinv gamma, K (Kalman gain).

Pins (all in tests/test_oracle_*.py): the Fraction run equals the independent
exact solver ``lstsq_exact`` bit for bit; hand-derived worked examples; the
Penrose equations on the pseudoinverse rebuilt by Theorem 1; truncated-SVD
solutions; closed forms for a single row, A = I and full column rank.  The
maintained pseudoinverse of Theorems 2 and 3 (``track_pinv``) is pinned in
tests/test_oracle_pinv_update.py: exact Penrose equations and B C = A on
Fraction runs, the closed form of [I_n; 1^T], the SVD pseudoinverse in FP64.  The
orthogonal rank factorization variants of Section 2.2 (``variant=``) are
pinned in tests/test_oracle_variants.py: exactly against the same solver and
factor invariants for alpha = 1, in FP64 for the orthonormal one.
"""
from fractions import Fraction
import math

__all__ = [
    "RGState", "default_eps", "is_dependent", "update_least_squares",
    "solve_stream", "lstsq_exact", "rref_row_basis", "pinv_from_state",
    "lstsq_svd", "penrose_residuals", "stability_factor", "residual_error",
]


class RGState:
    """State kept by Algorithm 1 between rows: X, C, Ct, Pinv (all lists).

    Initial state (a reading: the algorithm is stated without an init step):
    rank 0, C and Ct have no rows, Pinv is 0 x 0 and X = 0, i.e. A_0^+ = 0.
    The first non-negligible row is then independent (gamma is empty and
    Gamma_r = Gamma).
    """

    def __init__(self, m, zero, variant="base", track_pinv=False):
        if variant not in ("base", "orthogonal", "orthonormal"):
            raise ValueError(variant)
        self.m = m
        self.zero = zero
        self.variant = variant
        # Theorems 2 and 3 (optional): the pseudoinverse A_n^+ (m x n, list of m
        # rows) and the coordinate factor B_n (n x r, list of n rows) with
        # A_n = B_n C_n, both maintained row by row.
        self.track_pinv = track_pinv
        self.Ap = [[] for _ in range(m)] if track_pinv else None
        self.B = [] if track_pinv else None
        self.X = [zero] * m
        self.C = []      # list of rows (length m)
        self.Ct = []     # list of rows (length m)
        self.Pinv = []   # r x r, list of rows
        self.decisions = []  # True = independent (rank grew) per pushed row

    @property
    def r(self):
        return len(self.C)


def default_eps(m, r, eps_machine):
    """Default threshold of the rank test (Section 3, rank threshold):
    eps = (m^2 r + m r + m) * eps_M.  The paper does not say which r; we take
    the rank before the current row (reading R4)."""
    return (m * m * r + m * r + m) * eps_machine


def is_dependent(Gamma_r, Gamma, eps):
    """Rank test of Section 3: Gamma is treated as a linear combination of the
    previous observations iff ||Gamma_r|| < eps or ||Gamma_r|| < eps*||Gamma||.

    eps = 0 (exact rational runs) reduces this to Gamma_r == 0 exactly, as the
    plain statement of Algorithm 1 has it.  Norms are square roots of sums of
    squares; for exact scalars we compare squares to stay rational."""
    s = sum(v * v for v in Gamma_r)
    if eps == 0:
        return s == 0
    if isinstance(s, Fraction):
        g = sum(v * v for v in Gamma)
        e2 = Fraction(eps) ** 2
        return s < e2 or s < e2 * g
    nr = math.sqrt(s)
    ng = math.sqrt(sum(v * v for v in Gamma))
    return nr < eps or nr < eps * ng


def update_least_squares(st, Gamma, y, eps):
    """One call of Algorithm 1 (UpdateLeastSquares) on state ``st``.

    Independent case: Theorem 4 (x update, K = Gamma_r / ||Gamma_r||^2) and
    Theorem 6 (C gets Gamma appended, Ct <- [Ct - gamma K^T; K^T],
    Pinv <- diag(Pinv, 1)).
    Dependent case: Theorem 5 (K = Ct^T zeta / (1 + gamma^T zeta)) and
    Theorem 6 (Sherman-Morrison downdate Pinv <- Pinv - zeta zeta^T/(1+gamma^T zeta);
    C and Ct unchanged).
    Both: X <- X + K (y - Gamma^T X), with the X from before this row.
    Returns True when the row was independent.

    With ``st.track_pinv`` the same K also updates the pseudoinverse
    (Theorem 2, independent; Theorem 3, dependent):
    A^+ <- [A^+ 0] + K (-beta^T, 1), beta = B zeta, zeta = Pinv gamma, with B
    and Pinv from before this row.  The new row of B holds the coordinates of
    Gamma in the new basis: gamma (dependent), e_{r+1} (base factorization,
    where Gamma itself joins C; old rows gain a zero), or (gamma, 1/alpha)
    (Section 2.2, where alpha Gamma_r joins C).

    Orthogonal rank factorization (Section 2.2): the
    independent case stores a rescaled rejection alpha Gamma_r in C instead of
    Gamma, appends Gamma_r / (alpha ||Gamma_r||^2) to Ct without touching its
    other rows, and borders Pinv with -alpha zeta and alpha^2 (1 + gamma^T zeta),
    zeta = Pinv gamma.  alpha = 1 ("orthogonal", rational) or
    alpha = 1 / ||Gamma_r|| ("orthonormal": C has orthonormal rows, Ct = C).
    The X update (Theorem 4) and the dependent case are the same.
    """
    m, r = st.m, st.r
    Gamma = list(Gamma)
    # gamma = Ct Gamma (projection coordinates in the basis of C's rows)
    z = st.zero
    gamma = [sum((st.Ct[k][j] * Gamma[j] for j in range(m)), z) for k in range(r)]
    # Gamma_r = Gamma - C^T gamma (rejection from the row space)
    Gamma_r = [Gamma[j] - sum((st.C[k][j] * gamma[k] for k in range(r)), z) for j in range(m)]
    eps_r = eps(r) if callable(eps) else eps
    # a priori residual, taken before X changes
    dy = y - sum((Gamma[j] * st.X[j] for j in range(m)), z)
    if st.track_pinv:
        zeta_old = [sum((st.Pinv[i][k] * gamma[k] for k in range(r)), z) for i in range(r)]
        beta = [sum((st.B[i][k] * zeta_old[k] for k in range(r)), z) for i in range(len(st.B))]
    if not is_dependent(Gamma_r, Gamma, eps_r):
        nrm2 = sum((v * v for v in Gamma_r), z)
        K = [v / nrm2 for v in Gamma_r]
        if st.variant == "base":
            st.C.append(list(Gamma))
            st.Ct = [[st.Ct[k][j] - gamma[k] * K[j] for j in range(m)] for k in range(r)]
            st.Ct.append(list(K))
            st.Pinv = [row + [z] for row in st.Pinv] + [[z] * r + [z + 1]]
        else:
            alpha = (z + 1) if st.variant == "orthogonal" else (z + 1) / math.sqrt(nrm2)
            zeta = [sum((st.Pinv[i][k] * gamma[k] for k in range(r)), z) for i in range(r)]
            gz = sum((gamma[k] * zeta[k] for k in range(r)), z)
            st.C.append([alpha * v for v in Gamma_r])
            st.Ct.append([v / (alpha * nrm2) for v in Gamma_r])
            st.Pinv = ([st.Pinv[i] + [-alpha * zeta[i]] for i in range(r)]
                       + [[-alpha * zeta[k] for k in range(r)] + [alpha * alpha * ((z + 1) + gz)]])
        indep = True
    else:
        zeta = [sum((st.Pinv[i][k] * gamma[k] for k in range(r)), z) for i in range(r)]
        den = (z + 1) + sum((gamma[k] * zeta[k] for k in range(r)), z)
        K = [sum((st.Ct[k][j] * zeta[k] for k in range(r)), z) / den for j in range(m)]
        st.Pinv = [[st.Pinv[i][k] - zeta[i] * zeta[k] / den for k in range(r)] for i in range(r)]
        indep = False
    if st.track_pinv:
        st.Ap = [[st.Ap[j][i] - K[j] * beta[i] for i in range(len(beta))] + [K[j]] for j in range(m)]
        if not indep:
            st.B.append(list(gamma))
        else:
            st.B = [row + [z] for row in st.B]
            last = (z + 1) if st.variant == "base" else (z + 1) / alpha
            st.B.append(([z] * r if st.variant == "base" else list(gamma)) + [last])
    st.X = [st.X[j] + K[j] * dy for j in range(m)]
    st.decisions.append(indep)
    return indep


def solve_stream(A, Y, eps=None, exact=False, variant="base", track_pinv=False):
    """Push the rows of A (n x m) with targets Y through Algorithm 1.

    exact=True runs over Fractions with the exact zero test (eps = 0).
    Otherwise floats; eps=None uses the paper's default threshold with
    eps_M = 2^-52 evaluated at the current rank.  variant selects the rank
    factorization: "base" (C = raw rows), "orthogonal" or "orthonormal".
    track_pinv also maintains A^+ and B (Theorems 2 and 3).
    Returns the final RGState (X, C, Ct, Pinv, decisions[, Ap, B]).
    """
    n = len(A)
    m = len(A[0]) if n else 0
    if exact:
        if variant == "orthonormal":
            raise ValueError("the orthonormal variant takes square roots: not rational")
        st = RGState(m, Fraction(0), variant, track_pinv)
        for i in range(n):
            update_least_squares(st, [Fraction(v) for v in A[i]], Fraction(Y[i]), 0)
        return st
    st = RGState(m, 0.0, variant, track_pinv)
    if eps is None:
        eps = lambda r: default_eps(m, r, 2.0 ** -52)
    for i in range(n):
        update_least_squares(st, [float(v) for v in A[i]], float(Y[i]), eps)
    return st


# --------------------------------------------------------------------------
# Independent exact solver (no recursion): the plain definition of x_n.
# --------------------------------------------------------------------------

def rref_row_basis(A):
    """Reduced row echelon form over Fractions; returns the non-zero rows, a
    basis R (r x m) of the row space Im(A^T)."""
    M = [[Fraction(v) for v in row] for row in A]
    n = len(M)
    m = len(M[0]) if n else 0
    piv_row = 0
    for col in range(m):
        p = None
        for i in range(piv_row, n):
            if M[i][col] != 0:
                p = i
                break
        if p is None:
            continue
        M[piv_row], M[p] = M[p], M[piv_row]
        pv = M[piv_row][col]
        M[piv_row] = [v / pv for v in M[piv_row]]
        for i in range(n):
            if i != piv_row and M[i][col] != 0:
                f = M[i][col]
                M[i] = [a - f * b for a, b in zip(M[i], M[piv_row])]
        piv_row += 1
        if piv_row == n:
            break
    return M[:piv_row]


def _solve_exact(S, b):
    """Gauss-Jordan solve of a non-singular Fraction system S c = b."""
    r = len(S)
    M = [list(S[i]) + [b[i]] for i in range(r)]
    for col in range(r):
        p = next(i for i in range(col, r) if M[i][col] != 0)
        M[col], M[p] = M[p], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for i in range(r):
            if i != col and M[i][col] != 0:
                f = M[i][col]
                M[i] = [a - f * c for a, c in zip(M[i], M[col])]
    return [M[i][r] for i in range(r)]


def lstsq_exact(A, Y):
    """Minimum-norm least-squares solution x = A^+ Y in exact rationals,
    computed straight from its definition (the introduction's arg-min of
    ||x|| over the minimisers of ||A x - Y||), without any recursion:

    the minimum-norm minimiser lies in the row space Im(A^T) = span(R^T), so
    x = R^T c, and the normal equations restricted to that space read
    (R A^T A R^T) c = R A^T Y, whose matrix is non-singular for a basis R.
    Returns (x, rank)."""
    A = [[Fraction(v) for v in row] for row in A]
    Y = [Fraction(v) for v in Y]
    n = len(A)
    m = len(A[0]) if n else 0
    R = rref_row_basis(A)
    r = len(R)
    if r == 0:
        return [Fraction(0)] * m, 0
    AR = [[sum(A[i][j] * R[k][j] for j in range(m)) for k in range(r)] for i in range(n)]  # A R^T, n x r
    S = [[sum(AR[i][a] * AR[i][b] for i in range(n)) for b in range(r)] for a in range(r)]
    rhs = [sum(AR[i][a] * Y[i] for i in range(n)) for a in range(r)]
    c = _solve_exact(S, rhs)
    x = [sum(R[k][j] * c[k] for k in range(r)) for j in range(m)]
    return x, r


# --------------------------------------------------------------------------
# Theorem 1, SVD references and the Penrose equations (numpy, FP64).
# --------------------------------------------------------------------------

def pinv_from_state(A, st):
    """Theorem 1: A^+ = C^T (C C^T)^-1 (B^T B)^-1 B^T = Ct^T Pinv B^T, with the
    coordinate matrix B = A Ct^T (rows gamma_i, Section 2.1).  Generic over
    the scalar type of ``st``; returns an m x n list of lists."""
    n = len(A)
    m, r = st.m, st.r
    B = [[sum(A[i][j] * st.Ct[k][j] for j in range(m)) for k in range(r)] for i in range(n)]
    PB = [[sum(st.Pinv[a][k] * B[i][k] for k in range(r)) for i in range(n)] for a in range(r)]
    return [[sum(st.Ct[a][j] * PB[a][i] for a in range(r)) for i in range(n)] for j in range(m)]


def lstsq_svd(A, Y, rank=None):
    """FP64 min-norm least squares via the SVD: x = V_r S_r^-1 U_r^T Y.
    rank=None keeps singular values above max(n,m) * s_max * 2^-52 (the usual
    pinv cut); an integer keeps exactly that many (truncated SVD)."""
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    if rank is None:
        tol = max(A.shape) * (s[0] if s.size else 0.0) * 2.0 ** -52
        rank = int((s > tol).sum())
    Ur, sr, Vr = U[:, :rank], s[:rank], Vt[:rank].T
    return Vr @ ((Ur.T @ Y) / sr[:, None] if Y.ndim == 2 else (Ur.T @ Y) / sr)


def penrose_residuals(A, Ap):
    """Max-abs residuals of the four Penrose equations (introduction):
    A Ap A = A, Ap A Ap = Ap, (A Ap)^T = A Ap, (Ap A)^T = Ap A.
    Works for numpy float arrays and for object arrays of Fractions."""
    import numpy as np
    A = np.asarray(A)
    Ap = np.asarray(Ap)
    AAp = A.dot(Ap)
    ApA = Ap.dot(A)
    r1 = A.dot(ApA) - A
    r2 = Ap.dot(AAp) - Ap
    r3 = AAp.T - AAp
    r4 = ApA.T - ApA
    return [abs(np.asarray(r)).max() if r.size else 0 for r in (r1, r2, r3, r4)]


# --------------------------------------------------------------------------
# Stability measures of Section 4.2 (numpy, FP64).
# --------------------------------------------------------------------------

def stability_factor(Ap_algo, Ap_exact, A, eps_machine=2.0 ** -52):
    """Stability factor of a computed pseudoinverse (Section 4.2, first
    measure): ||Ap_algo - A^+||_2 / (eps_M ||A^+||_2 kappa_2(A)), with the
    2-norm the largest singular value and kappa_2 = s_max / s_min of A."""
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    s = np.linalg.svd(A, compute_uv=False)
    kappa = s[0] / s[-1]
    num = np.linalg.norm(np.asarray(Ap_algo, np.float64) - np.asarray(Ap_exact, np.float64), 2)
    return num / (eps_machine * np.linalg.norm(np.asarray(Ap_exact, np.float64), 2) * kappa)


def residual_error(Ap_algo, A):
    """Residual error of a computed pseudoinverse (Section 4.2, second
    measure): ||Ap_algo A - I||_2 / (||A||_2 ||Ap_algo||_2), I the identity
    of the size of Ap_algo A."""
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    Ap = np.asarray(Ap_algo, dtype=np.float64)
    R = Ap @ A - np.eye(A.shape[1])
    return np.linalg.norm(R, 2) / (np.linalg.norm(A, 2) * np.linalg.norm(Ap, 2))
