"""p-step backward-difference (BDF) all-at-once systems and their BEC
preconditioner (Section 4, eqs. (pstepscheme), (pstepbecpreconditioner),
(repsdiagform)).  Test infrastructure, like the rest of this package: plain,
slow FP64 code that the GPU path is checked against, never called by it.

    L   = R (x) M + tau I_N (x) K,     R   banded lower Toeplitz with r_0..r_p
    P_e = R_e (x) M + tau I_N (x) K,   R_e = R plus e r_j wrapped into the
                                             top-right corner
    lambda_k = sum_j r_j e^{j/N} theta^{kj}

with M = I (finite differences).  BDF1 (backward Euler) is r = (1, -1); BDF2 is
r = (3/2, -2, 1/2) (Section 5, Example 1 with Table bdf2table).

Start-up (the paper does not say how the p-step scheme obtains its first
values): `start="be"` takes the first step with backward Euler, so row 1 of L
reads u^1 + tau K u^1 = tau f^1 + u^0 and the later rows are the BDF2 rows with
u^0 moved to the right-hand side; `start="u0"` keeps R Toeplitz in every row by
setting u^{-1} = u^0.  The preconditioner is the Toeplitz R_e in both cases.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import heat

BDF1 = (1.0, -1.0)
BDF2 = (1.5, -2.0, 0.5)


def r0_first(r, start: str) -> float:
    """Coefficient of u^1 in row 1 of L."""
    if start == "be":
        return 1.0
    if start == "u0":
        return r[0]
    raise ValueError(start)


def apply_L(K: sp.spmatrix, tau: float, r, v: np.ndarray, start: str = "be") -> np.ndarray:
    """(L v)^k = sum_{j=0}^{p} r_j v^{k-j} + tau K v^k with v^{<1} = 0 and row 1
    as set by `start` (eq. (pstepscheme))."""
    v = np.asarray(v, dtype=np.float64)
    out = tau * (K @ v.T).T
    for j, rj in enumerate(r):
        if j == 0:
            out += rj * v
        else:
            out[j:] += rj * v[:-j]
    if start == "be":
        # row 1 is the backward-Euler step: coefficient 1 on u^1 and nothing else
        out[0] += (1.0 - r[0]) * v[0]
    return out


def apply_P(K: sp.spmatrix, tau: float, r, eps: float, v: np.ndarray) -> np.ndarray:
    """P_eps v with the Toeplitz R_eps of eq. (pstepbecpreconditioner): the
    terms j that reach before the first level wrap to level N + k - j, times eps."""
    v = np.asarray(v, dtype=np.float64)
    n = v.shape[0]
    out = apply_L(K, tau, r, v, start="u0")
    for j, rj in enumerate(r):
        for k in range(min(j, n)):
            out[k] += eps * rj * v[n + k - j]
    return out


def build_rhs(f: np.ndarray, u0: np.ndarray, tau: float, r, start: str = "be") -> np.ndarray:
    """Right-hand side of L u = rhs: tau f^k plus the known initial value moved
    to the rows that reference it.  "be": row 1 gets u^0 (backward Euler), row
    j (2 <= j <= p) gets -r_j u^0.  "u0": u^{-q} = u^0 for every missing level,
    so row k gets -(r_k + ... + r_p) u^0 for k <= p."""
    rhs = tau * np.asarray(f, dtype=np.float64).copy()
    n = rhs.shape[0]
    p = len(r) - 1
    if start == "be":
        rhs[0] += u0
        for j in range(2, p + 1):
            if j - 1 < n:
                rhs[j - 1] -= r[j] * u0
    elif start == "u0":
        for k in range(1, p + 1):
            if k - 1 < n:
                rhs[k - 1] -= sum(r[k:]) * u0
    else:
        raise ValueError(start)
    return rhs


def sequential(K: sp.spmatrix, tau: float, r, rhs: np.ndarray, start: str = "be") -> np.ndarray:
    """Exact solution of L u = rhs by stepping: (c_k I + tau K) u^k = rhs^k -
    sum_{j>=1} r_j u^{k-j}, with c_1 from `start` and c_k = r_0 after."""
    m = K.shape[0]
    n = rhs.shape[0]
    lus = {}
    u = np.zeros_like(rhs, dtype=np.float64)
    for k in range(n):
        ck = r0_first(r, start) if k == 0 else r[0]
        if ck not in lus:
            lus[ck] = spla.splu((ck * sp.identity(m) + tau * K).tocsc())
        b = rhs[k].copy()
        for j in range(1, len(r)):
            if k - j >= 0:
                b -= r[j] * u[k - j]
        u[k] = lus[ck].solve(b)
    return u


def apply_Pinv(K: sp.spmatrix, tau: float, r, eps: float, y: np.ndarray,
               factors=None) -> np.ndarray:
    """P_eps^{-1} y by the three steps of Section 4 with lambda_k of eq.
    (repsdiagform) for the given r; blocks k = 0..N/2 only (R_eps is real)."""
    n = y.shape[0]
    lam = heat.lambdas(n, eps, r)
    yt = heat.step1(y, eps)
    zt = heat.step2(K, tau, lam[: n // 2 + 1], yt, factors)
    return heat.step3(zt, eps, n)


def dense_L(K, n: int, tau: float, r, start: str = "be") -> np.ndarray:
    K = np.asarray(K.todense() if sp.issparse(K) else K)
    m = K.shape[0]
    R = heat.r_eps_dense(n, 0.0, r)
    R[0, 0] = r0_first(r, start)
    return np.kron(R, np.eye(m)) + tau * np.kron(np.eye(n), K)


def dense_P(K, n: int, tau: float, r, eps: float) -> np.ndarray:
    K = np.asarray(K.todense() if sp.issparse(K) else K)
    m = K.shape[0]
    return np.kron(heat.r_eps_dense(n, eps, r), np.eye(m)) + tau * np.kron(np.eye(n), K)


class Problem:
    """The p-step all-at-once problem on the unit square/cube grid of `heat`,
    with the BEC preconditioner (eps default min(0.5, 0.5 tau), Section 5)."""

    def __init__(self, m1: int, dim: int, n: int, r=BDF2, T: float = 1.0,
                 eps: float | None = None, start: str = "be", a: float = 1.0):
        self.m1, self.dim, self.n, self.r, self.start = m1, dim, n, tuple(r), start
        self.tau = T / n
        self.eps = min(0.5, 0.5 * self.tau) if eps is None else eps
        self.K = a * heat.stiffness(m1, dim)
        self.m = self.K.shape[0]
        self._factors = None

    def L(self, v):
        return apply_L(self.K, self.tau, self.r, np.asarray(v).reshape(self.n, self.m), self.start)

    def P(self, v):
        return apply_P(self.K, self.tau, self.r, self.eps, np.asarray(v).reshape(self.n, self.m))

    def Pinv(self, v):
        if self._factors is None:
            lam = heat.lambdas(self.n, self.eps, self.r)[: self.n // 2 + 1]
            self._factors = heat.block_factors(self.K, self.tau, lam)
        return apply_Pinv(self.K, self.tau, self.r, self.eps,
                          np.asarray(v).reshape(self.n, self.m), self._factors)

    def rhs(self, f, u0):
        return build_rhs(f, u0, self.tau, self.r, self.start)

    def exact(self, rhs):
        return sequential(self.K, self.tau, self.r, rhs, self.start)

    def gmres(self, rhs, tol=1e-8, maxit=200, restart=50):
        A = lambda v: self.L(v).reshape(-1)                                 # noqa: E731
        M = lambda v: self.Pinv(v).reshape(-1)                              # noqa: E731
        x, it, hist = heat.fgmres(A, M, rhs.reshape(-1), tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist

    def gmres_left(self, rhs, tol=1e-7, maxit=300, restart=50):
        A = lambda v: self.Pinv(self.L(v)).reshape(-1)                      # noqa: E731
        b = self.Pinv(rhs).reshape(-1)
        x, it, hist = heat.fgmres(A, lambda v: v, b, tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist
