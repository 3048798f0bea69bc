"""Q1 finite elements on uniform grids of the unit square (Section 5 discretises
space this way; Section 4's L and P_eps carry the mass matrix M).  Test
infrastructure, like the rest of this package.

    M = M1 (x) M1,   K = M1 (x) K1 + K1 (x) M1      (x fastest, Dirichlet 0)
    M1 = h/6 tridiag(1, 4, 1),   K1 = 1/h tridiag(-1, 2, -1),   h = 1/(m1+1)

for a constant coefficient (K scaled by a).  The all-at-once system of a
p-step scheme (eq. (pstepscheme)) is L = R (x) M + tau I (x) K and the BEC
preconditioner (eq. (pstepbecpreconditioner)) P_eps = R_eps (x) M + tau I (x) K,
inverted by Section 4's three steps with blocks B_k = lambda_k M + tau K
(eq. (becblockdiag)).  The right-hand side is the FE load: tau M f^k with the
source sampled at the nodes, plus M u^0 in the first row (and -r_2 M u^0 in the
second for BDF2, R17's start-up: a backward-Euler first step).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bdf, heat


def mass_1d(m1: int) -> sp.csr_matrix:
    h = 1.0 / (m1 + 1)
    return (sp.diags([np.full(m1 - 1, 1.0), np.full(m1, 4.0), np.full(m1 - 1, 1.0)],
                     [-1, 0, 1]) * (h / 6.0)).tocsr()


def stiff_1d(m1: int) -> sp.csr_matrix:
    h = 1.0 / (m1 + 1)
    return (sp.diags([np.full(m1 - 1, -1.0), np.full(m1, 2.0), np.full(m1 - 1, -1.0)],
                     [-1, 0, 1]) / h).tocsr()


def q1_matrices(m1: int, a: float = 1.0):
    """(M, K) of Q1 elements on the m1 x m1 interior grid (x fastest)."""
    M1, K1 = mass_1d(m1), stiff_1d(m1)
    M = sp.kron(M1, M1).tocsr()
    K = (a * (sp.kron(M1, K1) + sp.kron(K1, M1))).tocsr()
    return M, K


def apply_L(M, K, tau: float, r, v: np.ndarray, start: str = "be") -> np.ndarray:
    """(L v)^k = sum_j r_j M v^{k-j} + tau K v^k, v^{<1} = 0, row 1 with
    coefficient 1 on M v^1 for start = "be" (eq. (pstepscheme))."""
    v = np.asarray(v, dtype=np.float64)
    Mv = (M @ v.T).T
    out = tau * (K @ v.T).T
    for j, rj in enumerate(r):
        if j == 0:
            out += rj * Mv
        else:
            out[j:] += rj * Mv[:-j]
    if start == "be":
        out[0] += (1.0 - r[0]) * Mv[0]
    return out


def build_rhs(M, f: np.ndarray, u0: np.ndarray, tau: float, r, start: str = "be") -> np.ndarray:
    return (M @ bdf.build_rhs(f, u0, tau, r, start).T).T


def block_factors(M, K, tau: float, lam: np.ndarray):
    Mc = M.astype(np.complex128).tocsc()
    Kc = K.astype(np.complex128).tocsc()
    return [spla.splu((lk * Mc + tau * Kc).tocsc()) for lk in lam]


def apply_Pinv(M, K, tau: float, r, eps: float, y: np.ndarray, factors=None) -> np.ndarray:
    """Section 4's three steps with B_k = lambda_k M + tau K (eq. (becblockdiag))."""
    n = y.shape[0]
    lam = heat.lambdas(n, eps, r)[: n // 2 + 1]
    if factors is None:
        factors = block_factors(M, K, tau, lam)
    yt = heat.step1(y, eps)
    zt = np.empty_like(yt)
    for k in range(yt.shape[0]):
        zt[k] = factors[k].solve(np.ascontiguousarray(yt[k]))
    return heat.step3(zt, eps, n)


def sequential(M, K, tau: float, r, rhs: np.ndarray, start: str = "be") -> np.ndarray:
    """(c_k M + tau K) u^k = rhs^k - sum_{j>=1} r_j M u^{k-j}, c_1 by `start`."""
    n = rhs.shape[0]
    lus = {}
    u = np.zeros_like(rhs, dtype=np.float64)
    for k in range(n):
        ck = bdf.r0_first(r, start) if k == 0 else r[0]
        if ck not in lus:
            lus[ck] = spla.splu((ck * M + tau * K).tocsc())
        b = rhs[k].copy()
        for j in range(1, len(r)):
            if k - j >= 0:
                b -= r[j] * (M @ u[k - j])
        u[k] = lus[ck].solve(b)
    return u


def dense_P(M, K, n: int, tau: float, r, eps: float) -> np.ndarray:
    M = np.asarray(M.todense())
    K = np.asarray(K.todense())
    return np.kron(heat.r_eps_dense(n, eps, r), M) + tau * np.kron(np.eye(n), K)


def dense_L(M, K, n: int, tau: float, r, start: str = "be") -> np.ndarray:
    M = np.asarray(M.todense())
    K = np.asarray(K.todense())
    R = heat.r_eps_dense(n, 0.0, r)
    R[0, 0] = bdf.r0_first(r, start)
    return np.kron(R, M) + tau * np.kron(np.eye(n), K)


class Problem:
    """Q1-FE all-at-once problem on the m1 x m1 interior grid of the unit square."""

    def __init__(self, m1: int, n: int, r=bdf.BDF1, T: float = 1.0, eps: float | None = None,
                 a: float = 1.0, start: str = "be"):
        self.m1, self.n, self.r, self.start = m1, n, tuple(r), start
        self.tau = T / n
        self.eps = min(0.5, 0.5 * self.tau) if eps is None else eps
        self.M, self.K = q1_matrices(m1, a)
        self.m = m1 * m1
        self._factors = None

    def L(self, v):
        return apply_L(self.M, self.K, self.tau, self.r, np.asarray(v).reshape(self.n, self.m),
                       self.start)

    def Pinv(self, v):
        if self._factors is None:
            lam = heat.lambdas(self.n, self.eps, self.r)[: self.n // 2 + 1]
            self._factors = block_factors(self.M, self.K, self.tau, lam)
        return apply_Pinv(self.M, self.K, self.tau, self.r, self.eps,
                          np.asarray(v).reshape(self.n, self.m), self._factors)

    def rhs(self, f, u0):
        return build_rhs(self.M, f, u0, self.tau, self.r, self.start)

    def exact(self, rhs):
        return sequential(self.M, self.K, self.tau, self.r, rhs, self.start)

    def gmres(self, rhs, tol=1e-8, maxit=200, restart=50):
        A = lambda v: self.L(v).reshape(-1)                                 # noqa: E731
        Mi = lambda v: self.Pinv(v).reshape(-1)                             # noqa: E731
        x, it, hist = heat.fgmres(A, Mi, rhs.reshape(-1), tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist

    def gmres_left(self, rhs, tol=1e-7, maxit=300, restart=50):
        A = lambda v: self.Pinv(self.L(v)).reshape(-1)                      # noqa: E731
        b = self.Pinv(rhs).reshape(-1)
        x, it, hist = heat.fgmres(A, lambda v: v, b, tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist
