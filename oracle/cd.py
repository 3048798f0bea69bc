"""Convection-diffusion with a circulating wind and a hot wall: the stand-in for
Section 5, Example 3.  Test infrastructure, like the rest of this package.

    u_t = nu Laplace(u) - w . grad(u)   on (-1, 1)^2 x (0, T],
    w(x, y) = (2y(1 - x^2), -2x(1 - y^2)),   nu = 1/200,
    u = (1 - exp(-10 t)) phi on the boundary, phi = 1 on the wall x = 1, else 0,
    u(., 0) = 0.

The paper discretises space with Q1 elements and SUPG stabilisation (matrices
from a package that is not available here); this stand-in uses five-point
finite differences with first-order upwinding of the convection term on the
m1 x m1 interior nodes, h = 2/(m1+1), so M = I and K is a nonsymmetric
M-matrix.  Node (j, i) (x fastest) couples to its four neighbours with

    W = nu/h^2 + max(w1, 0)/h,   E = nu/h^2 + max(-w1, 0)/h,
    S = nu/h^2 + max(w2, 0)/h,   N = nu/h^2 + max(-w2, 0)/h,

(K u)_ji = (W + E + S + N) u_ji - W u_west - E u_east - S u_south - N u_north,
the wind taken at the node.  Known boundary values move to the right-hand
side: b^k = couplings to boundary nodes times the Dirichlet data at t_k.
Time: backward Euler (eq. (backwarddiff)); the all-at-once system, P_eps and
its three-step inverse are those of `heat` with this K (they need K real, not
symmetric).  The inner solves of Step 2 are either exact (sparse LU per block)
or one V-cycle of `mg` on the coupling planes, the coarse levels rediscretised
with the wind taken at the coarse nodes (injection) and h doubled.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import heat, mg

NU = 1.0 / 200.0


def nodes(m1: int) -> np.ndarray:
    """Interior node coordinates on (-1, 1): -1 + (i+1) h, h = 2/(m1+1)."""
    h = 2.0 / (m1 + 1)
    return -1.0 + h * np.arange(1, m1 + 1)


def wind(X, Y):
    """The circulating wind of Example 3."""
    return 2.0 * Y * (1.0 - X ** 2), -2.0 * X * (1.0 - Y ** 2)


def couplings(nu: float, h: float, w1: np.ndarray, w2: np.ndarray):
    """(W, E, S, N) planes of the upwinded operator for the wind sampled at the nodes."""
    d = nu / h ** 2
    return (d + np.maximum(w1, 0.0) / h, d + np.maximum(-w1, 0.0) / h,
            d + np.maximum(w2, 0.0) / h, d + np.maximum(-w2, 0.0) / h)


def stiffness_planes(W, E, S, N) -> sp.csr_matrix:
    """Sparse K from its coupling planes (x fastest, zero Dirichlet data)."""
    m2, m1 = W.shape
    idx = np.arange(m1 * m2).reshape(m2, m1)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [(W + E + S + N).ravel()]
    for plane, sl_node, sl_nbr in (
            (W, np.s_[:, 1:], np.s_[:, :-1]), (E, np.s_[:, :-1], np.s_[:, 1:]),
            (S, np.s_[1:, :], np.s_[:-1, :]), (N, np.s_[:-1, :], np.s_[1:, :])):
        rows.append(idx[sl_node].ravel())
        cols.append(idx[sl_nbr].ravel())
        vals.append(-plane[sl_node].ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m1 * m2, m1 * m2))
    return K.tocsr()


def boundary_load(W, E, S, N, gw, ge, gs, gn) -> np.ndarray:
    """Couplings to the boundary nodes times their values: gw, ge [m2] on the
    walls left and right of each row, gs, gn [m1] below and above each column."""
    b = np.zeros(W.shape)
    b[:, 0] += W[:, 0] * gw
    b[:, -1] += E[:, -1] * ge
    b[0, :] += S[0, :] * gs
    b[-1, :] += N[-1, :] * gn
    return b.reshape(-1)


def hot_wall(m1: int, t: float):
    """Boundary values (west, east, south, north) at time t: the east wall
    x = 1 carries 1 - exp(-10 t), the others 0 (the corners of the east wall
    are no neighbour of an interior node)."""
    z = np.zeros(m1)
    return z, np.full(m1, 1.0 - math.exp(-10.0 * t)), z, z


def mg_levels(m1: int, nu: float, tau: float):
    """V-cycle levels (m, tau W, tau E, tau S, tau N): m -> (m-1)/2 while m is odd
    and >= 3, each level the same upwind discretisation with the wind at its
    nodes (coarse node I is fine node 2I+1) and h doubled."""
    x = nodes(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    w1, w2 = wind(X, Y)
    h = 2.0 / (m1 + 1)
    m = m1
    out = []
    while True:
        out.append((m,) + tuple(tau * c for c in couplings(nu, h, w1, w2)))
        if m < 3 or m % 2 == 0:
            break
        w1 = w1[1::2, 1::2]
        w2 = w2[1::2, 1::2]
        m = (m - 1) // 2
        h *= 2.0
    return out


class Problem:
    """The all-at-once backward-Euler system of the stand-in on m1 x m1 nodes."""

    def __init__(self, m1: int, n: int, T: float = 1.0, eps: float | None = None,
                 nu: float = NU):
        self.m1, self.n, self.T, self.nu = m1, n, T, nu
        self.tau = T / n
        self.eps = min(0.5, 0.5 * self.tau) if eps is None else eps
        self.h = 2.0 / (m1 + 1)
        x = nodes(m1)
        X, Y = np.meshgrid(x, x, indexing="xy")
        self.w1, self.w2 = wind(X, Y)
        self.planes = couplings(nu, self.h, self.w1, self.w2)
        self.K = stiffness_planes(*self.planes)
        self.m = m1 * m1
        self._factors = None
        self._levels = None

    def source(self) -> np.ndarray:
        """f^k = boundary load of the hot wall at t_k = k tau, k = 1..n."""
        return np.stack([boundary_load(*self.planes, *hot_wall(self.m1, (k + 1) * self.tau))
                         for k in range(self.n)])

    def rhs(self, f=None, u0=None):
        f = self.source() if f is None else f
        u0 = np.zeros(self.m) if u0 is None else u0
        return heat.build_rhs(f, u0, self.tau)

    def L(self, v):
        return heat.apply_L(self.K, self.tau, np.asarray(v).reshape(self.n, self.m))

    def Pinv(self, v):
        if self._factors is None:
            lam = heat.lambdas(self.n, self.eps)[: self.n // 2 + 1]
            self._factors = heat.block_factors(self.K, self.tau, lam)
        return heat.apply_Pinv(self.K, self.tau, self.eps, np.asarray(v).reshape(self.n, self.m),
                               self._factors)

    def levels(self):
        if self._levels is None:
            self._levels = mg_levels(self.m1, self.nu, self.tau)
        return self._levels

    def Pinv_mg(self, v, cycles: int = 1):
        """P_eps^{-1} with `cycles` V-cycles per block in Step 2."""
        n = self.n
        y = np.asarray(v).reshape(n, self.m)
        lam = heat.lambdas(n, self.eps)[: n // 2 + 1]
        zt = mg.step2_levels(self.levels(), lam, heat.step1(y, self.eps), cycles)
        return heat.step3(zt, self.eps, n)

    def exact(self, rhs):
        return heat.sequential_be(self.K, self.tau, np.asarray(rhs).reshape(self.n, self.m))

    def gmres(self, rhs, tol=1e-8, maxit=200, restart=50, inner="lu", cycles=1):
        Mi = (lambda v: self.Pinv(v).reshape(-1)) if inner == "lu" else \
            (lambda v: self.Pinv_mg(v, cycles).reshape(-1))                 # noqa: E731
        A = lambda v: self.L(v).reshape(-1)                                 # noqa: E731
        x, it, hist = heat.fgmres(A, Mi, np.asarray(rhs).reshape(-1), tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist

    def gmres_left(self, rhs, tol=1e-7, maxit=300, restart=50, inner="lu", cycles=1):
        Pi = self.Pinv if inner == "lu" else (lambda v: self.Pinv_mg(v, cycles))  # noqa: E731
        A = lambda v: Pi(self.L(v)).reshape(-1)                             # noqa: E731
        b = Pi(np.asarray(rhs).reshape(self.n, self.m)).reshape(-1)
        x, it, hist = heat.fgmres(A, lambda v: v, b, tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist
