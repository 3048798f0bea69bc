"""Oracle: geometric multigrid V-cycle for the shifted blocks of the BEC inverse.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a variable coefficient the blocks B_k = lambda_k I + tau K_a of Step 2
(Section 4, eq. (blockdiaginv)) no longer diagonalise by sine transforms; the
paper solves each one approximately with one V-cycle of geometric multigrid
with one pre- and one post-smoothing step, linear interpolation and its
transpose (Section 4, closing paragraphs; Section 5, Example 2).  This module
writes that V-cycle out plainly for 2D grids, with these readings of what
the paper leaves open:

* smoother: red-black Gauss-Seidel (red = (i1 + i2) even), one red and one
  black half sweep per smoothing step (the paper's ILU smoother is sequential);
* restriction: full weighting, the transpose of bilinear interpolation divided by 4;
* prolongation: bilinear interpolation, zero on the Dirichlet boundary;
* coarse operators: the same flux-form discretisation on the coarse grid
  (h doubled), with each coarse face coefficient the harmonic mean of the two
  fine faces it spans along its normal direction;
* levels: m -> (m-1)/2 while m is odd and >= 3; the coarsest grid gets
  COARSE_SWEEPS red-black sweeps from zero (one point: the exact solve).

Grids are complex arrays [m][m] (y, x), x fastest as everywhere else.
"""
from __future__ import annotations

import numpy as np

COARSE_SWEEPS = 16


def harmonic(a, b):
    return 2.0 * a * b / (a + b)


def coarse_faces(ax: np.ndarray, ay: np.ndarray):
    """Coarse face coefficients of the rediscretised operator.

    ax: [m][m+1] x-faces (face f between nodes f-1 and f of a row),
    ay: [m+1][m] y-faces.  Coarse node I sits on fine node 2I+1; the coarse
    x-face I of coarse row J spans fine x-faces 2I and 2I+1 of fine row 2J+1."""
    m = ax.shape[0]
    mc = (m - 1) // 2
    rows = 2 * np.arange(mc) + 1
    I = np.arange(mc + 1)
    axc = harmonic(ax[np.ix_(rows, 2 * I)], ax[np.ix_(rows, 2 * I + 1)])
    ayc = harmonic(ay[np.ix_(2 * I, rows)], ay[np.ix_(2 * I + 1, rows)])
    return axc, ayc


def levels(ax, ay, tau: float):
    """List of (m, wx, wy) per level, w = tau / h_l^2 * a (face weights)."""
    out = []
    m = ax.shape[0]
    h = 1.0 / (m + 1)
    while True:
        out.append((m, tau / h ** 2 * ax, tau / h ** 2 * ay))
        if m < 3 or m % 2 == 0:
            break
        ax, ay = coarse_faces(ax, ay)
        m = (m - 1) // 2
        h *= 2.0
    return out


def planes(*c):
    """The four coupling planes (W, E, S, N), each [m][m], of one level: node
    (j, i) couples to its west, east, south and north neighbours with weights
    -W, -E, -S, -N and has diagonal W + E + S + N (a neighbour across the
    boundary is zero).  `c` is either the face weights (wx, wy) of the flux form
    (symmetric: W[j, i] = wx[j, i], E[j, i] = wx[j, i+1], S[j, i] = wy[j, i],
    N[j, i] = wy[j+1, i]) or the four planes themselves (a nonsymmetric operator
    such as upwinded convection-diffusion)."""
    if len(c) == 4:
        return c
    wx, wy = c
    m = wx.shape[0]
    return wx[:, :m], wx[:, 1:], wy[:m, :], wy[1:, :]


def _neighbour_sum(e, *c):
    """sum over neighbours of coupling * e_nbr (zero outside) and the diagonal."""
    W, E, S, N = planes(*c)
    s = np.zeros_like(e)
    s[:, 1:] += W[:, 1:] * e[:, :-1]            # west neighbour
    s[:, :-1] += E[:, :-1] * e[:, 1:]           # east neighbour
    s[1:, :] += S[1:, :] * e[:-1, :]            # south (lower) neighbour
    s[:-1, :] += N[:-1, :] * e[1:, :]           # north (upper) neighbour
    d = W + E + S + N
    return s, d


def apply_B(e, lam, *c):
    """(lambda I + tau K) e on one level; `c` as for `planes`."""
    s, d = _neighbour_sum(e, *c)
    return (lam + d) * e - s


def rbgs(e, r, lam, *c):
    """One red-black Gauss-Seidel sweep: red points, then black points."""
    m = e.shape[0]
    jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    e = e.copy()
    for color in (0, 1):
        s, d = _neighbour_sum(e, *c)
        upd = (r + s) / (lam + d)
        mask = (ii + jj) % 2 == color
        e[mask] = upd[mask]
    return e


def interp_1d(mf: int, mc: int) -> np.ndarray:
    """Bilinear (1D linear) interpolation matrix mf x mc with zero boundary values."""
    P = np.zeros((mf, mc))
    for I in range(mc):
        i = 2 * I + 1
        P[i, I] = 1.0
        P[i - 1, I] += 0.5
        if i + 1 < mf:
            P[i + 1, I] += 0.5
    return P


def restrict(r, mc):
    """Full weighting: (1/4) P^T r with P the 2D bilinear interpolation."""
    P = interp_1d(r.shape[0], mc)
    return 0.25 * (P.T @ r @ P)


def prolong(ec, mf):
    P = interp_1d(mf, ec.shape[0])
    return P @ ec @ P.T


def vcycle(lvls, level: int, r: np.ndarray, lam: complex, pre: int = 1, post: int = 1):
    """One V-cycle for B e = r from a zero initial guess on `level`."""
    m, *c = lvls[level]
    e = np.zeros_like(r, dtype=np.complex128)
    if level == len(lvls) - 1:
        for _ in range(COARSE_SWEEPS):
            e = rbgs(e, r, lam, *c)
        return e
    for _ in range(pre):
        e = rbgs(e, r, lam, *c)
    res = r - apply_B(e, lam, *c)
    mc = lvls[level + 1][0]
    ec = vcycle(lvls, level + 1, restrict(res, mc), lam, pre, post)
    e = e + prolong(ec, m)
    for _ in range(post):
        e = rbgs(e, r, lam, *c)
    return e


def step2_mg(ax, ay, tau: float, lam: np.ndarray, yt: np.ndarray, cycles: int = 1):
    """Step 2 with `cycles` V-cycles per block (each cycle a correction of the
    previous iterate); yt: [nk][m*m] complex; returns the same shape."""
    lv = levels(np.asarray(ax, float), np.asarray(ay, float), tau)
    return step2_levels(lv, lam, yt, cycles)


def step2_levels(lv, lam: np.ndarray, yt: np.ndarray, cycles: int = 1):
    """Step 2 on a ready level list (entries (m, *couplings) as `planes` takes)."""
    m = lv[0][0]
    out = np.empty_like(yt, dtype=np.complex128)
    for k in range(yt.shape[0]):
        r = yt[k].reshape(m, m)
        e = np.zeros((m, m), dtype=np.complex128)
        for _ in range(cycles):
            e = e + vcycle(lv, 0, r - apply_B(e, lam[k], *lv[0][1:]), lam[k])
        out[k] = e.reshape(-1)
    return out


def mean_coefficient(ax, ay) -> float:
    """Arithmetic mean over all faces: the constant coefficient of the
    mean-coefficient sine-transform inner solve."""
    return float((np.sum(ax) + np.sum(ay)) / (np.size(ax) + np.size(ay)))
