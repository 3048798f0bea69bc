"""Pins of the p-step (BDF2) oracle, oracle/bdf.py, against what the paper
and the mathematics fix (Section 4, eqs. (pstepscheme), (pstepbecpreconditioner),
(repsdiagform); Section 5, Table bdf2table):

* time order: on an exact eigenvector of K the semi-discrete solution is known,
  so the error is the time discretisation's alone; BDF2 with a backward-Euler
  first step is second order, with u^{-1} = u^0 only first order (the reading
  the library takes is the second-order one);
* L, P_eps and P_eps^{-1} against the dense matrices written out from the
  paper's displays of R and R_eps;
* the stepping solver against a dense solve of L u = rhs;
* rank(P_eps^{-1} L - I) <= p J (R - R_eps lives in the first p rows);
* backward Euler through the p-step code equals the BE oracle of heat.py;
* Table bdf2table, qualitatively: GMRES-BEC needs far fewer iterations than
  GMRES-BC, and the BEC count does not grow with the grid.  (The printed counts,
  13 and ~80, are not reproduced: with a = 1e-5 the preconditioned matrix is
  essentially R_eps^{-1} R, whose corner eigenvalues sit within O(eps) of 1 for
  eps = 0.5 tau, so this discretisation converges in 3 and 13 iterations; the
  paper does not state the start-up or the finite-element details that would
  explain its counts.)
"""
import math

import numpy as np
import pytest

from oracle import bdf, heat
import workloads as W


def _order_errors(start):
    m1 = 31
    h = 1.0 / (m1 + 1)
    s = np.sin(math.pi * np.arange(1, m1 + 1) * h)
    mu = 4.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2
    K = heat.stiffness(m1, 1)
    assert np.allclose(K @ s, mu * s)
    errs = []
    for n in (16, 32, 64, 128):
        tau = 1.0 / n
        t = (np.arange(n) + 1) * tau
        f = ((mu - 1.0) * np.exp(-t))[:, None] * s[None, :]      # u = exp(-t) s exactly
        rhs = bdf.build_rhs(f, s, tau, bdf.BDF2, start)
        u = bdf.sequential(K, tau, bdf.BDF2, rhs, start)
        errs.append(np.abs(u - np.exp(-t)[:, None] * s[None, :]).max())
    return errs


def test_bdf2_be_start_is_second_order():
    errs = _order_errors("be")
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert ratios[-1] >= 3.3, ratios          # -> 4


def test_bdf2_u0_start_is_first_order():
    errs = _order_errors("u0")
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert ratios[-1] <= 2.2, ratios          # -> 2


@pytest.mark.parametrize("r", [bdf.BDF1, bdf.BDF2], ids=["bdf1", "bdf2"])
@pytest.mark.parametrize("dim,m1,n,eps", [(1, 5, 8, 0.3), (2, 3, 6, 0.05), (1, 4, 4, 1.0)])
def test_operators_match_dense(r, dim, m1, n, eps):
    K = heat.stiffness(m1, dim)
    tau = 1.0 / n
    m = K.shape[0]
    rng = np.random.default_rng(31)
    v = rng.standard_normal((n, m))
    for start in ("be", "u0"):
        L = bdf.dense_L(K, n, tau, r, start)
        assert np.allclose(bdf.apply_L(K, tau, r, v, start).reshape(-1), L @ v.reshape(-1),
                           atol=1e-13)
    P = bdf.dense_P(K, n, tau, r, eps)
    assert np.allclose(bdf.apply_P(K, tau, r, eps, v).reshape(-1), P @ v.reshape(-1), atol=1e-13)
    z = bdf.apply_Pinv(K, tau, r, eps, v)
    assert np.allclose(z.reshape(-1), np.linalg.solve(P, v.reshape(-1)), atol=1e-11)


def test_stepping_matches_dense_solve():
    m1, dim, n = 4, 2, 8
    K = heat.stiffness(m1, dim)
    tau = 1.0 / n
    rhs = np.random.default_rng(32).standard_normal((n, K.shape[0]))
    for start in ("be", "u0"):
        u = bdf.sequential(K, tau, bdf.BDF2, rhs, start)
        ud = np.linalg.solve(bdf.dense_L(K, n, tau, bdf.BDF2, start), rhs.reshape(-1))
        assert np.allclose(u.reshape(-1), ud, atol=1e-12)


def test_rank_of_preconditioned_minus_identity():
    m1, n, eps = 4, 8, 0.3
    K = heat.stiffness(m1, 1)
    tau = 1.0 / n
    L = bdf.dense_L(K, n, tau, bdf.BDF2, "be")
    P = bdf.dense_P(K, n, tau, bdf.BDF2, eps)
    G = np.linalg.solve(P, L) - np.eye(n * m1)
    sv = np.linalg.svd(G, compute_uv=False)
    assert int((sv > 1e-10 * sv[0]).sum()) <= 2 * m1


def test_bdf1_through_pstep_code_is_backward_euler():
    m1, dim, n, eps = 6, 2, 8, 0.2
    K = heat.stiffness(m1, dim)
    tau = 1.0 / n
    rng = np.random.default_rng(33)
    v = rng.standard_normal((n, K.shape[0]))
    u0 = rng.standard_normal(K.shape[0])
    assert np.allclose(bdf.apply_L(K, tau, bdf.BDF1, v), heat.apply_L(K, tau, v), atol=1e-14)
    assert np.allclose(bdf.apply_Pinv(K, tau, bdf.BDF1, eps, v),
                       heat.apply_Pinv(K, tau, eps, v), atol=1e-13)
    assert np.allclose(bdf.build_rhs(v, u0, tau, bdf.BDF1), heat.build_rhs(v, u0, tau))


def _table_bdf2(n, J1, bec):
    m1 = J1 - 1
    x = W.node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = (X * (X - 1) * Y * (Y - 1)).reshape(-1)
    p = bdf.Problem(m1, 2, n, r=bdf.BDF2, eps=None if bec else 1.0, a=1e-5)
    rhs = p.rhs(np.zeros((n, p.m)), u0)
    u, it, _ = p.gmres_left(rhs, tol=1e-7)
    return it, np.linalg.norm(rhs - p.L(u)) / np.linalg.norm(rhs)


@pytest.mark.slow
def test_table_bdf2_qualitative():
    it32, _ = _table_bdf2(64, 32, True)
    it64, res64 = _table_bdf2(64, 64, True)
    bc64, bcres64 = _table_bdf2(64, 64, False)
    assert abs(it32 - it64) <= 1                 # flat in the grid
    assert bc64 >= 3 * it64                       # BEC far ahead of BC
    assert res64 < bcres64                        # and more accurate in RES
