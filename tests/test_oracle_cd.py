"""Pins of the convection-diffusion oracle (oracle/cd.py), each against
something other than the oracle itself:

* linear functions are reproduced exactly by the upwinded operator with its
  boundary load (K u - b = w . grad u), for a random wind of both signs: pins
  the walls, the two wind components and their signs;
* the truncation error on x^2 and y^2 is that of the upwind (not downwind or
  central) difference: -2 nu + w_d (2 x_d - h sign(w_d));
* K is an M-matrix (nonpositive off-diagonals, nonnegative row sums);
* constants are steady (K 1 = b(1));
* the steady problem converges at first order to a manufactured solution;
* P_eps^{-1} with this nonsymmetric K equals a dense solve, and GMRES-BEC with
  exact inner solves equals sequential backward Euler;
* each coarse multigrid level equals the discretisation assembled directly on
  the coarse grid; V-cycles in correction form converge to the direct solve;
* Section 5, Example 3 / Table 3 qualitatively: GMRES-BEC needs far fewer
  iterations than GMRES-BC, flat in the grid, and reaches a smaller RES.
"""
import math

import numpy as np
import pytest

from oracle import cd, heat, mg


def _random_wind(m1, rng):
    return rng.standard_normal((m1, m1)), rng.standard_normal((m1, m1))


def _walls(fun, m1):
    """Boundary values of fun(x, y) next to each interior row / column."""
    x = cd.nodes(m1)
    return fun(-1.0, x), fun(1.0, x), fun(x, -1.0), fun(x, 1.0)


def test_linear_functions_are_exact():
    m1, nu = 9, 0.3
    rng = np.random.default_rng(71)
    w1, w2 = _random_wind(m1, rng)
    h = 2.0 / (m1 + 1)
    P = cd.couplings(nu, h, w1, w2)
    K = cd.stiffness_planes(*P)
    a, b, c = 0.7, -1.3, 0.4
    fun = lambda x, y: a * x + b * y + c                           # noqa: E731
    X, Y = np.meshgrid(cd.nodes(m1), cd.nodes(m1), indexing="xy")
    u = fun(X, Y).reshape(-1)
    got = K @ u - cd.boundary_load(*P, *_walls(fun, m1))
    assert np.allclose(got, (a * w1 + b * w2).reshape(-1), atol=1e-11)


@pytest.mark.parametrize("axis", [0, 1])
def test_upwind_truncation_on_quadratics(axis):
    m1, nu = 11, 0.05
    rng = np.random.default_rng(72)
    w1, w2 = _random_wind(m1, rng)
    h = 2.0 / (m1 + 1)
    P = cd.couplings(nu, h, w1, w2)
    K = cd.stiffness_planes(*P)
    fun = (lambda x, y: x * x + 0 * y) if axis == 0 else (lambda x, y: y * y + 0 * x)
    X, Y = np.meshgrid(cd.nodes(m1), cd.nodes(m1), indexing="xy")
    u = fun(X, Y).reshape(-1)
    got = K @ u - cd.boundary_load(*P, *_walls(fun, m1))
    w, z = (w1, X) if axis == 0 else (w2, Y)
    want = -2.0 * nu + w * (2.0 * z - h * np.sign(w))
    assert np.allclose(got, want.reshape(-1), atol=1e-10)


def test_m_matrix():
    p = cd.Problem(15, 4)
    K = p.K.toarray()
    off = K - np.diag(np.diag(K))
    assert (off <= 0).all()
    assert (K.sum(axis=1) >= -1e-9).all()
    assert (np.diag(K) > 0).all()
    assert not np.allclose(K, K.T)                 # nonsymmetric


def test_constants_are_steady():
    p = cd.Problem(15, 4)
    one = lambda x, y: 1.0 + 0 * x + 0 * y         # noqa: E731
    b = cd.boundary_load(*p.planes, *_walls(one, 15))
    assert np.allclose(p.K @ np.ones(p.m), b, rtol=1e-13, atol=1e-9)


def test_steady_state_first_order():
    """-nu Lap u + w . grad u = f with u = sin(pi x) sin(pi y) (zero on the
    boundary): the upwinded solution converges at first order in h."""
    nu = 0.05
    errs = []
    for m1 in (31, 63, 127):
        x = cd.nodes(m1)
        X, Y = np.meshgrid(x, x, indexing="xy")
        w1, w2 = cd.wind(X, Y)
        u = np.sin(math.pi * X) * np.sin(math.pi * Y)
        f = (2 * nu * math.pi ** 2 * u + w1 * math.pi * np.cos(math.pi * X) * np.sin(math.pi * Y)
             + w2 * math.pi * np.sin(math.pi * X) * np.cos(math.pi * Y))
        K = cd.stiffness_planes(*cd.couplings(nu, 2.0 / (m1 + 1), w1, w2))
        from scipy.sparse.linalg import spsolve
        U = spsolve(K.tocsc(), f.reshape(-1))
        errs.append(np.max(np.abs(U - u.reshape(-1))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.6 < r1 < 2.6 and 1.7 < r2 < 2.4, errs
    assert errs[-1] < 0.05


def test_hot_wall_source():
    p = cd.Problem(7, 4)
    f = p.source()
    for k in range(4):
        g = 1.0 - math.exp(-10.0 * (k + 1) * p.tau)
        want = np.zeros((7, 7))
        want[:, -1] = p.planes[1][:, -1] * g
        assert np.allclose(f[k].reshape(7, 7), want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("eps", [0.05, 1.0])
def test_pinv_matches_dense_solve(eps):
    p = cd.Problem(3, 6, eps=eps, nu=0.1)
    y = np.random.default_rng(73).standard_normal((6, 9))
    P = heat.dense_P(p.K.toarray(), 6, p.tau, eps)
    assert np.allclose(p.Pinv(y).reshape(-1), np.linalg.solve(P, y.reshape(-1)), atol=1e-12)


def test_gmres_bec_equals_sequential():
    p = cd.Problem(15, 16)
    rhs = p.rhs()
    u, it, _ = p.gmres(rhs, tol=1e-12)
    ex = p.exact(rhs)
    assert np.linalg.norm(u - ex) / np.linalg.norm(ex) <= 1e-10
    assert it <= 8


def test_coarse_levels_are_rediscretisations():
    m1, n = 15, 8
    p = cd.Problem(m1, n)
    lv = p.levels()
    assert [l[0] for l in lv] == [15, 7, 3, 1]
    rng = np.random.default_rng(74)
    lam = 0.4 + 0.3j
    for m, *planes in lv:
        x = cd.nodes(m)                          # coarse nodes, h = 2/(m+1)
        X, Y = np.meshgrid(x, x, indexing="xy")
        Kc = cd.stiffness_planes(*cd.couplings(p.nu, 2.0 / (m + 1), *cd.wind(X, Y)))
        e = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        got = mg.apply_B(e, lam, *planes).reshape(-1)
        want = lam * e.reshape(-1) + p.tau * (Kc @ e.reshape(-1))
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("lam", [0.02 + 0.0j, 0.6 + 0.8j])
def test_vcycles_converge_to_direct_solve(lam):
    m1, n = 31, 16
    p = cd.Problem(m1, n)
    lv = p.levels()
    r = np.random.default_rng(75).standard_normal(p.m) + 0j
    B = (lam * np.eye(p.m) + p.tau * p.K.toarray())
    want = np.linalg.solve(B, r)
    e = mg.step2_levels(lv, np.array([lam]), r[None, :], cycles=60)[0]
    assert np.linalg.norm(e - want) / np.linalg.norm(want) <= 1e-9


@pytest.mark.slow
def test_table3_qualitative():
    """Example 3 set-up (left GMRES(50), zero guess, 1e-7 drop of the
    preconditioned residual), three V-cycles per block (a red-black smoother
    needs about three to do what the paper's one ILU-smoothed cycle does on
    this recirculating flow): BEC (eps = 0.5 tau) needs far fewer iterations
    than BC (eps = 1), about the same on two grids, and ends at a smaller RES.
    (Exact inner solves: 4 against 14-16 iterations.)"""
    its = {}
    for m1 in (15, 31):
        n = 32
        for name, eps in (("bec", None), ("bc", 1.0)):
            p = cd.Problem(m1, n, eps=eps)
            rhs = p.rhs()
            u, it, _ = p.gmres_left(rhs, tol=1e-7, inner="mg", cycles=3)
            res = np.linalg.norm(rhs - p.L(u)) / np.linalg.norm(rhs)
            its[(m1, name)] = (it, res)
    for m1 in (15, 31):
        assert 2 * its[(m1, "bec")][0] <= its[(m1, "bc")][0], its
        assert its[(m1, "bec")][1] < its[(m1, "bc")][1], its
    assert abs(its[(15, "bec")][0] - its[(31, "bec")][0]) <= 1, its
