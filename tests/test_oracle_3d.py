"""Pins of the oracle's exact solve on 3D grids: sequential backward Euler
(Section 2, eq. (stepsystem)) with each step solved in the sine basis.

The sine-basis solve rests on two textbook facts, pinned here against
definitions written out independently of it: the orthonormal DST-I matrix S is
symmetric with S^2 = I, and S diagonalises the finite-difference K_h with the
closed-form eigenvalues.  The stepping itself is pinned against the sparse-LU
stepping (the plain definition), a closed-form eigenmode decay, and the
residual of L u = f.
"""
import math

import numpy as np
import pytest

from oracle import heat
import workloads as W


def dst_matrix(m):
    """S_{ij} = sqrt(2/(m+1)) sin(pi i j/(m+1)), i, j = 1..m, written out."""
    i = np.arange(1, m + 1)
    return math.sqrt(2.0 / (m + 1)) * np.sin(math.pi * np.outer(i, i) / (m + 1))


def test_sine_transform_is_the_written_out_dst_matrix():
    rng = np.random.default_rng(0)
    ms = (5, 4, 3)                     # x, y, z
    v = rng.standard_normal(tuple(reversed(ms)))
    Sx, Sy, Sz = (dst_matrix(m) for m in ms)
    want = np.einsum("ai,bj,ck,kji->cba", Sx, Sy, Sz, v)
    assert np.allclose(heat.sine_transform(v), want, atol=1e-14)


def test_sine_transform_is_an_involution():
    v = np.random.default_rng(1).standard_normal((6, 7, 9))
    assert np.allclose(heat.sine_transform(heat.sine_transform(v)), v, atol=1e-14)


@pytest.mark.parametrize("ms", [(5, 4, 3), (9, 9, 9), (8, 3, 6)])
def test_sine_basis_diagonalises_K(ms):
    """K_h (Kronecker sum with per-axis spacing) = S diag(mu) S."""
    K = heat.stiffness_rect(ms)
    mu = heat.fd_eigenvalues(ms)
    x = np.random.default_rng(2).standard_normal(mu.shape)
    lhs = (K @ x.reshape(-1)).reshape(mu.shape)
    rhs = heat.sine_transform(mu * heat.sine_transform(x))
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-10 * np.abs(lhs).max())


@pytest.mark.parametrize("m1,n", [(7, 8), (12, 5), (15, 16)])
def test_sine_stepping_equals_sparse_lu_stepping(m1, n):
    p = heat.Problem(m1, 3, n)
    rng = np.random.default_rng(3)
    rhs = p.rhs(rng.standard_normal((n, p.m)), rng.standard_normal(p.m))
    a = heat.sequential_be_sine((m1,) * 3, p.tau, rhs)
    b = heat.sequential_be(p.K, p.tau, rhs)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13
    assert np.abs(a - b).max() / np.abs(b).max() < 1e-13
    assert np.array_equal(p.exact(rhs), a)       # Problem.exact takes this route in 3D


def test_sine_stepping_eigenmode_closed_form():
    """f = 0, u0 = sin(pi x) sin(2 pi y) sin(3 pi z): u^k = (1 + tau mu)^{-k} u0 with
    mu = sum_d 4 h^-2 sin^2(p_d pi h / 2) (backward Euler on an eigenvector)."""
    m1, n = 15, 12
    tau = 1.0 / n
    x = W.node_coords(m1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u0 = (np.sin(math.pi * X) * np.sin(2 * math.pi * Y) * np.sin(3 * math.pi * Z)).reshape(-1)
    h = 1.0 / (m1 + 1)
    mu = sum(4 / h ** 2 * math.sin(p * math.pi * h / 2) ** 2 for p in (1, 2, 3))
    rhs = heat.build_rhs(np.zeros((n, u0.size)), u0, tau)
    u = heat.sequential_be_sine((m1,) * 3, tau, rhs)
    want = np.stack([(1 + tau * mu) ** -(k + 1) * u0 for k in range(n)])
    assert np.abs(u - want).max() <= 1e-14 * np.abs(u0).max()


def test_sine_stepping_residual_medium_grid():
    """|L u - f| / |f| at rounding level on a 31^3 x 16 grid with white-noise data."""
    m1, n = 31, 16
    p = heat.Problem(m1, 3, n)
    rng = np.random.default_rng(4)
    rhs = p.rhs(rng.standard_normal((n, p.m)), rng.standard_normal(p.m))
    u = p.exact(rhs)
    assert np.linalg.norm(p.L(u) - rhs) / np.linalg.norm(rhs) < 1e-14


def test_sine_stepping_rectangular():
    ms, n = (9, 6, 4), 8
    K = heat.stiffness_rect(ms)
    tau = 1.0 / n
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal((n, K.shape[0]))
    a = heat.sequential_be_sine(ms, tau, rhs)
    b = heat.sequential_be(K, tau, rhs)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13


@pytest.mark.parametrize("ms,n", [((31, 31), 8), ((20, 9), 6), ((63,), 16)])
def test_sine_stepping_1d_2d(ms, n):
    """The same route on 1D and 2D grids (the benchmark's oracle references for
    its 2D workloads use it) against the sparse-LU stepping."""
    K = heat.stiffness_rect(ms)
    tau = 1.0 / n
    rng = np.random.default_rng(6)
    rhs = rng.standard_normal((n, K.shape[0]))
    a = heat.sequential_be_sine(ms, tau, rhs)
    b = heat.sequential_be(K, tau, rhs)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13
    assert np.abs(a - b).max() / np.abs(b).max() < 1e-13


@pytest.mark.parametrize("ms,n", [((7, 5, 6), 4), ((9, 8), 6), ((11,), 8)])
def test_step2_sine_equals_sparse_lu_step2(ms, n):
    """Step 2 in the sine basis against the sparse complex LU of every block
    B_k = lambda_k I + tau K_h (the oracle's plain Step 2) on rectangular grids:
    the same linear solves, so agreement to rounding."""
    K = heat.stiffness_rect(ms)
    tau, eps = 1.0 / n, 0.2
    lam = heat.lambdas(n, eps)[: n // 2 + 1]
    rng = np.random.default_rng(5)
    yt = rng.standard_normal((n // 2 + 1, K.shape[0])) + 1j * rng.standard_normal(
        (n // 2 + 1, K.shape[0]))
    want = heat.step2(K, tau, lam, yt)
    got = heat.step2_sine(ms, tau, lam, yt)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13
