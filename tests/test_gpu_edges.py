"""Degenerate and maximum spatial sizes, through the C ABI, against the oracle.

* One interior point per axis (m = 1, h = 1/2): K is the scalar 2 d / h^2,
  the sine transform of length one is the identity, and the fold's only
  element is its own mirror.  Full parity: L, P^{-1} and the solve.
* The longest axis the library accepts (m = 1024, padded length P = 1024):
  1D with full parity (the dense product with P^{-1} from the oracle's
  per-frequency factorisations); 2D at 1024^2 (one-level fold with 512-wide
  halves) and 1023^2 (two-level fold at P = 1024), where the oracle's sparse
  LU per frequency is out of reach, through what holds at any size: L against
  the oracle's sparse matvec, and z = P^{-1} b for b = P v formed by the
  oracle, with backward error |P z - b| / |b| and forward error |z - v| / |v|.
  tau = 1/1024 keeps cond(P) ~ 1 + 8 tau / h^2 near 8e3, as in the full-size
  workloads.

For b = P v with white-noise v the residual |P z - b| / |b| of z = P^{-1} b
stays at a few ulps (orthogonal transforms and a diagonal divide), while the
error |z - v| / |v|, and the difference from the oracle's P^{-1} y on white
noise y, carry cond(P) ~ 1 + 4 d tau / h^2: their tolerance is
max(1e-11, 4 eps_mach cond(P)), 5.8e-11 at m = 1024 in 1D with tau = 1/64
(cond(P) = 6.6e4).
"""
import numpy as np
import pytest

from oracle import heat
from errnorms import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fwd_tol(dim, m1, tau):
    cond = 1.0 + 4.0 * dim * tau * (m1 + 1) ** 2
    return max(1e-11, 4.0 * np.finfo(np.float64).eps * cond)


def solver(dim, m1, n, T, eps):
    from paper_2002_01108_amd import Solver
    return Solver(dim, m1, n, T=T, eps=eps)


@pytest.mark.parametrize("dim,n,eps", [(1, 4, 0.5), (2, 8, 0.25), (3, 2, 1.0)])
def test_one_point_grid(dim, n, eps):
    p = heat.Problem(1, dim, n, eps=eps)
    assert p.m == 1 and p.K.toarray()[0, 0] == 8.0 * dim
    rng = np.random.default_rng(21 + dim)
    s = solver(dim, 1, n, 1.0, eps)
    x = rng.standard_normal((n, 1))
    assert rel(host(s.apply_A(dev(x))), p.L(x)) <= 1e-12
    y = rng.standard_normal((n, 1))
    z = host(s.apply_Pinv(dev(y)))
    assert rel(z, p.Pinv(y)) <= 1e-11
    assert rel(p.P(z), y) <= 1e-11
    f = rng.standard_normal((n, 1))
    u0 = rng.standard_normal(1)
    rhs = p.rhs(f, u0)
    u, info = s.solve(s.build_rhs(dev(f), dev(u0)), tol=1e-12)
    assert info["status"] == 0
    assert rel(host(u), p.exact(rhs)) <= 1e-10


def test_longest_axis_1d():
    m1, n, eps = 1024, 64, 0.05
    p = heat.Problem(m1, 1, n, eps=eps)
    rng = np.random.default_rng(31)
    s = solver(1, m1, n, 1.0, eps)
    x = rng.standard_normal((n, m1))
    assert rel(host(s.apply_A(dev(x))), p.L(x)) <= 1e-12
    y = rng.standard_normal((n, m1))
    z = host(s.apply_Pinv(dev(y)))
    assert rel(z, p.Pinv(y)) <= fwd_tol(1, m1, p.tau)
    b = p.P(x)
    z = host(s.apply_Pinv(dev(b)))
    assert rel(p.P(z), b) <= 1e-13
    assert rel(z, x) <= fwd_tol(1, m1, p.tau)
    f = rng.standard_normal((n, m1))
    u0 = rng.standard_normal(m1)
    # cond(L) ~ 1 + 4 tau / h^2 = 6.6e4 bounds the error by 6.6e4 x the residual
    u, info = s.solve(s.build_rhs(dev(f), dev(u0)), tol=1e-13)
    assert info["status"] == 0
    assert rel(host(u), p.exact(p.rhs(f, u0))) <= 1e-8


@pytest.mark.parametrize("m1", [1024, 1023])
def test_longest_axis_2d(m1):
    n, eps = 2, 0.1
    T = n / 1024.0
    p = heat.Problem(m1, 2, n, T=T, eps=eps)
    rng = np.random.default_rng(41 + m1)
    s = solver(2, m1, n, T, eps)
    x = rng.standard_normal((n, p.m))
    assert rel(host(s.apply_A(dev(x))), p.L(x)) <= 1e-12
    b = p.P(x)
    z = host(s.apply_Pinv(dev(b)))
    back, fwd = rel(p.P(z), b), rel(z, x)
    print(f"m1 {m1}: P^-1 backward {back:.2e} forward {fwd:.2e}", flush=True)
    assert back <= 1e-13
    assert fwd <= fwd_tol(2, m1, p.tau)
    if m1 == 1023:
        f = rng.standard_normal((n, p.m))
        u0 = rng.standard_normal(p.m)
        rhs = p.rhs(f, u0)
        u, info = s.solve(s.build_rhs(dev(f), dev(u0)), tol=1e-10)
        assert info["status"] == 0
        assert rel(p.L(host(u)), rhs) <= 2e-10
