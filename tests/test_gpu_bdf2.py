"""BDF2 (aao_set_scheme(ctx, 2)) on the GPU against the p-step oracle
(oracle/bdf.py), through the C ABI.  Tolerances as for backward Euler:
L v and the right-hand side 1e-12, P^{-1} 1e-11, FP64 solves 1e-10, the FP32
preconditioner under FP64 FGMRES 1e-8 (derivations in the parity tests'
header; the BDF2 coefficients are O(1) and change none of them)."""
import numpy as np
import pytest

from oracle import bdf
import workloads as W
from errnorms import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solver(dim, m1, n, eps, T=1.0, precision="fp64", side="right"):
    from paper_2002_01108_amd import Solver
    s = Solver(dim, m1, n, T=T, eps=eps, precision=precision)
    s.set_scheme(2)
    s.set_side(side)
    return s


GRIDS = [(1, 63, 64, 0.125), (1, 5, 2, 0.5), (2, 37, 32, 0.1), (2, 127, 32, 0.15),
         (3, 13, 16, 0.25), (3, 20, 64, 0.125)]


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_apply_A_and_rhs(dim, m1, n, eps):
    p = bdf.Problem(m1, dim, n, r=bdf.BDF2, eps=eps)
    rng = np.random.default_rng(41)
    v = rng.standard_normal((n, p.m))
    f = rng.standard_normal((n, p.m))
    u0 = rng.standard_normal(p.m)
    s = solver(dim, m1, n, eps)
    assert rel(host(s.apply_A(dev(v))), p.L(v)) <= 1e-12
    assert rel(host(s.build_rhs(dev(f), dev(u0))), p.rhs(f, u0)) <= 1e-12


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_apply_Pinv(dim, m1, n, eps):
    p = bdf.Problem(m1, dim, n, r=bdf.BDF2, eps=eps)
    y = np.random.default_rng(42).standard_normal((n, p.m))
    s = solver(dim, m1, n, eps)
    assert rel(host(s.apply_Pinv(dev(y))), p.Pinv(y)) <= 1e-11


@pytest.mark.parametrize("dim,m1,n,eps", [(1, 63, 64, 0.125), (2, 37, 32, 0.1),
                                          (3, 13, 16, 0.25)])
def test_solve_matches_sequential_bdf2(dim, m1, n, eps):
    p = bdf.Problem(m1, dim, n, r=bdf.BDF2, eps=eps)
    rng = np.random.default_rng(43)
    rhs = p.rhs(rng.standard_normal((n, p.m)), rng.standard_normal(p.m))
    exact = p.exact(rhs)
    for side in ("right", "left"):
        s = solver(dim, m1, n, eps, side=side)
        u, info = s.solve(dev(rhs), tol=1e-12, maxit=200)
        assert info["status"] == 0
        assert rel(host(u), exact) <= 1e-10


def test_left_iterate_matches_oracle():
    """Equal step count, equal iterate (C1 grid, BDF2)."""
    w = W.WORKLOADS["heat1d_63x64"]
    p = bdf.Problem(w.m1, w.dim, w.n, r=bdf.BDF2, eps=w.epsilon)
    f, u0, _ = W.make(w)
    rhs = p.rhs(f, u0)
    for k in (1, 2, 3):
        x_or, it, _ = p.gmres_left(rhs, tol=0.0, maxit=k)
        s = solver(w.dim, w.m1, w.n, w.epsilon, side="left")
        u, info = s.solve(dev(rhs), tol=0.0, maxit=k)
        assert it == k and info["iters"] == k
        assert rel(host(u), x_or) <= 1e-10


def test_table_bdf2_counts_match_oracle():
    """The Table bdf2table set-up (a = 1e-5 as T = a, u0 = x(x-1)y(y-1), f = 0,
    left GMRES(50), 1e-7 drop), N = 64, 31^2 interior points: the GPU takes the
    oracle's iteration count for BEC (exactly) and BC (within one, for the
    reason given in the Table 1 test of the left/BC tests)."""
    n, m1, a = 64, 31, 1e-5
    x = W.node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = (X * (X - 1) * Y * (Y - 1)).reshape(-1)
    for bec in (True, False):
        eps = min(0.5, 0.5 / n) if bec else 1.0
        p = bdf.Problem(m1, 2, n, r=bdf.BDF2, eps=eps, a=a)
        rhs = p.rhs(np.zeros((n, p.m)), u0)
        _, it_or, _ = p.gmres_left(rhs, tol=1e-7)
        s = solver(2, m1, n, eps, T=a, side="left")
        u, info = s.solve(dev(rhs), tol=1e-7, maxit=300, restart=50)
        print(f"{'BEC' if bec else 'BC'}: GPU {info['iters']} oracle {it_or}", flush=True)
        assert info["status"] == 0
        assert (info["iters"] == it_or) if bec else (abs(info["iters"] - it_or) <= 1)


def test_fp32_preconditioner_recovers_fp64():
    dim, m1, n, eps = 2, 37, 32, 0.1
    p = bdf.Problem(m1, dim, n, r=bdf.BDF2, eps=eps)
    rng = np.random.default_rng(44)
    rhs = p.rhs(rng.standard_normal((n, p.m)), rng.standard_normal(p.m))
    exact = p.exact(rhs)
    s = solver(dim, m1, n, eps, precision="fp32")
    u, info = s.solve(dev(rhs), tol=1e-10, maxit=200)
    assert info["status"] == 0
    assert rel(host(u), exact) <= 1e-8


def test_scheme_switch_back_to_backward_euler():
    """Order 2 then order 1 on one context: L and P^{-1} are backward Euler again."""
    from oracle import heat
    dim, m1, n, eps = 2, 20, 16, 0.2
    s = solver(dim, m1, n, eps)
    s.set_scheme(1)
    p = heat.Problem(m1, dim, n, eps=eps)
    v = np.random.default_rng(45).standard_normal((n, p.m))
    assert rel(host(s.apply_A(dev(v))), p.L(v)) <= 1e-12
    assert rel(host(s.apply_Pinv(dev(v))), p.Pinv(v)) <= 1e-11
    assert s.lib.aao_set_scheme(s._h, 3) == -1      # AAO_EINVAL
