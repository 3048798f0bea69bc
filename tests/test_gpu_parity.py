"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (relative 2-norm unless stated), derived from the arithmetic:
  FP64 steps 1/3 and L v      1e-12   (u = 1.1e-16, log2 n passes, eps^{-1} <= 32)
  FP64 step 2 / P^{-1}        1e-11   (dense orthogonal transforms, K <= 1024 terms)
  FP64 solve                  1e-10   (iterate at equal k, and vs sequential BE)
  FP32 steps                  3e-5    (u = 6e-8, same growth factors)
  mixed / learned solves      1e-8    (after FGMRES, against the FP64 oracle)
"""
import math

import numpy as np
import pytest

from oracle import heat
import workloads as W
from errnorms import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solver(dim, m1, n, eps, precision="fp64", T=1.0):
    from paper_2002_01108_amd import Solver
    return Solver(dim, m1, n, T=T, eps=eps, precision=precision)


GRIDS = [  # (dim, m1, n, eps): ragged tiles, several tiles, every FFT length class
    (1, 63, 64, 0.125),
    (1, 5, 2, 0.5),
    (1, 37, 4, 0.3),
    (1, 64, 8, 0.2),
    (1, 130, 16, 0.25),
    (1, 19, 1024, 0.03),
    (2, 37, 32, 0.1),
    (2, 100, 128, 1.0 / 11),
    (2, 65, 512, 0.05),
    (2, 128, 256, 1.0),
    (2, 127, 32, 0.15),
    (3, 13, 16, 0.25),
    (3, 20, 64, 0.125),
    (3, 9, 2, 0.3),       # fewer time levels than one chunk
]


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_apply_A(dim, m1, n, eps):
    p = heat.Problem(m1, dim, n, eps=eps)
    x = _rand((n, p.m), 1)
    s = solver(dim, m1, n, eps)
    y = host(s.apply_A(dev(x)))
    assert rel(y, p.L(x)) <= 1e-12


@pytest.mark.parametrize("m1,n,two", [(70, 8, False), (70, 8, True), (130, 2, False),
                                      (67, 16, True)])
def test_apply_A_3d_walk(m1, n, two):
    """3D L v (backward Euler, and BDF2's three-term rows) across several z
    ranges of the z-marching walk (64 planes each, ragged last range) and time
    chunks, including fewer levels than one chunk."""
    from oracle import bdf
    x = _rand((n, m1 ** 3), 31)
    s = solver(3, m1, n, 0.2)
    if two:
        s.set_scheme(2)
        want = bdf.Problem(m1, 3, n, r=bdf.BDF2, eps=0.2).L(x)
    else:
        want = heat.Problem(m1, 3, n, eps=0.2).L(x)
    assert rel(host(s.apply_A(dev(x))), want) <= 1e-12


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_step1(dim, m1, n, eps):
    p = heat.Problem(m1, dim, n, eps=eps)
    y = _rand((n, p.m), 2)
    s = solver(dim, m1, n, eps)
    yt = host(s.step1(dev(y)))
    got = yt[..., 0] + 1j * yt[..., 1]
    want = heat.step1(y, eps)
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_step3(dim, m1, n, eps):
    p = heat.Problem(m1, dim, n, eps=eps)
    rng = np.random.default_rng(3)
    zt = rng.standard_normal((n // 2 + 1, p.m, 2))
    s = solver(dim, m1, n, eps)
    z = host(s.step3(dev(zt)))
    want = heat.step3(zt[..., 0] + 1j * zt[..., 1], eps, n)
    assert rel(z, want) <= 1e-12


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_step2(dim, m1, n, eps):
    p = heat.Problem(m1, dim, n, eps=eps)
    rng = np.random.default_rng(4)
    yt = rng.standard_normal((n // 2 + 1, p.m, 2))
    yt[0, :, 1] = 0.0
    yt[-1, :, 1] = 0.0
    s = solver(dim, m1, n, eps)
    zt = host(s.step2(dev(yt)))
    lam = heat.lambdas(n, eps)[: n // 2 + 1]
    want = heat.step2(p.K, p.tau, lam, yt[..., 0] + 1j * yt[..., 1])
    assert rel(zt[..., 0] + 1j * zt[..., 1], want) <= 1e-11


@pytest.mark.parametrize("dim,m1,n,eps", GRIDS)
def test_apply_Pinv(dim, m1, n, eps):
    p = heat.Problem(m1, dim, n, eps=eps)
    y = _rand((n, p.m), 5)
    s = solver(dim, m1, n, eps)
    z = host(s.apply_Pinv(dev(y)))
    assert rel(z, p.Pinv(y)) <= 1e-11
    assert rel(p.P(z), y) <= 1e-11


def test_apply_Pinv_in_place():
    dim, m1, n, eps = 2, 37, 32, 0.1
    p = heat.Problem(m1, dim, n, eps=eps)
    y = _rand((n, p.m), 6)
    s = solver(dim, m1, n, eps)
    t = dev(y)
    s.apply_Pinv(t, out=t)
    assert rel(host(t), p.Pinv(y)) <= 1e-11


def test_build_rhs():
    w = W.WORKLOADS["heat1d_63x64"]
    f, u0, _ = W.make(w)
    s = solver(1, w.m1, w.n, w.epsilon)
    got = host(s.build_rhs(dev(f), dev(u0)))
    assert np.array_equal(got, heat.build_rhs(f, u0, w.tau)) or rel(got, heat.build_rhs(f, u0, w.tau)) <= 1e-15


def test_repeat_is_deterministic():
    dim, m1, n, eps = 2, 100, 32, 0.1
    y = dev(_rand((n, m1 * m1), 7))
    s = solver(dim, m1, n, eps)
    a = host(s.apply_Pinv(y))
    b = host(s.apply_Pinv(y))
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ solve

def _c1():
    w = W.WORKLOADS["heat1d_63x64"]
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    f, u0, _ = W.make(w)
    return w, p, p.rhs(f, u0)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_solve_iterate_matches_oracle_gmres(k):
    """Same Krylov step count k on both sides (tol = 0, maxit = k)."""
    w, p, rhs = _c1()
    x_or, it, _ = p.gmres(rhs, tol=0.0, maxit=k)
    assert it == k
    s = solver(w.dim, w.m1, w.n, w.epsilon)
    u, info = s.solve(dev(rhs), tol=0.0, maxit=k)
    assert info["iters"] == k
    assert rel(host(u), x_or) <= 1e-10


def test_solve_matches_sequential_be():
    w, p, rhs = _c1()
    exact = p.exact(rhs)
    s = solver(w.dim, w.m1, w.n, w.epsilon)
    u, info = s.solve(dev(rhs), tol=1e-12)
    assert info["status"] == 0
    assert rel(host(u), exact) <= 1e-10


def test_solve_metric_run_c1():
    """tol 1e-8: same iteration count as the oracle, explicit RES within tol."""
    w, p, rhs = _c1()
    _, it_or, hist_or = p.gmres(rhs, tol=1e-8)
    s = solver(w.dim, w.m1, w.n, w.epsilon)
    u, info = s.solve(dev(rhs), tol=1e-8)
    assert info["iters"] == it_or == 2
    assert info["final_res"] <= 1e-8
    np.testing.assert_allclose(info["hist"], hist_or, rtol=1e-6)


@pytest.mark.parametrize("dim,m1,n", [(2, 100, 32), (3, 20, 16), (2, 65, 512), (3, 70, 8)])
def test_solve_grids(dim, m1, n):
    p = heat.Problem(m1, dim, n)
    f = _rand((n, p.m), 8)
    u0 = W.initial_value(m1, dim, "modes", 9)
    rhs = p.rhs(f, u0)
    exact = p.exact(rhs)
    s = solver(dim, m1, n, p.eps)
    u, info = s.solve(dev(rhs), tol=1e-12)
    assert info["status"] == 0 and info["iters"] <= 4
    assert rel(host(u), exact) <= 1e-10


def test_solve_restart_and_guess():
    """Restart length 1 (many cycles) and a warm start reach the same solution."""
    w, p, rhs = _c1()
    exact = p.exact(rhs)
    s = solver(w.dim, w.m1, w.n, w.epsilon)
    u, info = s.solve(dev(rhs), tol=1e-12, restart=1, maxit=20)
    assert info["status"] == 0
    assert rel(host(u), exact) <= 1e-10
    u2, info2 = s.solve(dev(rhs), tol=1e-12, u=u.clone(), use_guess=True)
    assert info2["iters"] <= 1
    assert rel(host(u2), exact) <= 1e-10


def test_solve_not_converged_and_nan():
    from paper_2002_01108_amd import AaoError
    w, p, rhs = _c1()
    s = solver(w.dim, w.m1, w.n, 1.0)          # block circulant: slow convergence
    u, info = s.solve(dev(rhs), tol=1e-14, maxit=2)
    assert info["status"] == 1 and info["iters"] == 2
    bad = rhs.copy()
    bad[3, 5] = np.nan
    with pytest.raises(AaoError) as e:
        s.solve(dev(bad))
    assert e.value.status == -4


def test_zero_rhs():
    s = solver(1, 15, 8, 0.2)
    u, info = s.solve(dev(np.zeros((8, 15))))
    assert info["iters"] == 0 and np.all(host(u) == 0)


# ------------------------------------------------------------------ FP32 preconditioner

@pytest.mark.parametrize("dim,m1,n,eps", [(1, 63, 64, 0.125), (2, 100, 128, 1.0 / 11),
                                          (3, 20, 64, 0.125), (2, 65, 512, 0.05),
                                          (2, 255, 8, 0.1), (2, 511, 4, 0.1)])
def test_fp32_steps(dim, m1, n, eps):
    """FP32 Steps 1 and P^{-1} against the oracle; 255^2 and 511^2 reach the
    two-level fold with 64 quarter indices per block (P = 256, 512)."""
    p = heat.Problem(m1, dim, n, eps=eps)
    s = solver(dim, m1, n, eps, precision="fp32")
    y = _rand((n, p.m), 10)
    yt = host(s.step1(dev(y)))
    assert rel(yt[..., 0] + 1j * yt[..., 1], heat.step1(y, eps)) <= 3e-5
    z = host(s.apply_Pinv(dev(y)))
    assert rel(z, p.Pinv(y)) <= 3e-5


@pytest.mark.parametrize("dim,m1,n", [(1, 63, 64), (2, 100, 32), (3, 20, 16)])
def test_fp32_fgmres_recovers_fp64(dim, m1, n):
    p = heat.Problem(m1, dim, n)
    f = _rand((n, p.m), 11)
    rhs = p.rhs(f, W.initial_value(m1, dim, "modes", 12))
    exact = p.exact(rhs)
    s = solver(dim, m1, n, p.eps, precision="fp32")
    u, info = s.solve(dev(rhs), tol=1e-10)
    assert info["status"] == 0
    assert info["final_res"] <= 1e-10
    assert rel(host(u), exact) <= 1e-8


# ------------------------------------------------------------------ BF16 hi/lo preconditioner
# Per product the split drops lo*lo (<= 2^-18 |ab|) and rounds both lo parts
# (<= 2^-17 |ab| each): <= 1.9e-5 relative, about 1e-5 for a sum of K random-sign
# terms; four mode products and the Gamma_eps^-1 growth (<= 33) give 3e-4.

@pytest.mark.parametrize("dim,m1,n,eps", [(1, 63, 64, 0.125), (2, 100, 128, 1.0 / 11),
                                          (3, 20, 64, 0.125), (2, 65, 512, 0.05)])
def test_bf16x3_steps(dim, m1, n, eps):
    p = heat.Problem(m1, dim, n, eps=eps)
    s = solver(dim, m1, n, eps, precision="bf16x3")
    y = _rand((n, p.m), 13)
    z = host(s.apply_Pinv(dev(y)))
    err = rel(z, p.Pinv(y))
    assert err <= 3e-4
    assert err >= 1e-9          # it really ran in reduced precision
    rng = np.random.default_rng(14)
    yt = rng.standard_normal((n // 2 + 1, p.m, 2))
    yt[0, :, 1] = 0.0
    yt[-1, :, 1] = 0.0
    zt = host(s.step2(dev(yt)))
    lam = heat.lambdas(n, eps)[: n // 2 + 1]
    want = heat.step2(p.K, p.tau, lam, yt[..., 0] + 1j * yt[..., 1])
    assert rel(zt[..., 0] + 1j * zt[..., 1], want) <= 3e-4


@pytest.mark.parametrize("dim,m1,n", [(1, 63, 64), (2, 100, 32), (3, 20, 16)])
def test_bf16x3_fgmres_recovers_fp64(dim, m1, n):
    p = heat.Problem(m1, dim, n)
    f = _rand((n, p.m), 15)
    rhs = p.rhs(f, W.initial_value(m1, dim, "modes", 16))
    exact = p.exact(rhs)
    s = solver(dim, m1, n, p.eps, precision="bf16x3")
    u, info = s.solve(dev(rhs), tol=1e-10)
    assert info["status"] == 0
    assert info["final_res"] <= 1e-10
    assert rel(host(u), exact) <= 1e-8


# ---------------------------------------------------------------------------
# rectangular grids: every axis has its own length and spacing 1/(m_d + 1);
# mixes the one- and two-level folded products (odd/even lengths, paddings of
# 64 and 128) across the axes
RECT = [  # (dim, (m1, m2[, m3]), n, eps)
    (2, (37, 20), 16, 0.2),
    (2, (101, 65), 8, 0.15),
    (2, (64, 127), 8, 0.1),
    (3, (13, 9, 5), 8, 0.25),
    (3, (65, 20, 33), 4, 0.2),
    (3, (9, 33, 130), 4, 0.2),   # 3D walk: three z ranges (64 + 64 + 2 planes)
    (3, (127, 127, 3), 4, 0.2),  # FP64: x and y in one slab launch (P1 = P2 = 128, m1 = m2)
    (3, (65, 65, 2), 8, 0.15),   # the same at the shortest length accepted there
]


def rect_solver(dim, ms, n, eps, precision="fp64"):
    from paper_2002_01108_amd import Solver
    ms = list(ms) + [1] * (3 - len(ms))
    return Solver(dim, ms[0], n, T=1.0, eps=eps, precision=precision, m2=ms[1], m3=ms[2])


@pytest.mark.parametrize("dim,ms,n,eps", RECT)
def test_rect_apply_A_and_Pinv(dim, ms, n, eps):
    K = heat.stiffness_rect(ms)
    m = K.shape[0]
    tau = 1.0 / n
    s = rect_solver(dim, ms, n, eps)
    v = _rand((n, m), 40 + dim)
    assert rel(host(s.apply_A(dev(v))), heat.apply_L(K, tau, v)) < 1e-12
    assert rel(host(s.apply_Pinv(dev(v))), heat.apply_Pinv(K, tau, eps, v)) < 1e-11


@pytest.mark.parametrize("dim,ms,n,eps", [RECT[4], RECT[6], RECT[7]])
def test_rect_step2(dim, ms, n, eps):
    """Step 2 alone on rectangular 3D grids (the x-y slab launch with unpacked
    frequency blocks on RECT[6], RECT[7]) against the oracle's block solves."""
    K = heat.stiffness_rect(ms)
    m = K.shape[0]
    tau = 1.0 / n
    rng = np.random.default_rng(41)
    yt = rng.standard_normal((n // 2 + 1, m, 2))
    yt[0, :, 1] = 0.0
    yt[-1, :, 1] = 0.0
    s = rect_solver(dim, ms, n, eps)
    zt = host(s.step2(dev(yt)))
    lam = heat.lambdas(n, eps)[: n // 2 + 1]
    want = heat.step2(K, tau, lam, yt[..., 0] + 1j * yt[..., 1])
    assert rel(zt[..., 0] + 1j * zt[..., 1], want) <= 1e-11


@pytest.mark.parametrize("dim,ms,n,eps", [RECT[1], RECT[4]])
def test_rect_solve_matches_sequential_be(dim, ms, n, eps):
    K = heat.stiffness_rect(ms)
    m = K.shape[0]
    tau = 1.0 / n
    s = rect_solver(dim, ms, n, eps)
    rhs = _rand((n, m), 50 + dim)
    u, info = s.solve(dev(rhs), tol=1e-12, maxit=50)
    assert info["status"] == 0
    assert rel(host(u), heat.sequential_be(K, tau, rhs)) < 1e-10


def test_pinv_127_cubed_elementwise():
    """127^3 x 4 (m + 1 = 128 on every axis): the x-y slab launch and the
    in-place z pass (forward product, divide, inverse product) on the third
    fold, against the oracle's three steps with Step 2 in the sine basis,
    element by element; FP32 (its own z kernel) by the backward error."""
    ms, n, eps = (127, 127, 127), 4, 0.2
    m = 127 ** 3
    tau = 1.0 / n
    v = _rand((n, m), 70)
    lam = heat.lambdas(n, eps)[: n // 2 + 1]
    want = heat.step3(heat.step2_sine(ms, tau, lam, heat.step1(v, eps), workers=8), eps, n)
    s = rect_solver(3, ms, n, eps)
    z = host(s.apply_Pinv(dev(v)))
    err = rel(z, want)
    mx = float(np.abs(z - want).max() / np.abs(want).max())
    print(f"127^3 x 4 P^-1: rel {err:.2e}, max-abs {mx:.2e}", flush=True)
    assert err < 1e-11 and mx < 1e-11
    s32 = rect_solver(3, ms, n, eps, precision="fp32")
    z32 = host(s32.apply_Pinv(dev(v)))
    back = rel(heat.apply_P(heat.stiffness_rect(ms), tau, eps, z32), v)
    assert 1e-9 <= back < 5e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("dim,ms,n,eps", RECT)
def test_rect_reduced_Pinv(dim, ms, n, eps, precision):
    """Reduced-precision preconditioner on every rectangular grid (both fold
    tile heights, ragged lengths along each axis, several z ranges), above 1e-9
    so that it did run in reduced precision.
    FP32: backward error against the oracle's P_eps, 5e-5 (the forward error
    also carries cond(P_eps) ~ 1 + 4 d tau / h^2 on white noise; the two-level
    fold rounds the +- combinations of the inputs once more: 3.3e-5 measured
    on (64, 127) x 8).
    BF16x3: forward error against the oracle's P_eps^{-1} at the bound of the
    split (3e-4, as for the square grids).  Its backward error multiplies the
    white split error of the inverse sine transforms by lambda + tau mu, up to
    1e4 on these grids: 3e-4 to 7e-4 measured, printed here."""
    K = heat.stiffness_rect(ms)
    tau = 1.0 / n
    s = rect_solver(dim, ms, n, eps, precision=precision)
    v = _rand((n, K.shape[0]), 60 + dim)
    z = host(s.apply_Pinv(dev(v)))
    back = rel(heat.apply_P(K, tau, eps, z), v)
    if precision == "fp32":
        assert 1e-9 <= back < 5e-5
    else:
        fwd = rel(z, heat.apply_Pinv(K, tau, eps, v))
        print(f"{ms} x {n} bf16x3: forward {fwd:.2e}, backward {back:.2e}", flush=True)
        assert 1e-9 <= fwd <= 3e-4
