"""Equal-step-count parity of the Krylov iterates: the GPU's FGMRES iterate after
exactly k Arnoldi steps (tol = 0, maxit = k) against the oracle's textbook
FGMRES iterate after k steps with the oracle's own preconditioner (Section 5:
restarted GMRES from a zero guess; right preconditioning).

* FP64 exact inner solve, 1D/2D/3D: both sides apply the same P_eps^{-1}, so the
  iterates agree to rounding: 1e-10.
* FP64 multigrid inner solve (variable coefficient, Section 5, Example 2's one
  V-cycle): the oracle's V-cycle of oracle/mg.py in Step 2: 1e-10.
* FP32 and BF16x3 preconditioners against the oracle's FP64 P_eps^{-1}: the
  iterates differ by the preconditioner's own error (3e-5 and 3e-4, the
  tolerances of the reduced-precision P^{-1} parity), not more: a wrong
  Arnoldi or update step would show an O(1) difference.
* The learned inner solve (FP32 network) against oracle/cnn.py's inner_apply:
  the network's FP32 rounding on its correction, 1e-5 (the FP32 network
  tolerance of the other learned-solve tests).
"""
import numpy as np
import pytest

from errnorms import rel
from oracle import cnn, heat, mg
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def problem_rhs(p, seed):
    f = np.random.default_rng(seed).standard_normal((p.n, p.m))
    return p.rhs(f, W.initial_value(p.m1, p.dim, "modes", seed + 1))


def gpu_iterate(s, rhs, k):
    u, info = s.solve(dev(rhs), tol=0.0, maxit=k, restart=50)
    assert info["iters"] == k
    return host(u), info


def _same_history(got, want):
    """Givens residual estimates agree where they are above rounding level."""
    got, want = np.asarray(got), np.asarray(want)
    assert got.shape == want.shape
    big = want > 1e-11
    # relative 1e-6 where the estimate is large; below, the Givens recurrence
    # carries rounding of order 1e-16 relative to ||rhs|| (CGS2 against MGS)
    np.testing.assert_allclose(got[big], want[big], rtol=1e-6, atol=1e-14)
    assert np.all(got[~big] <= 1e-10)


CASES = [(1, 63, 64, 0.125), (2, 37, 32, 0.1), (2, 100, 16, 1.0 / 11), (3, 13, 16, 0.25),
         (3, 20, 8, 0.125)]


@pytest.mark.parametrize("dim,m1,n,eps", CASES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 3e-5), ("bf16x3", 3e-4)])
def test_iterates_equal_k(dim, m1, n, eps, prec, tol):
    from paper_2002_01108_amd import Solver
    p = heat.Problem(m1, dim, n, eps=eps)
    rhs = problem_rhs(p, 50 + dim)
    s = Solver(dim, m1, n, T=1.0, eps=eps, precision=prec)
    for k in (1, 2, 3):
        x_or, it, hist_or = p.gmres(rhs, tol=0.0, maxit=k)
        assert it == k
        u, info = gpu_iterate(s, rhs, k)
        err = rel(u, x_or)
        print(f"{dim}D {m1} x {n} {prec} k={k}: iterate error {err:.2e}", flush=True)
        assert err <= tol
        if prec == "fp64":
            _same_history(info["hist"], hist_or)
        if prec == "bf16x3":
            assert err >= 1e-10 or k > 1     # the reduced precision really ran


def _mg_pinv(p, faces, cycles):
    lam = heat.lambdas(p.n, p.eps)[: p.n // 2 + 1]
    lv = mg.levels(np.asarray(faces[0], float), np.asarray(faces[1], float), p.tau)

    def Minv(v):
        yt = heat.step1(v.reshape(p.n, p.m), p.eps)
        zt = mg.step2_levels(lv, lam, yt, cycles)
        return heat.step3(zt, p.eps, p.n).reshape(-1)
    return Minv


@pytest.mark.parametrize("m1,n,cycles", [(31, 16, 1), (63, 8, 2)])
def test_iterates_equal_k_multigrid(m1, n, cycles):
    from paper_2002_01108_amd import Solver
    faces = W.grf_faces(m1, 2, seed=60)
    p = heat.Problem(m1, 2, n, faces=faces)
    rhs = problem_rhs(p, 61)
    s = Solver(2, m1, n, T=1.0, eps=p.eps)
    s.set_coefficient(faces)
    s.set_inner("mg", cycles)
    Minv = _mg_pinv(p, faces, cycles)
    for k in (1, 2, 3):
        x_or, it, hist_or = p.gmres(rhs, tol=0.0, maxit=k, Minv=Minv)
        u, info = gpu_iterate(s, rhs, k)
        err = rel(u, x_or)
        print(f"MG {m1} x {n} cycles {cycles} k={k}: iterate error {err:.2e}", flush=True)
        assert err <= 1e-10
        _same_history(info["hist"], hist_or)


def test_iterates_equal_k_learned():
    from paper_2002_01108_amd import Solver
    m1, n = 31, 8
    faces = W.grf_faces(m1, 2, seed=62)
    p = heat.Problem(m1, 2, n, faces=faces)
    rhs = problem_rhs(p, 63)
    prm = (W.cnn_init_params(5) + 0.05 * np.random.default_rng(64).standard_normal(
        W.cnn_init_params(5).size)).astype(np.float32)
    s = Solver(2, m1, n, T=1.0, eps=p.eps)
    s.set_coefficient(faces)
    s.cnn_set_params(prm)
    s.set_inner("cnn")
    lam = heat.lambdas(n, p.eps)[: n // 2 + 1]
    lv = mg.levels(faces[0], faces[1], p.tau)
    loga = cnn.node_log_coefficient(*faces)
    prm64 = prm.astype(np.float64)

    def Minv(v):
        yt = heat.step1(v.reshape(n, p.m), p.eps)
        zt = np.stack([cnn.inner_apply(prm64, lv, yt[k].reshape(m1, m1), lam[k], loga).reshape(-1)
                       for k in range(n // 2 + 1)])
        return heat.step3(zt, p.eps, n).reshape(-1)

    for k in (1, 2):
        x_or, it, _ = p.gmres(rhs, tol=0.0, maxit=k, Minv=Minv)
        u, _ = gpu_iterate(s, rhs, k)
        err = rel(u, x_or)
        print(f"CNN {m1} x {n} k={k}: iterate error {err:.2e}", flush=True)
        assert err <= 1e-5
