"""Parity at the full workload sizes, in the launch configuration the benchmark
times, through the C ABI.

  * L v against the oracle's sparse operator (whole array: 2D and the 3D
    127^3 x 256 workload);
  * P^{-1} against the oracle's three-step inverse (naive DFT + sparse LU per
    block) on the whole heat2d 255^2 x 256 array, element by element;
  * P^{-1} (P v) = v, with P v = L v - eps [v^N, 0, ..., 0] (Section 3), for
    every precision and for the 3D workload (the oracle's P^{-1} is out of
    reach there);
  * the solves against the oracle's sequential backward-Euler solution (2D:
    sparse LU per step; 3D: the sine-basis solve of each step), FP64 at
    1e-10 and the reduced-precision preconditioners at 1e-8 after FGMRES.
Tolerances as in the small-size parity tests; P^{-1} P v carries the
eps^{-1} growth of the Gamma_eps scaling.
"""
import os

import numpy as np
import pytest

from oracle import heat
import workloads as W
from errnorms import rel, trel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


def make_solver(w, precision):
    from paper_2002_01108_amd import Solver
    return Solver(w.dim, w.m1, w.n, T=w.T, eps=w.epsilon, precision=precision)


def seeded_gpu(w, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn((w.n, w.m), dtype=torch.float64, device="cuda", generator=g)


def oracle_workers():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.mark.parametrize("name", ["heat2d_255x256", "heat2d_511x512", "heat3d_127x256"])
def test_apply_A_full(name):
    w = W.WORKLOADS[name]
    s = make_solver(w, "fp64")
    x = seeded_gpu(w, 11)
    y = s.apply_A(x)
    torch.cuda.synchronize()
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    ref = p.L(x.cpu().numpy())
    assert rel(y.cpu().numpy(), ref) < 1e-12


def test_pinv_vs_oracle_c2():
    """heat2d 255^2 x 256, FP64: the GPU's P^{-1} against the oracle's three steps
    (explicit Fourier matrix, one sparse complex LU per kept block) on the whole
    array, element by element (relative 2-norm and normalised max-abs)."""
    w = W.WORKLOADS["heat2d_255x256"]
    s = make_solver(w, "fp64")
    x = seeded_gpu(w, 13)
    z = s.apply_Pinv(x)
    torch.cuda.synchronize()
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    ref = p.Pinv(x.cpu().numpy())
    err = rel(z.cpu().numpy(), ref)
    print(f"P^-1 vs oracle at 255^2 x 256: {err:.2e}", flush=True)
    assert err < 1e-11


PINV_CASES = [  # (workload, precision, forward tolerance, backward tolerance)
    ("heat2d_255x256", "fp64", 1e-11, 1e-13),
    ("heat2d_511x512", "fp64", 1e-11, 1e-13),
    ("heat2d_511x512", "fp32", None, 3e-5),
    ("heat2d_511x512", "bf16x3", None, 3e-4),
    ("heat3d_127x256", "fp32", None, 3e-5),
    ("heat3d_127x256", "fp64", 1e-11, 1e-13),
]


def apply_P(s, w, v):
    pv = s.apply_A(v)
    pv[0] -= w.epsilon * v[-1]
    return pv


@pytest.mark.parametrize("name,precision,ftol,btol", PINV_CASES)
def test_pinv_inverts_P_full(name, precision, ftol, btol):
    """z = P^{-1} b for b = P v.  Backward error |P z - b|/|b| (what the outer
    FGMRES sees) for every precision; forward error |z - v|/|v| in FP64 only,
    since in reduced precision it also carries cond(P) ~ 1 + 4 d tau/h^2
    (thousands here) on a white-noise v."""
    w = W.WORKLOADS[name]
    s = make_solver(w, precision)
    v = seeded_gpu(w, 12)
    b = apply_P(s, w, v)
    z = s.apply_Pinv(b)
    back = trel(apply_P(s, w, z), b)
    fwd = trel(z, v)
    torch.cuda.synchronize()
    print(f"{name} {precision}: forward {fwd:.2e} backward {back:.2e}", flush=True)
    assert back < btol
    if ftol is not None:
        assert fwd < ftol


@pytest.fixture(scope="module")
def c3_exact():
    w = W.WORKLOADS["heat2d_511x512"]
    f, u0, _ = W.make(w)
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    return w, f, u0, p.exact(p.rhs(f, u0))


def _gpu_solve(w, f, u0, precision, tol, restart=50):
    s = make_solver(w, precision)
    rhs = s.build_rhs(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda())
    u, info = s.solve(rhs, tol=tol, maxit=200, restart=restart)
    torch.cuda.synchronize()
    return u.cpu().numpy(), info


def test_solve_c2_fp64_vs_sequential_be():
    w = W.WORKLOADS["heat2d_255x256"]
    f, u0, _ = W.make(w)
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    exact = p.exact(p.rhs(f, u0))
    u, info = _gpu_solve(w, f, u0, "fp64", 1e-8)
    assert info["status"] == 0 and info["final_res"] <= 1e-8
    assert rel(u, exact) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_solve_c3_vs_sequential_be(c3_exact, precision):
    w, f, u0, exact = c3_exact
    u, info = _gpu_solve(w, f, u0, precision, 1e-8)
    assert info["status"] == 0 and info["final_res"] <= 1e-8
    err = rel(u, exact)
    print(f"{precision}: iters {info['iters']} rel.err {err:.2e}", flush=True)
    assert err < (1e-10 if precision == "fp64" else 1e-8)


@pytest.fixture(scope="module")
def c4_exact():
    w = W.WORKLOADS["heat3d_127x256"]
    f, u0, _ = W.make(w)
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    rhs = p.rhs(f, u0)
    return w, p, f, u0, rhs, p.exact(rhs, workers=oracle_workers())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_c4_vs_sequential_be(c4_exact, precision):
    """heat3d 127^3 x 256 (524 M unknowns) against the oracle's sequential
    backward Euler: FP64 1e-10, the FP32 preconditioner 1e-8 after FGMRES; the
    oracle's residual of the GPU solution as well."""
    w, p, f, u0, rhs, exact = c4_exact
    u, info = _gpu_solve(w, f, u0, precision, 1e-8, restart=10)
    assert info["status"] == 0 and info["final_res"] <= 1e-8
    err = rel(u, exact)
    res = float(np.linalg.norm(p.L(u) - rhs) / np.linalg.norm(rhs))
    print(f"{precision}: iters {info['iters']} rel.err {err:.2e} oracle relres {res:.2e}",
          flush=True)
    assert err < (1e-10 if precision == "fp64" else 1e-8)
    assert res < 2e-8
