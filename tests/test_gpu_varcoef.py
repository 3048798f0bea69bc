"""Variable-coefficient path on the GPU against the oracle: flux-form L v, the
multigrid and mean-coefficient inner solves of Step 2, and FGMRES solves.

Tolerances: FP64 1e-12 (L v), 1e-11 (one or more V-cycles: a few hundred
flops per point per level, no cancellation); FP32 V-cycle 1e-5; solves 1e-8
against sequential backward Euler with K_a.
"""
import numpy as np
import pytest

from oracle import heat, mg
import workloads as W
from errnorms import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_faces(m1, dim, seed):
    rng = np.random.default_rng(seed)
    return tuple(np.exp(rng.uniform(-2.3, 2.3, s)) for s in W.face_shapes(m1, dim))


def solver(dim, m1, n, eps=None, precision="fp64", faces=None, inner=None, cycles=1):
    from paper_2002_01108_amd import Solver
    s = Solver(dim, m1, n, eps=eps, precision=precision)
    if faces is not None:
        s.set_coefficient(faces)
    if inner:
        s.set_inner(inner, cycles)
    return s


@pytest.mark.parametrize("dim,m1,n", [(1, 37, 16), (2, 63, 32), (2, 70, 8), (3, 13, 8),
                                      (3, 66, 4)])
def test_apply_A_variable(dim, m1, n):
    faces = rand_faces(m1, dim, 1)
    p = heat.Problem(m1, dim, n, faces=faces)
    x = np.random.default_rng(2).standard_normal((n, p.m))
    s = solver(dim, m1, n, faces=faces)
    assert rel(host(s.apply_A(dev(x))), p.L(x)) <= 1e-12


def _yt(n, m, seed):
    rng = np.random.default_rng(seed)
    yt = rng.standard_normal((n // 2 + 1, m, 2))
    yt[0, :, 1] = 0.0
    yt[-1, :, 1] = 0.0
    return yt


@pytest.mark.parametrize("m1,n,cycles,prec,tol", [(31, 16, 1, "fp64", 1e-11),
                                                  (63, 32, 1, "fp64", 1e-11),
                                                  (63, 8, 3, "fp64", 1e-11),
                                                  (37, 4, 1, "fp64", 1e-11),
                                                  (63, 32, 1, "fp32", 1e-5)])
def test_step2_multigrid(m1, n, cycles, prec, tol):
    faces = W.grf_faces(m1, 2, seed=3)
    p = heat.Problem(m1, 2, n, faces=faces)
    s = solver(2, m1, n, eps=p.eps, precision=prec, faces=faces, inner="mg", cycles=cycles)
    yt = _yt(n, p.m, 4)
    got = host(s.step2(dev(yt)))
    lam = heat.lambdas(n, p.eps)[: n // 2 + 1]
    want = mg.step2_mg(faces[0], faces[1], p.tau, lam, yt[..., 0] + 1j * yt[..., 1], cycles)
    assert rel(got[..., 0] + 1j * got[..., 1], want) <= tol


def test_step2_multigrid_constant_coefficient_is_close_to_exact():
    """With a = 1, many V-cycles approach the exact sine-transform solve."""
    m1, n = 63, 16
    p = heat.Problem(m1, 2, n)
    s = solver(2, m1, n, eps=p.eps, inner="mg", cycles=12)
    yt = _yt(n, p.m, 5)
    got = host(s.step2(dev(yt)))
    lam = heat.lambdas(n, p.eps)[: n // 2 + 1]
    want = heat.step2(p.K, p.tau, lam, yt[..., 0] + 1j * yt[..., 1])
    assert rel(got[..., 0] + 1j * got[..., 1], want) <= 1e-9


def test_step2_mean_coefficient():
    m1, n = 63, 16
    faces = W.grf_faces(m1, 2, seed=6)
    p = heat.Problem(m1, 2, n, faces=faces)
    s = solver(2, m1, n, eps=p.eps, faces=faces, inner="dst_mean")
    yt = _yt(n, p.m, 7)
    got = host(s.step2(dev(yt)))
    abar = mg.mean_coefficient(*faces)
    lam = heat.lambdas(n, p.eps)[: n // 2 + 1]
    want = heat.step2(abar * heat.stiffness(m1, 2), p.tau, lam, yt[..., 0] + 1j * yt[..., 1])
    assert rel(got[..., 0] + 1j * got[..., 1], want) <= 1e-11


@pytest.mark.parametrize("inner,prec", [("mg", "fp64"), ("mg", "fp32"), ("dst_mean", "fp64")])
def test_solve_variable_coefficient(inner, prec):
    m1, n = 63, 64
    faces = W.grf_faces(m1, 2, seed=8)
    p = heat.Problem(m1, 2, n, faces=faces)
    f = np.random.default_rng(9).standard_normal((n, p.m))
    rhs = p.rhs(f, W.initial_value(m1, 2, "modes", 10))
    exact = p.exact(rhs)
    s = solver(2, m1, n, eps=p.eps, precision=prec, faces=faces, inner=inner)
    u, info = s.solve(dev(rhs), tol=1e-10, maxit=200)
    assert info["status"] == 0 and info["final_res"] <= 1e-10
    assert rel(host(u), exact) <= 1e-8
    if inner == "mg":
        assert info["iters"] <= 12


def test_exact_inner_rejected_for_variable_coefficient():
    from paper_2002_01108_amd import AaoError
    m1, n = 15, 8
    faces = rand_faces(m1, 2, 11)
    s = solver(2, m1, n, faces=faces)
    with pytest.raises(AaoError) as e:
        s.apply_Pinv(dev(np.ones((n, m1 * m1))))
    assert e.value.status == -5
    bad = (faces[0] * -1.0, faces[1])
    with pytest.raises(AaoError) as e:
        s.set_coefficient(bad)
    assert e.value.status == -1
    with pytest.raises(AaoError):
        solver(1, 15, 8).set_inner("mg")


def test_coefficient_reset():
    m1, n = 31, 8
    p = heat.Problem(m1, 2, n)
    s = solver(2, m1, n, faces=rand_faces(m1, 2, 12))
    s.set_coefficient(None)
    x = np.random.default_rng(13).standard_normal((n, p.m))
    assert rel(host(s.apply_A(dev(x))), p.L(x)) <= 1e-12
    assert rel(host(s.apply_Pinv(dev(x))), p.Pinv(x)) <= 1e-11
