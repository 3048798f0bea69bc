"""Argument checks at the C ABI and in its binding, on the GPU.

* aao_solve rejects a right-hand side that shares memory with the solution
  (the Krylov basis starts from rhs, which the solve keeps reading while it
  writes u): AAO_EINVAL, nothing written.
* A rejected aao_set_coefficient leaves the previous operator in place (here
  the convection-diffusion stand-in of Section 5, Example 3).
* The binding refuses arrays of the wrong size before any device call.
* Restarted solves (restart shorter than the iteration count) are
  deterministic from call to call and reach the oracle's sequential solution:
  the restart's unit coefficient has a slot of its own, so it cannot overwrite
  the solution-update coefficients while their copy is still queued.
"""
import numpy as np
import pytest

from errnorms import rel
from oracle import cd, heat
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solver(dim, m1, n, eps, **kw):
    from paper_2002_01108_amd import Solver
    return Solver(dim, m1, n, T=1.0, eps=eps, **kw)


def test_solve_rejects_rhs_aliasing_u(lib):
    import ctypes
    from paper_2002_01108_amd import binding
    s = solver(2, 15, 8, 0.2)
    rhs = dev(np.random.default_rng(1).standard_normal((8, 225)))
    keep = host(rhs).copy()
    it = ctypes.c_int(-7)
    fres = ctypes.c_double(-1.0)
    for u_ptr in (rhs.data_ptr(), rhs.data_ptr() + 8 * 17):   # same array, partial overlap
        st = lib.aao_solve(s._h, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(u_ptr), 0,
                           1e-8, 10, 5, ctypes.byref(it), None, 0, None, ctypes.byref(fres))
        assert st == binding.EINVAL
        assert b"overlap" in lib.aao_last_error(s._h)
    assert np.array_equal(host(rhs), keep)
    # adjacent but disjoint ranges are fine
    both = torch.zeros((2, 8, 225), dtype=torch.float64, device="cuda")
    both[0] = rhs
    u, info = s.solve(both[0], tol=1e-10, u=both[1])
    p = heat.Problem(15, 2, 8, eps=0.2)
    assert info["status"] == 0 and rel(host(u), p.exact(keep)) <= 1e-10


def test_binding_checks_sizes_and_dtypes():
    s = solver(2, 15, 8, 0.2)
    good = torch.zeros((8, 225), dtype=torch.float64, device="cuda")
    short = torch.zeros((8, 224), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        s.apply_A(short)
    with pytest.raises(ValueError):
        s.apply_A(good, out=short)
    with pytest.raises(ValueError):
        s.apply_Pinv(short)
    with pytest.raises(ValueError):
        s.solve(good, u=short)
    with pytest.raises(ValueError):
        s.build_rhs(good, torch.zeros(224, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        s.step3(torch.zeros((5, 225, 1), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        s.apply_A(good.float())
    with pytest.raises(TypeError):
        s.apply_A(good.cpu())
    with pytest.raises(ValueError):
        s.set_coefficient((np.ones((15, 16)), np.ones((15, 15))))   # ay: 225 values, not 240


def test_rejected_coefficient_keeps_convection():
    from paper_2002_01108_amd import AaoError
    m1, n, eps = 15, 8, 0.2
    p = cd.Problem(m1, n, eps=eps)
    s = solver(2, m1, n, eps)
    w1, w2 = W.cd_wind(m1)
    s.set_convection(W.CD_NU / 4.0, (w1 / 2.0, w2 / 2.0))
    s.set_inner("mg", 1)
    v = np.random.default_rng(3).standard_normal((n, p.m))
    before = host(s.apply_A(dev(v)))
    assert rel(before, p.L(v)) <= 1e-12
    ax, ay = W.constant_faces(m1, 2)
    ax = ax.copy()
    ax[3, 4] = 0.0                         # not positive: rejected
    with pytest.raises(AaoError) as e:
        s.set_coefficient((ax, ay))
    assert e.value.status == -1
    after = host(s.apply_A(dev(v)))
    assert np.array_equal(after, before)
    with pytest.raises(AaoError):          # the convection context still refuses DST_MEAN
        s.set_inner("dst_mean")
    z = host(s.apply_Pinv(dev(v)))         # and its multigrid hierarchy still works
    assert np.all(np.isfinite(z))


@pytest.mark.parametrize("side", ["right", "left"])
def test_restarted_solve_is_deterministic(side):
    """Restart shorter than the iteration count, three calls each: bit-identical
    iterates, histories and iteration counts.
    (a) 2D 100^2 x 32, eps = 0.1, restart 1: three steps, two restarts; the
        solution matches sequential backward Euler.
    (b) block circulant (eps = 1) with slow diffusion (T = 1e-5, Section 5's
        Example 1 setting) on 63^2 x 32, restart 4, 24 steps (not converged):
        with right preconditioning the explicit final residual equals the
        Givens estimate, which a wrong update coefficient would break."""
    cases = [((100, 32, 1.0, 0.1), 1, 60, 1e-12), ((63, 32, 1e-5, 1.0), 4, 24, 0.0)]
    for (m1, n, T, eps), restart, maxit, tol in cases:
        p = heat.Problem(m1, 2, n, T=T, eps=eps)
        f = np.random.default_rng(21).standard_normal((n, p.m))
        rhs = p.rhs(f, W.initial_value(m1, 2, "modes", 22))
        from paper_2002_01108_amd import Solver
        s = Solver(2, m1, n, T=T, eps=eps)
        s.set_side(side)
        rd = dev(rhs)
        runs = [s.solve(rd, tol=tol, maxit=maxit, restart=restart) for _ in range(3)]
        us = [host(u) for u, _ in runs]
        its = [info["iters"] for _, info in runs]
        assert its[0] > restart                    # restarts happened
        assert its[0] == its[1] == its[2]
        assert np.array_equal(us[0], us[1]) and np.array_equal(us[0], us[2])
        assert runs[1][1]["hist"] == runs[0][1]["hist"] == runs[2][1]["hist"]
        if tol > 0:
            assert runs[0][1]["status"] == 0
            exact = p.exact(rhs)
            assert rel(us[0], exact) <= (1e-10 if side == "right" else 1e-9)
        else:
            assert runs[0][1]["status"] == 1 and its[0] == maxit
            res = np.linalg.norm(p.L(us[0]) - rhs) / np.linalg.norm(rhs)
            assert abs(runs[0][1]["final_res"] / res - 1.0) < 1e-6
            if side == "right":
                assert abs(runs[0][1]["final_res"] / runs[0][1]["hist"][-1] - 1.0) < 1e-3
