"""Q1 finite elements (aao_set_discretisation(ctx, AAO_DISC_Q1)) on the GPU
against the FE oracle (oracle/fe.py), through the C ABI, and Section 5's
Table 1 reproduced row by row.

Tolerances as for finite differences (L v and the right-hand side 1e-12,
P^{-1} 1e-11, FP64 solves 1e-10, FP32 P^{-1} backward error 3e-5): M and
tau K are 9-point stencils with O(1) relative weights, and P^{-1} divides by
m_i (lambda_k + tau k_i / m_i) with m_i >= h^2/9, which changes none of the
growth factors those tolerances carry.

Table 1: BEC iteration counts exact and RES within 2 % of the printed
three-digit values (the oracle meets both on the rows it can afford); BC within
one iteration and 10 % (its 1e-7 threshold is crossed within a few per cent at
the printed step, see the Table 1 test of the left/BC tests).  The BC entry of
row N = 2^7, J+1 = 2^9 repeats the CPU time (11.92 s) and RES (2.81e-5) of row
N = 2^8, J+1 = 2^7, and that time is below the smaller J+1 = 2^8 row's: a copy
error in the table, so only its iteration count is compared.  The BEC RES of
row N = 2^8, J+1 = 2^8 (1.60e-11) is reproduced by neither side: the oracle
takes the printed two iterations and ends at RES 1.391e-11, the GPU at
1.390e-11, while the rows beside it (J+1 = 2^7 and 2^9) match to three digits;
that entry is checked to lie between its printed neighbours instead."""
import os

import numpy as np
import pytest

from oracle import bdf, fe
import workloads as W
from errnorms import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(__file__)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solver(m1, n, eps, T=1.0, order=1, precision="fp64", side="right"):
    from paper_2002_01108_amd import Solver
    s = Solver(2, m1, n, T=T, eps=eps, precision=precision)
    s.set_scheme(order)
    s.set_discretisation("q1")
    s.set_side(side)
    return s


# (m1, n, eps): fold paths P = 64 (one-level fold), 128 and 256 (fused), even m1
GRIDS = [(63, 16, 0.1), (37, 8, 0.3), (127, 16, 0.05), (64, 8, 0.2), (255, 4, 0.1)]


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("m1,n,eps", GRIDS)
def test_apply_A_rhs_and_Pinv(m1, n, eps, order):
    r = bdf.BDF1 if order == 1 else bdf.BDF2
    p = fe.Problem(m1, n, r=r, eps=eps)
    rng = np.random.default_rng(61)
    v = rng.standard_normal((n, p.m))
    f = rng.standard_normal((n, p.m))
    u0 = rng.standard_normal(p.m)
    s = solver(m1, n, eps, order=order)
    assert rel(host(s.apply_A(dev(v))), p.L(v)) <= 1e-12
    assert rel(host(s.build_rhs(dev(f), dev(u0))), p.rhs(f, u0)) <= 1e-12
    assert rel(host(s.apply_Pinv(dev(v))), p.Pinv(v)) <= 1e-11


def test_Pinv_two_level_fold_divide():
    """P = 512 (m1 = 511): the divide runs in the two-level-fold y product."""
    m1, n, eps = 511, 2, 0.2
    p = fe.Problem(m1, n, eps=eps)
    v = np.random.default_rng(62).standard_normal((n, p.m))
    s = solver(m1, n, eps)
    assert rel(host(s.apply_Pinv(dev(v))), p.Pinv(v)) <= 1e-11


def test_fp32_Pinv_backward_error():
    m1, n, eps = 127, 16, 0.05
    p = fe.Problem(m1, n, eps=eps)
    v = np.random.default_rng(63).standard_normal((n, p.m))
    s = solver(m1, n, eps, precision="fp32")
    z = host(s.apply_Pinv(dev(v)))
    s64 = solver(m1, n, eps)
    Pz = host(s64.apply_A(dev(z)))
    Pz[0] -= eps * (p.M @ z[-1])          # P = L + the eps-wrapped corner (BDF1)
    # 2-norm: 3e-5 as for every FP32 P^{-1}.  Max-abs: the FP32 rounding of the
    # spectrum reaches time level j amplified by eps^{-j/n} (Step 3), the last
    # level by eps^{-(n-1)/n} = 16.6 here, against the root-mean-square growth of
    # 7.4 over all levels that the 2-norm sees: 1e-4.
    assert np.linalg.norm(Pz - v) / np.linalg.norm(v) <= 3e-5
    assert np.abs(Pz - v).max() / np.abs(v).max() <= 1e-4


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("side", ["right", "left"])
def test_solve_matches_sequential(order, side):
    m1, n, eps = 37, 32, 0.1
    r = bdf.BDF1 if order == 1 else bdf.BDF2
    p = fe.Problem(m1, n, r=r, eps=eps)
    rng = np.random.default_rng(64)
    rhs = p.rhs(rng.standard_normal((n, p.m)), rng.standard_normal(p.m))
    exact = p.exact(rhs)
    s = solver(m1, n, eps, order=order, side=side)
    u, info = s.solve(dev(rhs), tol=1e-12, maxit=200)
    assert info["status"] == 0
    assert rel(host(u), exact) <= 1e-10


def _table1_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_full.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows.append((int(t[0]), int(t[1]), int(t[2]), float(t[3]), int(t[4]),
                             float(t[5])))
    return rows


BC_RES_MISPRINTED = {(128, 512)}
BEC_RES_UNREPRODUCED = {(256, 256): (1.05e-11, 1.55e-11)}


@pytest.mark.parametrize("row", _table1_rows(), ids=lambda r: f"N{r[0]}_J{r[1]}")
def test_table1_row(row):
    n, J1, it_bec, res_bec, it_bc, res_bc = row
    m1, a = J1 - 1, 1e-5
    x = W.node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = dev((X * (X - 1) * Y * (Y - 1)).reshape(-1))
    f = torch.zeros((n, m1 * m1), dtype=torch.float64, device="cuda")
    for bec, want_it, want_res in ((True, it_bec, res_bec), (False, it_bc, res_bc)):
        eps = min(0.5, 0.5 / n) if bec else 1.0
        s = solver(m1, n, eps, T=a, side="left")
        rhs = s.build_rhs(f, u0)
        u, info = s.solve(rhs, tol=1e-7, maxit=200, restart=50)
        print(f"N={n} J+1={J1} {'BEC' if bec else 'BC'}: iterations {info['iters']} "
              f"(printed {want_it}), RES {info['final_res']:.3e} (printed {want_res:.2e})",
              flush=True)
        assert info["status"] == 0
        if bec:
            assert info["iters"] == want_it
            if (n, J1) in BEC_RES_UNREPRODUCED:
                lo, hi = BEC_RES_UNREPRODUCED[(n, J1)]
                assert lo <= info["final_res"] <= hi
            else:
                assert abs(info["final_res"] - want_res) <= 0.02 * want_res
        else:
            assert abs(info["iters"] - want_it) <= 1
            if (n, J1) not in BC_RES_MISPRINTED:
                assert abs(info["final_res"] - want_res) <= 0.10 * want_res
        del s, rhs, u
        torch.cuda.empty_cache()


def test_guards():
    from paper_2002_01108_amd import Solver
    s3 = Solver(3, 7, 4, eps=0.2, precision="fp64")
    assert s3.lib.aao_set_discretisation(s3._h, 1) == -1        # AAO_EINVAL: not 2D
    s = solver(15, 8, 0.2)
    assert s.lib.aao_set_precision(s._h, 2) == -5               # AAO_ESTATE: BF16x3
    assert s.lib.aao_set_inner(s._h, 2, 1) == -5                # AAO_ESTATE: multigrid
    assert s.lib.aao_set_discretisation(s._h, 5) == -1
    s.set_discretisation("fd")                                  # back to finite differences
    from oracle import heat
    p = heat.Problem(15, 2, 8, eps=0.2)
    v = np.random.default_rng(65).standard_normal((8, p.m))
    assert rel(host(s.apply_A(dev(v))), p.L(v)) <= 1e-12
    assert rel(host(s.apply_Pinv(dev(v))), p.Pinv(v)) <= 1e-11
