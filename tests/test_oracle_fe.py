"""Pins of the Q1 finite-element oracle (oracle/fe.py):

* M1, K1 and the 2D Q1 matrices against an independent element-by-element
  assembly with Gauss quadrature of the shape functions;
* the DST-I diagonalises M1 and K1 with the closed-form eigenvalues
  h/3 (2 + cos theta_p) and 2/h (1 - cos theta_p), theta_p = p pi h;
* P_eps^{-1} against a dense solve of R_eps (x) M + tau I (x) K, the stepping
  solver against a dense solve of L u = rhs (backward Euler and BDF2);
* Section 5, Example 1, Table 1, rows with J+1 = 2^6 for N = 2^6..2^9: the
  iteration counts of GMRES-BEC and GMRES-BC exactly, and RES to within 2 %
  of the printed three-digit values (tests/golden/table1_full.txt).
"""
import math
import os

import numpy as np
import pytest

from oracle import bdf, fe, heat
import workloads as W

HERE = os.path.dirname(__file__)
GAUSS = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))   # 2-point rule on [0, 1]


def _assemble_q1(m1, dim):
    """Element loop: (mass, stiffness) of P1 (dim 1) / Q1 (dim 2) elements with
    interior nodes only, shape functions evaluated at Gauss points."""
    h = 1.0 / (m1 + 1)
    nodes = m1 ** dim
    M = np.zeros((nodes, nodes))
    K = np.zeros((nodes, nodes))
    phi = [lambda s: 1.0 - s, lambda s: s]
    dphi = [lambda s: -1.0 / h, lambda s: 1.0 / h]
    for e in np.ndindex(*([m1 + 1] * dim)):          # element corners e..e+1 per axis
        locs = list(np.ndindex(*([2] * dim)))
        for a in locs:
            ia = [e[d] + a[d] - 1 for d in range(dim)]      # interior index (-1 = boundary)
            if any(i < 0 or i >= m1 for i in ia):
                continue
            for b in locs:
                ib = [e[d] + b[d] - 1 for d in range(dim)]
                if any(i < 0 or i >= m1 for i in ib):
                    continue
                mm = kk = 0.0
                for q in np.ndindex(*([2] * dim)):
                    s = [GAUSS[q[d]] for d in range(dim)]
                    w = (0.5 * h) ** dim
                    va = np.prod([phi[a[d]](s[d]) for d in range(dim)])
                    vb = np.prod([phi[b[d]](s[d]) for d in range(dim)])
                    mm += w * va * vb
                    for d in range(dim):
                        ga = dphi[a[d]](s[d]) * np.prod([phi[a[c]](s[c]) for c in range(dim) if c != d])
                        gb = dphi[b[d]](s[d]) * np.prod([phi[b[c]](s[c]) for c in range(dim) if c != d])
                        kk += w * ga * gb
                # x fastest: flat index = sum ia[d] * m1^d
                fa = sum(ia[d] * m1 ** d for d in range(dim))
                fb = sum(ib[d] * m1 ** d for d in range(dim))
                M[fa, fb] += mm
                K[fa, fb] += kk
    return M, K


def test_1d_matrices_match_element_assembly():
    M, K = _assemble_q1(6, 1)
    assert np.allclose(fe.mass_1d(6).toarray(), M, atol=1e-15)
    assert np.allclose(fe.stiff_1d(6).toarray(), K, atol=1e-12)


def test_2d_q1_matrices_match_element_assembly():
    M, K = _assemble_q1(4, 2)
    Mq, Kq = fe.q1_matrices(4)
    assert np.allclose(Mq.toarray(), M, atol=1e-15)
    assert np.allclose(Kq.toarray(), K, atol=1e-12)


def test_dst_diagonalises_mass_and_stiffness():
    m1 = 9
    h = 1.0 / (m1 + 1)
    p = np.arange(1, m1 + 1)
    S = math.sqrt(2 * h) * np.sin(np.outer(p, p) * math.pi * h)
    th = p * math.pi * h
    assert np.allclose(S @ fe.mass_1d(m1).toarray() @ S, np.diag(h / 3 * (2 + np.cos(th))),
                       atol=1e-14)
    assert np.allclose(S @ fe.stiff_1d(m1).toarray() @ S, np.diag(2 / h * (1 - np.cos(th))),
                       atol=1e-11)


@pytest.mark.parametrize("r", [bdf.BDF1, bdf.BDF2], ids=["bdf1", "bdf2"])
@pytest.mark.parametrize("eps", [0.1, 1.0])
def test_pinv_and_stepping_match_dense(r, eps):
    m1, n = 3, 6
    M, K = fe.q1_matrices(m1, a=0.7)
    tau = 1.0 / n
    rng = np.random.default_rng(51)
    y = rng.standard_normal((n, m1 * m1))
    z = fe.apply_Pinv(M, K, tau, r, eps, y)
    P = fe.dense_P(M, K, n, tau, r, eps)
    assert np.allclose(z.reshape(-1), np.linalg.solve(P, y.reshape(-1)), atol=1e-11)
    L = fe.dense_L(M, K, n, tau, r)
    v = rng.standard_normal((n, m1 * m1))
    assert np.allclose(fe.apply_L(M, K, tau, r, v).reshape(-1), L @ v.reshape(-1), atol=1e-13)
    u = fe.sequential(M, K, tau, r, y)
    assert np.allclose(u.reshape(-1), np.linalg.solve(L, y.reshape(-1)), atol=1e-11)


def table1_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_full.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows.append((int(t[0]), int(t[1]), int(t[2]), float(t[3]), int(t[4]),
                             float(t[5])))
    return rows


def table1_problem(n, J1, bec, oracle_problem=True):
    m1 = J1 - 1
    x = W.node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = (X * (X - 1) * Y * (Y - 1)).reshape(-1)
    p = fe.Problem(m1, n, r=bdf.BDF1, eps=None if bec else 1.0, a=1e-5)
    return p, p.rhs(np.zeros((n, p.m)), u0)


@pytest.mark.slow
@pytest.mark.parametrize("row", [r for r in table1_rows() if r[1] == 64],
                         ids=lambda r: f"N{r[0]}")
def test_table1_fe_rows(row):
    n, J1, it_bec, res_bec, it_bc, res_bc = row
    for bec, want_it, want_res in ((True, it_bec, res_bec), (False, it_bc, res_bc)):
        p, rhs = table1_problem(n, J1, bec)
        u, it, _ = p.gmres_left(rhs, tol=1e-7)
        res = np.linalg.norm(rhs - p.L(u)) / np.linalg.norm(rhs)
        assert it == want_it
        assert abs(res - want_res) <= 0.02 * want_res, (res, want_res)
