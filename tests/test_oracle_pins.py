"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each checks a closed form, a
textbook or library routine, a theorem of the paper, a brute-force computation
on a tiny input, or a value printed in the paper.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import heat
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- spatial operator

@pytest.mark.parametrize("m1", [1, 5, 16])
def test_laplacian_eigenpairs_1d(m1):
    """K_h sin(p pi x) = 4 h^-2 sin^2(p pi h/2) sin(p pi x) (textbook FD eigenpairs)."""
    K = heat.laplacian_1d(m1).toarray()
    x = W.node_coords(m1)
    h = 1.0 / (m1 + 1)
    for p in range(1, m1 + 1):
        v = np.sin(p * math.pi * x)
        mu = 4.0 / h ** 2 * math.sin(p * math.pi * h / 2) ** 2
        assert np.allclose(K @ v, mu * v, rtol=1e-12, atol=1e-9 * mu)


@pytest.mark.parametrize("dim", [2, 3])
def test_laplacian_eigenpairs_nd(dim):
    """Separable eigenvectors of the 5/7-point operator with eigenvalue the sum of 1D ones."""
    m1 = 6
    K = heat.stiffness(m1, dim)
    x = W.node_coords(m1)
    h = 1.0 / (m1 + 1)
    ps = [(1, 2, 3), (4, 1, 6), (6, 6, 6)]
    for p in ps:
        p = p[:dim]
        v = np.sin(p[0] * math.pi * x)
        mu = 4.0 / h ** 2 * math.sin(p[0] * math.pi * h / 2) ** 2
        for d in range(1, dim):
            v = np.multiply.outer(np.sin(p[d] * math.pi * x), v)
            mu += 4.0 / h ** 2 * math.sin(p[d] * math.pi * h / 2) ** 2
        v = v.reshape(-1)
        assert np.allclose(K @ v, mu * v, rtol=1e-12, atol=1e-9 * mu)


def test_face_operator_constant_is_laplacian():
    for dim in (1, 2, 3):
        m1 = 5
        Ka = heat.stiffness_faces(m1, dim, W.constant_faces(m1, dim))
        assert abs(Ka - heat.stiffness(m1, dim)).max() < 1e-9


def test_face_operator_exact_on_quadratics():
    """Flux-form FD is exact for -div(a grad u) with a linear in x, y and u quadratic:
    a = 1 + x + 2y, u = x^2 + y^2 gives -4 - 6x - 12y at every node away from the wall."""
    m1 = 9
    h = 1.0 / (m1 + 1)
    x = W.node_coords(m1)
    xf = (np.arange(m1 + 1) + 0.5) * h
    ax = 1 + xf[None, :] + 2 * x[:, None]           # [y node][x face]
    ay = 1 + x[None, :] + 2 * xf[:, None]           # [y face][x node]
    K = heat.stiffness_faces(m1, 2, (ax, ay))
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = (X ** 2 + Y ** 2).reshape(-1)
    got = (K @ u).reshape(m1, m1)
    want = -4 - 6 * X - 12 * Y
    assert np.allclose(got[1:-1, 1:-1], want[1:-1, 1:-1], rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------- all-at-once system

def test_sequential_be_closed_form():
    """f = 0, u0 = sin(pi x): u^k = (1 + tau mu_1)^{-k} sin(pi x) (Section 2, eq. (stepsystem))."""
    m1, n = 63, 64
    p = heat.Problem(m1, 1, n)
    u0 = W.initial_value(m1, 1, "sine")
    rhs = p.rhs(np.zeros((n, m1)), u0)
    u = p.exact(rhs)
    mu1 = heat.fd_eigenvalues_1d(m1)[0]
    want = np.array([(1 + p.tau * mu1) ** -(k + 1) * u0 for k in range(n)])
    assert np.abs(u - want).max() <= 1e-14


def test_apply_L_on_separable_vector():
    """For v^k = c_k phi with K phi = mu phi: (Lv)^k = ((1 + tau mu) c_k - c_{k-1}) phi."""
    m1, n = 10, 7
    p = heat.Problem(m1, 2, n)
    x = W.node_coords(m1)
    h = 1.0 / (m1 + 1)
    phi = np.multiply.outer(np.sin(2 * math.pi * x), np.sin(3 * math.pi * x)).reshape(-1)
    mu = 4 / h ** 2 * (math.sin(2 * math.pi * h / 2) ** 2 + math.sin(3 * math.pi * h / 2) ** 2)
    c = np.arange(1, n + 1) ** 2 * 0.1
    v = np.outer(c, phi)
    out = p.L(v)
    cprev = np.concatenate([[0.0], c[:-1]])
    want = np.outer((1 + p.tau * mu) * c - cprev, phi)
    assert np.abs(out - want).max() <= 1e-11 * np.abs(want).max()


def test_apply_L_P_match_block_matrices():
    """L and P_eps written block by block as displayed in Sections 2 and 3."""
    m1, n, eps = 4, 5, 0.3
    p = heat.Problem(m1, 1, n, eps=eps)
    m = m1
    A0 = np.eye(m) + p.tau * p.K.toarray()
    Lb = np.zeros((n * m, n * m))
    for k in range(n):
        Lb[k * m:(k + 1) * m, k * m:(k + 1) * m] = A0
        if k:
            Lb[k * m:(k + 1) * m, (k - 1) * m:k * m] = -np.eye(m)
    Pb = Lb.copy()
    Pb[:m, (n - 1) * m:] = -eps * np.eye(m)
    v = np.random.default_rng(0).standard_normal((n, m))
    assert np.allclose(p.L(v).reshape(-1), Lb @ v.reshape(-1), atol=1e-12)
    assert np.allclose(p.P(v).reshape(-1), Pb @ v.reshape(-1), atol=1e-12)
    assert np.allclose(heat.dense_L(p.K, n, p.tau), Lb)
    assert np.allclose(heat.dense_P(p.K, n, p.tau, eps), Pb)


def test_r_eps_matches_section3_for_backward_euler():
    """R_eps for p = 1: ones on the diagonal, -1 below it and -eps at the top right."""
    n, eps = 6, 0.2
    R = heat.r_eps_dense(n, eps)
    want = np.eye(n) - np.eye(n, k=-1)
    want[0, -1] = -eps
    assert np.array_equal(R, want)


# ---------------------------------------------------------------- diagonalisation

def test_fourier_matrix_against_numpy_fft():
    """F_n^* v is the DFT up to scaling (Section 4, after eq. (fouriermatdef))."""
    n = 16
    v = np.random.default_rng(1).standard_normal(n) + 1j * np.random.default_rng(2).standard_normal(n)
    F = heat.fourier_matrix(n)
    assert np.allclose(F.conj().T @ v, np.fft.fft(v) / math.sqrt(n), atol=1e-14)
    assert np.allclose(F @ F.conj().T, np.eye(n), atol=1e-14)


@pytest.mark.parametrize("n,eps", [(16, 0.25), (8, 1.0), (7, 0.05), (12, 1e-3)])
def test_r_eps_diagonalisation(n, eps):
    """R_eps = D^{-1} F^* Lambda F D (Section 4, eq. (repsdiagform); Bini et al.)."""
    F = heat.fourier_matrix(n)
    d = heat.eps_scaling(n, eps)
    lam = heat.lambdas(n, eps)
    R = np.diag(1 / d) @ F.conj().T @ np.diag(lam) @ F @ np.diag(d)
    assert np.abs(R - heat.r_eps_dense(n, eps)).max() <= 1e-13 / eps
    assert np.abs(R.imag).max() <= 1e-13 / eps


def test_r_eps_diagonalisation_bdf2():
    """The same identity for the two-step scheme r = (3/2, -2, 1/2) (Section 5, Example 1)."""
    n, eps = 10, 0.1
    r = (1.5, -2.0, 0.5)
    F = heat.fourier_matrix(n)
    d = heat.eps_scaling(n, eps)
    lam = heat.lambdas(n, eps, r)
    R = np.diag(1 / d) @ F.conj().T @ np.diag(lam) @ F @ np.diag(d)
    assert np.abs(R - heat.r_eps_dense(n, eps, r)).max() <= 1e-12


def test_step1_against_numpy_ifft():
    """ytilde = sqrt(N) * ifft(D_eps y) along time (numpy's ifft has the + sign and 1/N)."""
    n, m, eps = 16, 5, 0.125
    y = np.random.default_rng(3).standard_normal((n, m))
    d = heat.eps_scaling(n, eps)
    want = math.sqrt(n) * np.fft.ifft(d[:, None] * y, axis=0)
    assert np.allclose(heat.step1(y, eps, full=True), want, atol=1e-13)
    assert np.allclose(heat.step1(y, eps), want[: n // 2 + 1], atol=1e-13)


def test_step3_against_numpy_irfft():
    """z = D^{-1} F^* ztilde for a Hermitian ztilde equals sqrt(N) irfft(conj(half)) / D."""
    n, m, eps = 16, 5, 0.3
    rng = np.random.default_rng(4)
    half = rng.standard_normal((n // 2 + 1, m)) + 1j * rng.standard_normal((n // 2 + 1, m))
    d = heat.eps_scaling(n, eps)
    want = math.sqrt(n) * np.fft.irfft(np.conj(half), n=n, axis=0) / d[:, None]
    assert np.allclose(heat.step3(half, eps, n), want, atol=1e-13)


def test_conjugate_symmetry_of_blocks():
    """ytilde^{N-k} = conj(ytilde^k) and the all-block inverse is real and equals the
    half-block inverse (closing argument of Section 4)."""
    n, m1, eps = 12, 5, 0.2
    p = heat.Problem(m1, 2, n, eps=eps)
    y = np.random.default_rng(5).standard_normal((n, p.m))
    yt = heat.step1(y, eps, full=True)
    for k in range(1, n):
        assert np.allclose(yt[n - k], np.conj(yt[k]), atol=1e-14)
    zall = heat.apply_Pinv_all_blocks(p.K, p.tau, eps, y)
    assert np.abs(zall.imag).max() <= 1e-13 * np.abs(zall).max()
    assert np.allclose(zall.real, p.Pinv(y), atol=1e-13 * np.abs(zall).max())


# ---------------------------------------------------------------- the inverse

@pytest.mark.parametrize("dim,m1,n,eps", [(1, 63, 64, 0.125), (2, 20, 32, 0.05),
                                          (3, 6, 16, 0.25), (2, 9, 8, 1.0)])
def test_pinv_residual(dim, m1, n, eps):
    """P_eps (P_eps^{-1} y) = y with P_eps applied from its definition (Section 3);
    eps = 1 is the block-circulant preconditioner."""
    p = heat.Problem(m1, dim, n, eps=eps)
    y = np.random.default_rng(6).standard_normal((n, p.m))
    z = p.Pinv(y)
    assert np.linalg.norm(p.P(z) - y) <= 1e-12 * np.linalg.norm(y)


def test_pinv_against_smw_and_dense():
    """Three-step inverse == Sherman-Morrison-Woodbury form of Theorem 3.1 == dense solve."""
    m1, n, eps = 4, 6, 0.3
    p = heat.Problem(m1, 2, n, eps=eps)
    y = np.random.default_rng(7).standard_normal((n, p.m))
    z = p.Pinv(y).reshape(-1)
    smw = heat.smw_Pinv(p.K, n, p.tau, eps) @ y.reshape(-1)
    dense = np.linalg.solve(heat.dense_P(p.K, n, p.tau, eps), y.reshape(-1))
    assert np.allclose(z, smw, atol=1e-12)
    assert np.allclose(z, dense, atol=1e-12)


def _precond_matrix(p):
    nm = p.n * p.m
    L = heat.dense_L(p.K, p.n, p.tau)
    cols = [p.Pinv(L[:, j].reshape(p.n, p.m)).reshape(-1) for j in range(nm)]
    return np.array(cols).T


def test_spectrum_closed_form():
    """sigma(P^{-1} L) = {1}^{(N-1)J} U {lambda^N/(lambda^N - eps)}, lambda = 1 + tau mu_j,
    rank(P^{-1}L - I) = J (Section 3, Theorem 3.2 and eq. (lastdiagblockexpans))."""
    m1, n, T, eps = 7, 8, 0.01, 0.5
    p = heat.Problem(m1, 1, n, T=T, eps=eps)
    G = _precond_matrix(p)
    ev = np.linalg.eigvals(G)
    lam = 1 + p.tau * heat.fd_eigenvalues_1d(m1)
    nonunit = lam ** n / (lam ** n - eps)
    want = np.sort_complex(np.concatenate([np.ones((n - 1) * m1), nonunit]).astype(complex))
    got = np.sort_complex(ev)
    assert np.abs(got - want).max() <= 1e-8
    assert np.linalg.matrix_rank(G - np.eye(n * m1), tol=1e-9) == m1


def test_cluster_radius_and_norm_bound():
    """max |lambda - 1| <= eps/(1-eta) (Theorem 3.2) and
    ||P^{-1}L - I||_2 <= eps sqrt(N)/(1 - eps) with c0 = 1 (Lemma 3.5); the radius
    shrinks with eps."""
    m1, n = 6, 10
    radii = []
    for eps in (0.5, 0.1, 0.01):
        p = heat.Problem(m1, 1, n, eps=eps)
        G = _precond_matrix(p)
        ev = np.linalg.eigvals(G)
        r = np.abs(ev - 1).max()
        assert r <= eps / (1 - eps) + 1e-12
        assert np.linalg.norm(G - np.eye(n * m1), 2) <= eps * math.sqrt(n) / (1 - eps) + 1e-12
        radii.append(r)
    assert radii[0] > radii[1] > radii[2]


# ---------------------------------------------------------------- GMRES

def test_gmres_iterate_is_krylov_minimiser():
    """After k steps, right-preconditioned GMRES minimises ||b - L x|| over
    x in span{P^{-1} r0, P^{-1}(L P^{-1}) r0, ...}: brute force least squares."""
    m1, n, eps = 5, 6, 0.9
    p = heat.Problem(m1, 1, n, eps=eps)
    b = np.random.default_rng(8).standard_normal(n * m1)
    A = lambda v: p.L(v).reshape(-1)                          # noqa: E731
    M = lambda v: p.Pinv(v).reshape(-1)                       # noqa: E731
    for k in (1, 2, 3):
        x, it, _ = heat.fgmres(A, M, b, tol=0.0, maxit=k, restart=50)
        assert it == k
        basis = [b]
        for _ in range(k - 1):
            basis.append(A(M(basis[-1])))
        Q, _ = np.linalg.qr(np.array(basis).T)
        Y = np.array([M(q) for q in Q.T]).T          # candidate search directions
        AY = np.array([A(y) for y in Y.T]).T
        c, *_ = np.linalg.lstsq(AY, b, rcond=None)
        xb = Y @ c
        assert np.linalg.norm(x - xb) <= 1e-10 * np.linalg.norm(xb)


def test_gmres_terminates_within_J_plus_1():
    """rank(P^{-1}L - I) = J, so unrestarted GMRES is exact within J+1 steps (Section 3)."""
    m1, n, eps = 5, 16, 0.9
    p = heat.Problem(m1, 1, n, T=0.05, eps=eps)
    b = np.random.default_rng(9).standard_normal((n, m1))
    x, it, hist = p.gmres(b, tol=1e-13, restart=100)
    assert it <= m1 + 1
    assert np.linalg.norm(p.L(x) - b) <= 1e-11 * np.linalg.norm(b)


def test_gmres_rate_bound():
    """Theorem 3.7: with eps <= b_tau = delta sqrt(tau)/(delta sqrt(tau) + sqrt(T)) the
    left-preconditioned residuals obey ||r_k|| <= (2 sqrt(delta)/(1+delta))^k ||r_0||."""
    m1, n, T, delta = 15, 16, 1.0, 0.5
    tau = T / n
    b_tau = delta * math.sqrt(tau) / (delta * math.sqrt(tau) + math.sqrt(T))
    p = heat.Problem(m1, 1, n, T=T, eps=b_tau)
    f = np.random.default_rng(10).standard_normal((n, m1))
    _, it, hist = p.gmres_left(f, tol=1e-13, maxit=30)
    rate = 2 * math.sqrt(delta) / (1 + delta)
    for k, h in enumerate(hist, start=1):
        assert h <= rate ** k * (1 + 1e-9)


def test_gmres_matches_sequential_be():
    """At a tight tolerance the GMRES-BEC solution is the exact L^{-1} f (C1 workload)."""
    w = W.WORKLOADS["heat1d_63x64"]
    p = heat.Problem(w.m1, w.dim, w.n, eps=w.epsilon)
    f, u0, _ = W.make(w)
    rhs = p.rhs(f, u0)
    u = p.exact(rhs)
    assert np.linalg.norm(p.L(u) - rhs) <= 1e-13 * np.linalg.norm(rhs)
    x, it, hist = p.gmres(rhs, tol=1e-12)
    assert it <= 4
    assert np.linalg.norm(x - u) <= 1e-10 * np.linalg.norm(u)
    x8, it8, hist8 = p.gmres(rhs, tol=1e-8)
    assert it8 == 2 and hist8[-1] <= 1e-8


def _table1_row(n, J1, bec):
    m1 = J1 - 1
    tau = 1.0 / n
    eps = min(0.5, 0.5 * tau) if bec else 1.0
    p = heat.Problem(m1, 2, n, eps=eps)
    p.K = 1e-5 * heat.stiffness(m1, 2)
    x = W.node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = (X * (X - 1) * Y * (Y - 1)).reshape(-1)
    rhs = p.rhs(np.zeros((n, p.m)), u0)
    u, it, _ = p.gmres_left(rhs, tol=1e-7, maxit=200, restart=50)
    res = np.linalg.norm(rhs - p.L(u)) / np.linalg.norm(rhs)
    return it, res


def _golden_rows(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return rows


@pytest.mark.slow
@pytest.mark.parametrize("row", range(2))
def test_table1_iterations(row):
    """Iteration counts of GMRES-BEC and GMRES-BC printed in Table 1 (Section 5)."""
    n, J1, it_bec, res_bec, it_bc, res_bc = _golden_rows("table1_bdf1.txt")[row]
    it, res = _table1_row(int(n), int(J1), True)
    assert it == int(it_bec)
    assert res_bec / 4 <= res <= res_bec * 4
    it, res = _table1_row(int(n), int(J1), False)
    assert it == int(it_bc)
    assert res_bc / 4 <= res <= res_bc * 4


# ---------------------------------------------------------------- variable coefficient

def test_manufactured_solution_converges():
    """Example 2 (Section 5) with a = sin(pi x y): the error of the all-at-once solution
    against u = exp(-t) x(1-x) y(1-y) falls by ~4 when tau and h^2 are quartered."""
    errs = []
    for n, m1 in ((8, 7), (32, 15)):
        tau = 1.0 / n
        faces = W.manufactured_faces(m1)
        p = heat.Problem(m1, 2, n, faces=faces)
        f = np.array([W.manufactured_f(m1, (k + 1) * tau) for k in range(n)])
        u0 = W.manufactured_u(m1, 0.0)
        u = p.exact(p.rhs(f, u0))
        ustar = np.array([W.manufactured_u(m1, (k + 1) * tau) for k in range(n)])
        errs.append(np.abs(u - ustar).max())
    ratio = errs[0] / errs[1]
    assert 3.0 <= ratio <= 5.0, (errs, ratio)


def test_manufactured_source_is_consistent():
    """Finite-difference check of the printed source: f = u_t - div(sin(pi x y) grad u)."""
    m1 = 31
    t = 0.3
    x = W.node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    d = 1e-4
    u = lambda X, Y, t: math.exp(-t) * X * (1 - X) * Y * (1 - Y)     # noqa: E731
    a = lambda X, Y: np.sin(math.pi * X * Y)                          # noqa: E731
    ut = (u(X, Y, t + d) - u(X, Y, t - d)) / (2 * d)
    fx = (a(X + d / 2, Y) * (u(X + d, Y, t) - u(X, Y, t)) - a(X - d / 2, Y) * (u(X, Y, t) - u(X - d, Y, t))) / d ** 2
    fy = (a(X, Y + d / 2) * (u(X, Y + d, t) - u(X, Y, t)) - a(X, Y - d / 2) * (u(X, Y, t) - u(X, Y - d, t))) / d ** 2
    want = ut - fx - fy
    assert np.allclose(W.manufactured_f(m1, t).reshape(m1, m1), want, atol=1e-5)


def test_rectangular_stiffness_eigenvalues_and_square_case():
    """K_h on a rectangular grid: its eigenvalues are the sums of the 1D FD
    eigenvalues 4/h_d^2 sin^2(j pi h_d / 2) with each axis' own spacing (closed
    form), and a square grid reproduces the square-grid operator."""
    ms = (7, 4, 3)
    K = heat.stiffness_rect(ms).toarray()
    got = np.sort(np.linalg.eigvalsh(K))
    one = [4.0 * (m + 1) ** 2 * np.sin(np.arange(1, m + 1) * np.pi / (2 * (m + 1))) ** 2
           for m in ms]
    want = np.sort((one[0][None, None, :] + one[1][None, :, None]
                    + one[2][:, None, None]).ravel())
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9)
    # x fastest: the first coupling is along x with spacing 1/(m1+1)
    assert K[0, 1] == pytest.approx(-(ms[0] + 1) ** 2)
    assert K[0, ms[0]] == pytest.approx(-(ms[1] + 1) ** 2)
    assert K[0, ms[0] * ms[1]] == pytest.approx(-(ms[2] + 1) ** 2)
    sq = heat.stiffness(5, 2) - heat.stiffness_rect((5, 5))
    assert abs(sq).max() < 1e-9
