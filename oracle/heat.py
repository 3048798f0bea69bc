"""Oracle: the all-at-once heat system, the BEC preconditioner and GMRES (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper: N time steps (here `n`), tau = T/N, spatial
operator K (finite differences, so the mass matrix M is the identity, as the
Remark after Assumptions 1-3 of Section 2 allows), A0 = I + tau K,
all-at-once matrix L (Section 2, eq. (allatoncesystem)), preconditioner
P_eps (Section 3), its Fourier block diagonalisation (Section 4,
eqs. (repsdiagform), (becblockdiag)) and the three-step inverse
(Section 4, eqs. (ytild), (blockdiaginv), (zcompt)).

Space-time vectors are arrays of shape [n][m]: row k holds u^{k+1} on the
interior nodes, x fastest.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# ---------------------------------------------------------------------------
# spatial operator
# ---------------------------------------------------------------------------


def laplacian_1d(m1: int) -> sp.csr_matrix:
    """Three-point finite-difference -d^2/dx^2 on m1 interior nodes of (0,1),
    homogeneous Dirichlet: (2u_i - u_{i-1} - u_{i+1}) / h^2, h = 1/(m1+1).
    This is the constant-coefficient K of Section 2 (a = 1) in one dimension."""
    h = 1.0 / (m1 + 1)
    main = np.full(m1, 2.0)
    off = np.full(m1 - 1, -1.0)
    return (sp.diags([off, main, off], [-1, 0, 1]) / h ** 2).tocsr()


def stiffness(m1: int, dim: int) -> sp.csr_matrix:
    """K_h = discrete -Laplacian on the m1^dim grid, x fastest (Kronecker sum of
    the 1D operator; the 3/5/7-point stencil)."""
    K1 = laplacian_1d(m1)
    I1 = sp.identity(m1, format="csr")
    if dim == 1:
        return K1
    if dim == 2:
        return (sp.kron(I1, K1) + sp.kron(K1, I1)).tocsr()
    if dim == 3:
        return (sp.kron(I1, sp.kron(I1, K1)) + sp.kron(I1, sp.kron(K1, I1))
                + sp.kron(K1, sp.kron(I1, I1))).tocsr()
    raise ValueError(dim)


def stiffness_rect(ms) -> sp.csr_matrix:
    """K_h on a rectangular grid of (0,1)^d with ms = (m1[, m2[, m3]]) interior
    nodes per axis (spacing 1/(m_d+1) along axis d), x fastest: the Kronecker
    sum of the 1D operators (the 3/5/7-point stencil with per-axis spacing)."""
    ms = tuple(int(v) for v in ms)
    Ks = [laplacian_1d(v) for v in ms]
    Is = [sp.identity(v, format="csr") for v in ms]
    out = None
    for d in range(len(ms)):
        # factors ordered slowest (last axis) to fastest (x)
        term = None
        for e in range(len(ms) - 1, -1, -1):
            f = Ks[e] if e == d else Is[e]
            term = f if term is None else sp.kron(term, f)
        out = term if out is None else out + term
    return out.tocsr()


def stiffness_faces(m1: int, dim: int, faces) -> sp.csr_matrix:
    """Flux-form finite-difference discretisation K_a of -div(a grad u)
    (Section 2, the K of eq. (stepsystem) for a variable a(x)):

        (K_a u)_i = h^-2 * sum over the faces f of node i of a_f (u_i - u_nbr(f)),

    with u_nbr = 0 across the boundary.  `faces` holds the coefficient at face
    midpoints, shapes as in the `workloads` module (ax has m1+1 entries along x).
    """
    h2 = (1.0 / (m1 + 1)) ** 2
    shape = (m1,) * dim                    # [z][y][x]
    idx = np.arange(m1 ** dim).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(shape)
    for d in range(dim):
        axis = dim - 1 - d                 # array axis of spatial direction d
        a = np.asarray(faces[d], dtype=np.float64)
        # face j along `axis` lies between node j-1 and node j (j = 0..m1)
        lo = np.take(a, np.arange(m1), axis=axis)        # face below each node
        hi = np.take(a, np.arange(1, m1 + 1), axis=axis)  # face above each node
        diag += lo + hi
        # coupling node p -> node p+1 through the face between them (hi of p)
        src = np.take(idx, np.arange(m1 - 1), axis=axis)
        dst = np.take(idx, np.arange(1, m1), axis=axis)
        w = np.take(hi, np.arange(m1 - 1), axis=axis)
        rows += [src.ravel(), dst.ravel()]
        cols += [dst.ravel(), src.ravel()]
        vals += [-w.ravel(), -w.ravel()]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m1 ** dim, m1 ** dim))
    return (K / h2).tocsr()


def fd_eigenvalues_1d(m1: int) -> np.ndarray:
    """Eigenvalues of the 1D operator: 4 h^-2 sin^2(p pi h / 2), p = 1..m1
    (textbook closed form; eigenvectors sin(p pi x_i))."""
    h = 1.0 / (m1 + 1)
    p = np.arange(1, m1 + 1)
    return 4.0 / h ** 2 * np.sin(p * math.pi * h / 2.0) ** 2


# ---------------------------------------------------------------------------
# all-at-once system (Section 2)
# ---------------------------------------------------------------------------


def build_rhs(f: np.ndarray, u0: np.ndarray, tau: float) -> np.ndarray:
    """f_aao = (tau f^1 + M u^0; tau f^2; ...; tau f^N) with M = I
    (Section 2, eq. (allatoncesystem))."""
    rhs = tau * np.asarray(f, dtype=np.float64).copy()
    rhs[0] += u0
    return rhs


def apply_L(K: sp.spmatrix, tau: float, v: np.ndarray) -> np.ndarray:
    """L v for L = blockbidiag(-M, A0), A0 = M + tau K, M = I
    (Section 2, eq. (allatoncesystem)):  (Lv)^k = A0 v^k - v^{k-1}, v^0 = 0."""
    v = np.asarray(v, dtype=np.float64)
    out = v + tau * (K @ v.T).T
    out[1:] -= v[:-1]
    return out


def apply_P(K: sp.spmatrix, tau: float, eps: float, v: np.ndarray) -> np.ndarray:
    """P_eps v, P_eps = L with -eps M added in the top-right block (Section 3):
    (P v)^1 = A0 v^1 - eps v^N, (P v)^k = A0 v^k - v^{k-1} for k >= 2."""
    out = apply_L(K, tau, v)
    out[0] -= eps * v[-1]
    return out


def sequential_be(K: sp.spmatrix, tau: float, rhs: np.ndarray) -> np.ndarray:
    """Exact solution of L u = rhs by backward-Euler time stepping
    (Section 2, eq. (stepsystem)): A0 u^k = rhs^k + u^{k-1}, u^0 folded into rhs^1."""
    m = K.shape[0]
    A0 = (sp.identity(m) + tau * K).tocsc()
    lu = spla.splu(A0)
    u = np.empty_like(rhs, dtype=np.float64)
    prev = np.zeros(m)
    for k in range(rhs.shape[0]):
        prev = lu.solve(rhs[k] + prev)
        u[k] = prev
    return u


def fd_eigenvalues(ms) -> np.ndarray:
    """Eigenvalues of K_h on the grid ms = (m1[, m2[, m3]]) (spacing 1/(m_d+1) per
    axis), shape [m3][m2][m1] (x fastest): the sum over the axes of the 1D closed
    form 4 h_d^-2 sin^2(p_d pi h_d / 2), the eigenvector of index (p_1, p_2, p_3)
    being the product of sin(p_d pi x_d) (textbook; a Kronecker sum of 1D
    operators has the sums of their eigenvalues)."""
    ms = [int(v) for v in ms]
    mu = np.zeros(tuple(reversed(ms)))
    for d, md in enumerate(ms):
        shape = [1] * len(ms)
        shape[len(ms) - 1 - d] = md
        mu = mu + fd_eigenvalues_1d(md).reshape(shape)
    return mu


def sine_transform(v: np.ndarray, workers: int | None = None) -> np.ndarray:
    """Orthonormal DST-I along every axis of v: S_{ij} = sqrt(2/(m+1)) sin(pi i j/(m+1)),
    i, j = 1..m, per axis.  S is symmetric and S^2 = I (scipy.fft's type-1 DST with
    orthonormal scaling; a library primitive)."""
    import scipy.fft
    return scipy.fft.dstn(v, type=1, norm="ortho", workers=workers)


def sequential_be_sine(ms, tau: float, rhs: np.ndarray, workers: int | None = None) -> np.ndarray:
    """Exact solution of L u = rhs by backward-Euler time stepping (Section 2,
    eq. (stepsystem)), A0 u^k = rhs^k + u^{k-1}, with each step's A0 = I + tau K_h
    (constant coefficient, finite differences) solved in the sine basis that
    diagonalises K_h: A0^{-1} b = S diag(1 / (1 + tau mu)) S b.  Same result as
    `sequential_be` up to rounding, at a cost that 3D grids of 127^3 points allow
    (a sparse factorisation of the 3D A0 does not)."""
    ms = [int(v) for v in ms]
    shape = tuple(reversed(ms))
    d = 1.0 + tau * fd_eigenvalues(ms)
    rhs = np.asarray(rhs, dtype=np.float64)
    u = np.empty(rhs.shape, dtype=np.float64)
    prev = np.zeros(shape)
    for k in range(rhs.shape[0]):
        b = rhs[k].reshape(shape) + prev
        prev = sine_transform(sine_transform(b, workers) / d, workers)
        u[k] = prev.reshape(-1)
    return u


# ---------------------------------------------------------------------------
# epsilon-circulant diagonalisation (Section 4)
# ---------------------------------------------------------------------------


def fourier_matrix(n: int) -> np.ndarray:
    """F_n = n^{-1/2} [theta^{(i-1)(j-1)}], theta = exp(+2 pi i / n)
    (Section 4, eq. (fouriermatdef))."""
    j = np.arange(n)
    return np.exp(2j * math.pi * np.outer(j, j) / n) / math.sqrt(n)


def eps_scaling(n: int, eps: float) -> np.ndarray:
    """Diagonal of D_eps = diag(eps^{0/N}, ..., eps^{(N-1)/N}) (eq. (repsdiagform))."""
    return eps ** (np.arange(n) / n)


def lambdas(n: int, eps: float, r=(1.0, -1.0)) -> np.ndarray:
    """lambda_k = sum_j r_j eps^{j/N} theta^{kj}, k = 0..N-1 (eq. (repsdiagform));
    backward Euler has r = (1, -1), i.e. lambda_k = 1 - eps^{1/N} theta^k."""
    k = np.arange(n)
    lam = np.zeros(n, dtype=np.complex128)
    for j, rj in enumerate(r):
        lam += rj * eps ** (j / n) * np.exp(2j * math.pi * k * j / n)
    return lam


def r_eps_dense(n: int, eps: float, r=(1.0, -1.0)) -> np.ndarray:
    """R_eps written out (Section 4, eq. (pstepbecpreconditioner)): banded lower
    Toeplitz with r_0..r_p, plus eps r_j wrapped into the top-right corner."""
    R = np.zeros((n, n))
    for j, rj in enumerate(r):
        for i in range(n):
            if i - j >= 0:
                R[i, i - j] += rj
            else:
                R[i, n + i - j] += eps * rj
    return R


def step1(y: np.ndarray, eps: float, full: bool = False) -> np.ndarray:
    """Step 1 of the three-step inverse (eq. (ytild)): ytilde = (F_N D_eps (x) I) y,
    i.e. ytilde^{k+1} = N^{-1/2} sum_j theta^{kj} eps^{j/N} y^{j+1}.
    Returns k = 0..N/2 (the blocks that must be solved, see the conjugate-symmetry
    argument closing Section 4) unless `full`."""
    n = y.shape[0]
    W = fourier_matrix(n) * eps_scaling(n, eps)[None, :]
    out = W @ np.asarray(y, dtype=np.complex128)
    return out if full else out[: n // 2 + 1]


def block_factors(K: sp.spmatrix, tau: float, lam: np.ndarray):
    """Sparse complex LU factors of B_k = lambda_k M + tau K (eq. (becblockdiag))."""
    m = K.shape[0]
    I = sp.identity(m, dtype=np.complex128, format="csc")
    Kc = K.astype(np.complex128).tocsc()
    return [spla.splu((lk * I + tau * Kc).tocsc()) for lk in lam]


def step2(K: sp.spmatrix, tau: float, lam: np.ndarray, yt: np.ndarray,
          factors=None) -> np.ndarray:
    """Step 2 (eq. (blockdiaginv)): solve B_k ztilde^{k+1} = ytilde^{k+1} with
    B_k = lambda_k M + tau K (eq. (becblockdiag)), one sparse complex LU per block.
    `factors` may carry the LU factors of the same B_k from an earlier call."""
    if factors is None:
        factors = block_factors(K, tau, lam)
    out = np.empty_like(yt, dtype=np.complex128)
    for k in range(yt.shape[0]):
        out[k] = factors[k].solve(np.ascontiguousarray(yt[k]))
    return out


def step2_sine(ms, tau: float, lam: np.ndarray, yt: np.ndarray,
               workers: int | None = None) -> np.ndarray:
    """Step 2 (eq. (blockdiaginv)) for the constant-coefficient finite-difference
    K_h, in the sine basis that diagonalises it (Section 4: B_k = lambda_k I +
    tau K_h is diagonalised by the DST-I along every axis):
    ztilde_k = S diag(1 / (lambda_k + tau mu)) S ytilde_k, S applied to the real
    and imaginary parts.  Same result as `step2` up to rounding, at a cost that
    3D grids of 127^3 points allow."""
    ms = [int(v) for v in ms]
    shape = tuple(reversed(ms))
    mu = fd_eigenvalues(ms)
    out = np.empty(np.shape(yt), dtype=np.complex128)
    for k in range(yt.shape[0]):
        b = np.asarray(yt[k]).reshape(shape)
        sb = sine_transform(b.real, workers) + 1j * sine_transform(b.imag, workers)
        sb = sb / (lam[k] + tau * mu)
        z = sine_transform(sb.real, workers) + 1j * sine_transform(sb.imag, workers)
        out[k] = z.reshape(-1)
    return out


def hermitian_complete(zt_half: np.ndarray, n: int) -> np.ndarray:
    """Rebuild all N blocks from k = 0..N/2 using ztilde^{N-k} = conj(ztilde^k)
    (closing argument of Section 4).  The imaginary parts of blocks k = 0 and
    k = N/2 are dropped, which makes the completed spectrum exactly Hermitian."""
    if n % 2:
        raise ValueError("even n only")
    full = np.empty((n,) + zt_half.shape[1:], dtype=np.complex128)
    full[: n // 2 + 1] = zt_half
    full[0] = full[0].real
    full[n // 2] = full[n // 2].real
    for k in range(1, n // 2):
        full[n - k] = np.conj(zt_half[k])
    return full


def step3(zt_half: np.ndarray, eps: float, n: int) -> np.ndarray:
    """Step 3 (eq. (zcompt)): z = (D_eps^{-1} F_N^* (x) I) ztilde, real part of the
    result of a Hermitian spectrum (Section 4, conjugate-symmetry argument)."""
    full = hermitian_complete(zt_half, n)
    F = fourier_matrix(n)
    z = (F.conj().T @ full) / eps_scaling(n, eps)[:, None]
    return z.real


def apply_Pinv(K: sp.spmatrix, tau: float, eps: float, y: np.ndarray,
               factors=None) -> np.ndarray:
    """z = P_eps^{-1} y by the paper's three steps (Section 4), solving only the
    blocks k = 0..N/2."""
    n = y.shape[0]
    lam = lambdas(n, eps)
    yt = step1(y, eps)
    zt = step2(K, tau, lam[: n // 2 + 1], yt, factors)
    return step3(zt, eps, n)


def apply_Pinv_all_blocks(K, tau, eps, y):
    """Same as apply_Pinv but solving all N blocks (no conjugate symmetry used)."""
    n = y.shape[0]
    lam = lambdas(n, eps)
    yt = step1(y, eps, full=True)
    zt = step2(K, tau, lam, yt)
    F = fourier_matrix(n)
    z = (F.conj().T @ zt) / eps_scaling(n, eps)[:, None]
    return z


# ---------------------------------------------------------------------------
# dense small-size routes (Section 3)
# ---------------------------------------------------------------------------


def dense_L(K: np.ndarray, n: int, tau: float) -> np.ndarray:
    """L = R (x) M + tau I_N (x) K with R = bidiag(1, -1), M = I (eq. (pstepscheme))."""
    K = np.asarray(K.todense() if sp.issparse(K) else K)
    m = K.shape[0]
    R = r_eps_dense(n, 0.0)
    return np.kron(R, np.eye(m)) + tau * np.kron(np.eye(n), K)


def dense_P(K, n: int, tau: float, eps: float) -> np.ndarray:
    """P_eps = R_eps (x) M + tau I (x) K (eq. (pstepbecpreconditioner))."""
    K = np.asarray(K.todense() if sp.issparse(K) else K)
    m = K.shape[0]
    return np.kron(r_eps_dense(n, eps), np.eye(m)) + tau * np.kron(np.eye(n), K)


def smw_Pinv(K, n: int, tau: float, eps: float) -> np.ndarray:
    """P_eps^{-1} = L^{-1} + L^{-1} E_1 Z_eps^{-1} E_N^T L^{-1} with
    Z_eps = eps^{-1} [I - eps (A0^{-1} M)^N] M^{-1} (Section 3, Theorem 3.1)."""
    K = np.asarray(K.todense() if sp.issparse(K) else K)
    m = K.shape[0]
    A0 = np.eye(m) + tau * K
    A0inv = np.linalg.inv(A0)
    Linv = np.linalg.inv(dense_L(K, n, tau))
    Z = (np.eye(m) - eps * np.linalg.matrix_power(A0inv, n)) / eps
    E1 = np.zeros((n * m, m))
    E1[:m] = np.eye(m)
    EN = np.zeros((n * m, m))
    EN[-m:] = np.eye(m)
    return Linv + Linv @ E1 @ np.linalg.solve(Z, EN.T @ Linv)


# ---------------------------------------------------------------------------
# GMRES (Section 5: restarted GMRES, zero initial guess)
# ---------------------------------------------------------------------------


def fgmres(A, Minv, b: np.ndarray, tol: float = 1e-8, maxit: int = 100,
           restart: int = 50, x0: np.ndarray | None = None):
    """Textbook right-preconditioned flexible GMRES with modified Gram-Schmidt and
    Givens rotations (Saad, Iterative Methods, Alg. 9.6), restarted.

    A, Minv: callables on flat vectors.  The stopping test is on the true
    (unpreconditioned) relative residual ||b - A x|| / ||b||, which right
    preconditioning exposes as |g_{j+1}| / ||b||.  Returns
    (x, iterations, history) where history[j] is that estimate after step j.
    For a fixed Minv this is ordinary right-preconditioned GMRES.
    """
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).reshape(-1).copy()
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return np.zeros_like(b), 0, hist
    total = 0
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or total >= maxit:
            return x, total, hist
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        done = False
        j = 0
        for j in range(restart):
            z = Minv(V[j])
            Z.append(z)
            w = A(z)
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            hist.append(abs(g[j + 1]) / bnorm)
            breakdown = np.linalg.norm(w) == 0.0
            if hist[-1] <= tol or total >= maxit or breakdown:
                done = True
                break
            V.append(w / np.linalg.norm(w))
        k = j + 1
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        if done:
            return x, total, hist


# ---------------------------------------------------------------------------
# convenience: a whole problem
# ---------------------------------------------------------------------------


class Problem:
    """One all-at-once heat problem: K, tau, eps and the operators on it."""

    def __init__(self, m1: int, dim: int, n: int, T: float = 1.0, eps: float | None = None,
                 faces=None):
        self.m1, self.dim, self.n, self.T = m1, dim, n, T
        self.tau = T / n
        self.eps = min(0.5, math.sqrt(self.tau)) if eps is None else eps
        self.faces = faces
        self.K = stiffness(m1, dim) if faces is None else stiffness_faces(m1, dim, faces)
        self.m = self.K.shape[0]

    def L(self, v):
        return apply_L(self.K, self.tau, v.reshape(self.n, self.m))

    def P(self, v):
        return apply_P(self.K, self.tau, self.eps, v.reshape(self.n, self.m))

    def factors(self):
        key = (self.eps, self.tau, id(self.K))
        if getattr(self, "_fkey", None) != key:
            lam = lambdas(self.n, self.eps)[: self.n // 2 + 1]
            self._factors = block_factors(self.K, self.tau, lam)
            self._fkey = key
        return self._factors

    def Pinv(self, v):
        return apply_Pinv(self.K, self.tau, self.eps, v.reshape(self.n, self.m),
                          self.factors())

    def rhs(self, f, u0):
        return build_rhs(f.reshape(self.n, self.m), u0, self.tau)

    def exact(self, rhs, workers: int | None = None):
        """Sequential backward Euler: a sparse LU of A0 (1D/2D, any coefficient),
        or the sine-basis solve of each step (3D with a = 1)."""
        if self.dim == 3 and self.faces is None:
            return sequential_be_sine((self.m1,) * 3, self.tau, rhs.reshape(self.n, self.m),
                                      workers)
        return sequential_be(self.K, self.tau, rhs.reshape(self.n, self.m))

    def gmres(self, rhs, tol=1e-8, maxit=100, restart=50, Minv=None):
        """Right-preconditioned (F)GMRES on L u = rhs with P_eps^{-1} (default)."""
        A = lambda v: self.L(v).reshape(-1)                                 # noqa: E731
        M = Minv or (lambda v: self.Pinv(v).reshape(-1))                    # noqa: E731
        x, it, hist = fgmres(A, M, rhs.reshape(-1), tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist

    def gmres_left(self, rhs, tol=1e-7, maxit=200, restart=50):
        """GMRES on the left-preconditioned system P^{-1} L u = P^{-1} f
        (Section 3, eq. (preconditionedsystem)), stopping on the preconditioned
        residual ||r_k|| <= tol ||r_0|| from a zero guess as in Section 5."""
        A = lambda v: self.Pinv(self.L(v)).reshape(-1)                      # noqa: E731
        b = self.Pinv(rhs).reshape(-1)
        x, it, hist = fgmres(A, lambda v: v, b, tol, maxit, restart)
        return x.reshape(self.n, self.m), it, hist
