"""Pins of the oracle's multigrid V-cycle (variable-coefficient inner solve)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import heat, mg
import workloads as W


def _faces(m1, seed=0):
    rng = np.random.default_rng(seed)
    return (np.exp(rng.uniform(-1, 1, (m1, m1 + 1))), np.exp(rng.uniform(-1, 1, (m1 + 1, m1))))


def test_fine_operator_is_shifted_flux_form():
    """apply_B on the finest level equals lambda I + tau K_a from the independent assembly."""
    m1, tau, lam = 15, 1 / 16, 0.3 - 0.7j
    ax, ay = _faces(m1)
    lv = mg.levels(ax, ay, tau)
    rng = np.random.default_rng(1)
    e = rng.standard_normal((m1, m1)) + 1j * rng.standard_normal((m1, m1))
    K = heat.stiffness_faces(m1, 2, (ax, ay))
    want = lam * e.reshape(-1) + tau * (K @ e.reshape(-1))
    got = mg.apply_B(e, lam, lv[0][1], lv[0][2]).reshape(-1)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-12)


def test_coarse_operator_constant_coefficient():
    """With a = 1 the rediscretised coarse operator is the 5-point Laplacian with h doubled."""
    m1, tau, lam = 31, 0.01, 0.5
    ax, ay = W.constant_faces(m1, 2)
    lv = mg.levels(ax, ay, tau)
    assert [l[0] for l in lv] == [31, 15, 7, 3, 1]
    for m, wx, wy in lv:
        e = np.random.default_rng(m).standard_normal((m, m))
        want = lam * e.reshape(-1) + tau * (heat.stiffness(m, 2) @ e.reshape(-1))
        assert np.allclose(mg.apply_B(e, lam, wx, wy).reshape(-1), want, rtol=1e-12)


def test_full_weighting_symbol():
    """Full weighting maps sin(p pi x) sin(q pi y) to ((1+cos p pi h)/2)((1+cos q pi h)/2) times
    the same mode on the coarse grid (its Fourier symbol)."""
    mf = 31
    mc = 15
    h = 1 / (mf + 1)
    x = W.node_coords(mf)
    X = W.node_coords(mc)
    for p, q in ((1, 1), (3, 2), (7, 5)):
        f = np.outer(np.sin(q * math.pi * x), np.sin(p * math.pi * x))
        c = np.outer(np.sin(q * math.pi * X), np.sin(p * math.pi * X))
        sym = (1 + math.cos(p * math.pi * h)) / 2 * (1 + math.cos(q * math.pi * h)) / 2
        assert np.allclose(mg.restrict(f, mc), sym * c, atol=1e-13)


def test_bilinear_prolongation_exact_for_xy():
    """Bilinear interpolation reproduces f = x y (zero on the x = 0 and y = 0 walls)."""
    mf, mc = 31, 15
    x = W.node_coords(mf)
    X = W.node_coords(mc)
    got = mg.prolong(np.outer(X, X), mf)
    want = np.outer(x, x)
    assert np.allclose(got[:-1, :-1], want[:-1, :-1], atol=1e-14)


@pytest.mark.parametrize("lam", [0.0108, 0.5 + 0.9j, 1.9 + 0.1j])
def test_vcycles_converge_to_direct_solve(lam):
    """Repeated V-cycles (correction form) converge to the sparse LU solution of
    (lambda I + tau K_a) e = r, with a textbook contraction per cycle."""
    m1, n = 31, 32
    tau = 1.0 / n
    ax, ay = W.grf_faces(m1, 2, seed=3)
    K = heat.stiffness_faces(m1, 2, (ax, ay))
    B = (lam * sp.identity(m1 * m1) + tau * K).tocsc()
    rng = np.random.default_rng(4)
    r = rng.standard_normal(m1 * m1) + 1j * rng.standard_normal(m1 * m1)
    exact = spla.spsolve(B, r)
    errs = []
    for cycles in (1, 2, 4, 16):
        e = mg.step2_mg(ax, ay, tau, np.array([lam]), r[None, :], cycles=cycles)[0]
        errs.append(np.linalg.norm(e - exact) / np.linalg.norm(exact))
    assert errs[0] < 0.35
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[3] < 1e-10


def test_mean_coefficient():
    ax, ay = W.constant_faces(7, 2, 2.5)
    assert mg.mean_coefficient(ax, ay) == pytest.approx(2.5)


def test_grf_faces_contrast_and_shape():
    """The synthetic coefficient has the requested face shapes and max/min exactly 100."""
    ax, ay = W.grf_faces(255, 2, seed=2)
    assert ax.shape == (255, 256) and ay.shape == (256, 255)
    both = np.concatenate([ax.ravel(), ay.ravel()])
    assert both.max() / both.min() == pytest.approx(100.0, rel=1e-12)


# ---------------------------------------------------------------------------
# coarse faces: series conductance of the fine row (or column) through the
# coarse nodes.  In one dimension, eliminating the fine node that lies between
# two coarse nodes from the conservative flux matrix (h K_a, couplings a_f / h)
# leaves the conductance of the two fine faces in series between them, i.e. the
# coarse face coefficient a_c with a_c / (2h) = 1 / (h/a1 + h/a2): the harmonic
# mean.  Coarse node (J, I) sits on fine node (2J+1, 2I+1), so the x-couplings
# of coarse row J come from fine row 2J+1 and the y-couplings of coarse column I
# from fine column 2I+1.


def _schur_coarse_1d(a_faces, h):
    """Schur complement of the 1D conservative matrix h K_a (faces a_faces,
    m + 1 of them) onto the odd fine nodes (0-based 1, 3, ...)."""
    m = a_faces.size - 1
    K = (heat.stiffness_faces(m, 1, [a_faces]) * h).toarray()
    keep = np.arange(1, m, 2)
    drop = np.setdiff1d(np.arange(m), keep)
    A, B = K[np.ix_(keep, keep)], K[np.ix_(keep, drop)]
    C, D = K[np.ix_(drop, keep)], K[np.ix_(drop, drop)]
    return A - B @ np.linalg.solve(D, C)


def test_coarse_faces_are_series_conductances():
    m = 15
    mc = (m - 1) // 2
    h, H = 1.0 / (m + 1), 1.0 / (mc + 1)
    rng = np.random.default_rng(40)
    # a separable, strongly varying field: every fine row and column differs
    ax = np.exp(rng.uniform(-2, 2, (m, 1))) * np.exp(rng.uniform(-2, 2, (1, m + 1)))
    ay = np.exp(rng.uniform(-2, 2, (m + 1, 1))) * np.exp(rng.uniform(-2, 2, (1, m)))
    axc, ayc = mg.coarse_faces(ax, ay)
    assert axc.shape == (mc, mc + 1) and ayc.shape == (mc + 1, mc)
    for J in range(mc):
        want = _schur_coarse_1d(ax[2 * J + 1], h)
        got = (heat.stiffness_faces(mc, 1, [axc[J]]) * H).toarray()
        assert np.allclose(got, want, rtol=1e-12, atol=0)
    for I in range(mc):
        want = _schur_coarse_1d(ay[:, 2 * I + 1], h)
        got = (heat.stiffness_faces(mc, 1, [ayc[:, I]]) * H).toarray()
        assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_coarse_faces_layered_medium_exact_flux():
    """A medium layered in x (a depends on x only): the coarse x-faces reproduce
    the exact steady flux through each pair of fine cells (series law), not the
    arithmetic mean."""
    m = 31
    a1d = np.where(np.arange(m + 1) % 3 == 0, 100.0, 1.0)
    ax = np.tile(a1d, (m, 1))
    ay = np.ones((m + 1, m))
    axc, _ = mg.coarse_faces(ax, ay)
    I = np.arange((m - 1) // 2 + 1)
    want = 1.0 / (0.5 / a1d[2 * I] + 0.5 / a1d[2 * I + 1])
    assert np.allclose(axc, np.tile(want, ((m - 1) // 2, 1)), rtol=1e-14)
    assert not np.allclose(axc, 0.5 * (a1d[2 * I] + a1d[2 * I + 1]))


# ---------------------------------------------------------------------------
# red-black Gauss-Seidel: the same as one dense Gauss-Seidel sweep (forward
# substitution with the lower triangle) in the ordering "all red points, then
# all black points", red = (i1 + i2) even.


def _dense_gs_red_black(B, r, e, m, first=0):
    jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    red = ((ii + jj) % 2 == first).reshape(-1)
    order = np.concatenate([np.flatnonzero(red), np.flatnonzero(~red)])
    Bp = B[np.ix_(order, order)]
    lower = np.tril(Bp)
    upper = Bp - lower
    xp = np.linalg.solve(lower, r[order] - upper @ e[order])
    out = np.empty_like(xp)
    out[order] = xp
    return out


@pytest.mark.parametrize("lam", [0.0108, 0.4 - 1.3j])
def test_rbgs_is_dense_gauss_seidel_red_then_black(lam):
    m, tau = 7, 1 / 8
    ax, ay = _faces(m, seed=41)
    K = heat.stiffness_faces(m, 2, (ax, ay))
    B = (lam * np.eye(m * m) + tau * K.toarray()).astype(np.complex128)
    rng = np.random.default_rng(42)
    r = rng.standard_normal(m * m) + 1j * rng.standard_normal(m * m)
    e0 = rng.standard_normal(m * m) + 1j * rng.standard_normal(m * m)
    lv = mg.levels(ax, ay, tau)
    got = mg.rbgs(e0.reshape(m, m), r.reshape(m, m), lam, lv[0][1], lv[0][2]).reshape(-1)
    want = _dense_gs_red_black(B, r, e0, m)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    # black first, or both colours from the old iterate (Jacobi), give other results
    jac = e0 + (r - B @ e0) / np.diag(B)
    assert not np.allclose(got, jac, rtol=1e-6)
    assert not np.allclose(got, _dense_gs_red_black(B, r, e0, m, first=1), rtol=1e-6)


def test_rbgs_planes_match_dense_gauss_seidel():
    """The four-plane (nonsymmetric) form: upwinded convection-diffusion couplings."""
    from oracle import cd
    m, lam = 7, 0.7 + 0.2j
    p = cd.Problem(m, 4)
    W_, E_, S_, N_ = p.planes
    tau = p.tau
    B = lam * np.eye(m * m) + tau * p.K.toarray()
    rng = np.random.default_rng(43)
    r = rng.standard_normal(m * m) + 1j * rng.standard_normal(m * m)
    e0 = np.zeros(m * m, dtype=np.complex128)
    got = mg.rbgs(e0.reshape(m, m), r.reshape(m, m), lam, tau * W_, tau * E_, tau * S_,
                  tau * N_).reshape(-1)
    want = _dense_gs_red_black(B, r, e0, m)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
