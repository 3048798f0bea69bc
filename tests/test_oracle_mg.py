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
