"""Pins of the oracle's network arithmetic (the model itself is a design choice,
not the paper's; its convolution, gradients and optimiser are pinned here)."""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    got = cnn.conv3x3(x, w)
    for b in range(2):
        for o in range(4):
            want = sum(signal.correlate2d(x[b, c], w[o, c], mode="same", boundary="fill")
                       for c in range(3))
            assert np.allclose(got[b, o], want, atol=1e-12)


def test_conv_input_grad_is_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 6, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    dz = rng.standard_normal((2, 4, 6, 5))
    lhs = np.sum(cnn.conv3x3(x, w) * dz)
    rhs = np.sum(x * cnn.conv3x3_input_grad(dz, w))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _setup(seed=2, B=3, H=6, W=7):
    rng = np.random.default_rng(seed)
    params = cnn.init_params(seed)
    params += 0.05 * rng.standard_normal(params.size)     # non-zero FiLM maps and bias
    x = rng.standard_normal((B, 3, H, W))
    lam = 1 - 0.9 * np.exp(2j * np.pi * rng.uniform(size=B))
    t = rng.standard_normal((B, 2, H, W))
    return params, x, cnn.features(lam), t


def _loss(params, x, phi, t):
    y, _ = cnn.forward(params, x, phi)
    return cnn.loss(y, t)[0]


def test_backward_matches_central_differences():
    params, x, phi, t = _setup()
    y, cache = cnn.forward(params, x, phi)
    _, dy = cnn.loss(y, t)
    g, dx = cnn.backward(params, cache, dy)
    rng = np.random.default_rng(3)
    h = 1e-6
    for i in rng.choice(params.size, 40, replace=False):
        e = np.zeros_like(params)
        e[i] = h
        fd = (_loss(params + e, x, phi, t) - _loss(params - e, x, phi, t)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    for idx in [(0, 0, 2, 3), (2, 2, 0, 0), (1, 1, 5, 6)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (_loss(params, x + e, phi, t) - _loss(params, x - e, phi, t)) / (2 * h)
        assert dx[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def _resid_setup(seed=4, B=2, H=5, W=6):
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((B, 2, H, W))
    rho = rng.standard_normal((B, 2, H, W))
    lam = 1 - 0.9 * np.exp(2j * np.pi * rng.uniform(size=B))
    wx = np.exp(rng.uniform(-1, 1, (H, W + 1)))
    wy = np.exp(rng.uniform(-1, 1, (H + 1, W)))
    return y, rho, lam, wx, wy


def test_sweep_matches_mg_smoother():
    """The batched sweep is the multigrid module's red-black Gauss-Seidel sweep."""
    from oracle import mg
    y, rho, lam, wx, wy = _resid_setup(H=5, W=5)      # the multigrid module is square-only
    got = cnn.sweep(y, rho, lam, wx, wy)
    for b in range(y.shape[0]):
        e = y[b, 0] + 1j * y[b, 1]
        want = mg.rbgs(e, rho[b, 0] + 1j * rho[b, 1], lam[b], wx, wy)
        assert np.allclose(got[b, 0] + 1j * got[b, 1], want, atol=1e-13)


def test_residual_loss_gradient_matches_central_differences():
    y, rho, lam, wx, wy = _resid_setup()
    val, dy = cnn.residual_loss(y, rho, lam, wx, wy)
    h = 1e-6
    rng = np.random.default_rng(5)
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in y.shape)
        e = np.zeros_like(y)
        e[idx] = h
        fd = (cnn.residual_loss(y + e, rho, lam, wx, wy)[0]
              - cnn.residual_loss(y - e, rho, lam, wx, wy)[0]) / (2 * h)
        assert dy[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_residual_loss_of_exact_correction_is_zero():
    """If y / (lambda + d) solves B e = rho, the sweep keeps it and the loss vanishes."""
    from oracle import mg
    _, rho, lam, wx, wy = _resid_setup(B=1, H=4, W=4)
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    H = W = 4
    rows = []
    for j in range(H * W):
        e = np.zeros(H * W, complex)
        e[j] = 1.0
        rows.append(mg.apply_B(e.reshape(H, W), lam[0], wx, wy).reshape(-1))
    Bm = np.array(rows).T
    sol = np.linalg.solve(Bm, (rho[0, 0] + 1j * rho[0, 1]).reshape(-1)).reshape(H, W)
    # the loss divides the network output by lambda + d: feed the scaled solution
    from oracle.cnn import _diag
    sol = sol * (lam[0] + _diag(wx, wy))
    y = np.stack([sol.real, sol.imag])[None]
    assert cnn.residual_loss(y, rho, lam, wx, wy)[0] < 1e-24


def test_adam_first_step_is_signed_lr():
    """From zero moments the first bias-corrected Adam step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = cnn.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8))


def test_layout_size():
    _, total = cnn.layout()
    C = cnn.C_HIDDEN
    assert total == C * 27 + 4 * C * 4 + C * C * 9 + 2 * C * 9 + 2


def test_node_log_coefficient_written_out():
    """Each node's value is the log of the mean of its four faces (west x-face i,
    east x-face i + 1 of row j; south y-face j, north y-face j + 1 of column i),
    minus the mean over all nodes; written out node by node."""
    m = 5
    rng = np.random.default_rng(30)
    ax = np.exp(rng.uniform(-2, 2, (m, m + 1)))
    ay = np.exp(rng.uniform(-2, 2, (m + 1, m)))
    want = np.empty((m, m))
    for j in range(m):
        for i in range(m):
            want[j, i] = np.log((ax[j, i] + ax[j, i + 1] + ay[j, i] + ay[j + 1, i]) / 4.0)
    want -= want.mean()
    assert np.allclose(cnn.node_log_coefficient(ax, ay), want, atol=1e-14)


def test_node_log_coefficient_invariances():
    """A constant coefficient gives zeros; scaling every face by c changes nothing
    (the channel is centred); one node with all four faces v stands out by log v
    against a unit background before centring."""
    m = 7
    ones_x, ones_y = np.ones((m, m + 1)), np.ones((m + 1, m))
    assert np.allclose(cnn.node_log_coefficient(3.7 * ones_x, 3.7 * ones_y), 0.0, atol=1e-15)
    rng = np.random.default_rng(31)
    ax = np.exp(rng.uniform(-1, 1, (m, m + 1)))
    ay = np.exp(rng.uniform(-1, 1, (m + 1, m)))
    assert np.allclose(cnn.node_log_coefficient(50 * ax, 50 * ay),
                       cnn.node_log_coefficient(ax, ay), atol=1e-13)
    bx, by = ones_x.copy(), ones_y.copy()
    v, j, i = 9.0, 3, 2
    bx[j, i] = bx[j, i + 1] = by[j, i] = by[j + 1, i] = v
    out = cnn.node_log_coefficient(bx, by)
    # neighbours share one face of v: log((3 + v) / 4); the rest log 1 = 0
    assert out[j, i] - out[0, 0] == pytest.approx(np.log(v), rel=1e-14)
    assert out[j, i + 1] - out[0, 0] == pytest.approx(np.log((3 + v) / 4), rel=1e-14)
