"""Oracle: the learned per-frequency correction of the inner solve (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves the blocks B_k = lambda_k I + tau K_a of Step 2 approximately
with one multigrid V-cycle (Section 4; Section 5, Example 2).  The learned
inner solve keeps that V-cycle and adds a small convolutional network N that
maps the V-cycle's residual to a correction:

    e1 = V(r),  rho = r - B_k e1,  s = rms(rho),
    e  = S_r(e1 + s * N(rho / s, log a; lambda_k) / (lambda_k + d)),
where d is the diagonal of tau K_a at each node (the network's two output
channels are a complex field divided pointwise by the diagonal of B_k, so it
learns a correction relative to a Jacobi step) and S_r is one red-black
Gauss-Seidel sweep for B_k e = r started from its argument.

N (parity unpinned as a model: its architecture is chosen here, not taken from
the paper; its arithmetic is pinned below):
    x  = [Re rho/s, Im rho/s, log a - mean log a]          3 channels, H x W
    z1 = conv3x3(x, W1);  h1 = relu((1 + G1 phi) * z1 + H1 phi)     C channels
    z2 = conv3x3(h1, W2); h2 = relu((1 + G2 phi) * z2 + H2 phi)     C channels
    y  = conv3x3(h2, W3) + b3                                       2 channels
with phi = (Re lambda_k, Im lambda_k, log|lambda_k|, 1) (feature-wise linear
modulation), zero padding, cross-correlation convention.  Training loss per
block (residual_loss): ||rho_hat - B_k S(y / (lambda_k + d))||^2 / ||rho_hat||^2,
with rho_hat the normalised V-cycle residual, y the network output and S the
same sweep, averaged over the batch; Adam (Kingma & Ba) updates.  The plain
error loss ||y - t||^2 / ||t||^2 (loss) is kept for the gradient pins.

Parameter vector layout (float): W1[C][3][3][3], G1[C][4], H1[C][4],
W2[C][C][3][3], G2[C][4], H2[C][4], W3[2][C][3][3], b3[2].
"""
from __future__ import annotations

import numpy as np

C_HIDDEN = 8
N_FEAT = 4


def layout(C: int = C_HIDDEN):
    shapes = [("W1", (C, 3, 3, 3)), ("G1", (C, N_FEAT)), ("H1", (C, N_FEAT)),
              ("W2", (C, C, 3, 3)), ("G2", (C, N_FEAT)), ("H2", (C, N_FEAT)),
              ("W3", (2, C, 3, 3)), ("b3", (2,))]
    out, off = [], 0
    for name, shp in shapes:
        size = int(np.prod(shp))
        out.append((name, shp, off, size))
        off += size
    return out, off


def unpack(params: np.ndarray, C: int = C_HIDDEN) -> dict:
    lay, total = layout(C)
    assert params.size == total
    return {name: params[off:off + size].reshape(shp) for name, shp, off, size in lay}


def pack(d: dict, C: int = C_HIDDEN) -> np.ndarray:
    lay, total = layout(C)
    out = np.zeros(total)
    for name, shp, off, size in lay:
        out[off:off + size] = np.asarray(d[name]).reshape(-1)
    return out


def features(lam) -> np.ndarray:
    lam = np.asarray(lam, dtype=np.complex128)
    return np.stack([lam.real, lam.imag, np.log(np.abs(lam)), np.ones(lam.shape)], axis=-1)


def conv3x3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """out[b,o,i,j] = sum_c sum_{p,q in -1..1} w[o,c,p+1,q+1] x[b,c,i+p,j+q], zero outside."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((B, w.shape[0], H, W))
    for p in range(3):
        for q in range(3):
            patch = xp[:, :, p:p + H, q:q + W]
            out += np.einsum("oc,bchw->bohw", w[:, :, p, q], patch)
    return out


def conv3x3_input_grad(dz: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 with respect to its input."""
    B, Co, H, W = dz.shape
    dxp = np.zeros((B, w.shape[1], H + 2, W + 2))
    for p in range(3):
        for q in range(3):
            dxp[:, :, p:p + H, q:q + W] += np.einsum("oc,bohw->bchw", w[:, :, p, q], dz)
    return dxp[:, :, 1:-1, 1:-1]


def conv3x3_weight_grad(dz: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gradient of sum(dz * conv3x3(x, w)) with respect to w."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    g = np.zeros((dz.shape[1], Ci, 3, 3))
    for p in range(3):
        for q in range(3):
            g[:, :, p, q] = np.einsum("bohw,bchw->oc", dz, xp[:, :, p:p + H, q:q + W])
    return g


def forward(params: np.ndarray, x: np.ndarray, phi: np.ndarray, C: int = C_HIDDEN):
    """Network output y [B][2][H][W] and the cache for backward()."""
    P = unpack(params, C)
    g1 = 1.0 + phi @ P["G1"].T
    be1 = phi @ P["H1"].T
    z1 = conv3x3(x, P["W1"])
    a1 = g1[:, :, None, None] * z1 + be1[:, :, None, None]
    h1 = np.maximum(a1, 0.0)
    g2 = 1.0 + phi @ P["G2"].T
    be2 = phi @ P["H2"].T
    z2 = conv3x3(h1, P["W2"])
    a2 = g2[:, :, None, None] * z2 + be2[:, :, None, None]
    h2 = np.maximum(a2, 0.0)
    y = conv3x3(h2, P["W3"]) + P["b3"][None, :, None, None]
    cache = dict(x=x, phi=phi, z1=z1, a1=a1, h1=h1, g1=g1, z2=z2, a2=a2, h2=h2, g2=g2)
    return y, cache


def backward(params: np.ndarray, cache: dict, dy: np.ndarray, C: int = C_HIDDEN):
    """(parameter gradient vector, input gradient dx) for the loss gradient dy."""
    P = unpack(params, C)
    phi = cache["phi"]
    grads = {}
    grads["b3"] = dy.sum(axis=(0, 2, 3))
    grads["W3"] = conv3x3_weight_grad(dy, cache["h2"])
    dh2 = conv3x3_input_grad(dy, P["W3"])
    da2 = dh2 * (cache["a2"] > 0)
    dg2 = (da2 * cache["z2"]).sum(axis=(2, 3))          # [B][C]
    db2 = da2.sum(axis=(2, 3))
    grads["G2"] = dg2.T @ phi
    grads["H2"] = db2.T @ phi
    dz2 = cache["g2"][:, :, None, None] * da2
    grads["W2"] = conv3x3_weight_grad(dz2, cache["h1"])
    dh1 = conv3x3_input_grad(dz2, P["W2"])
    da1 = dh1 * (cache["a1"] > 0)
    dg1 = (da1 * cache["z1"]).sum(axis=(2, 3))
    db1 = da1.sum(axis=(2, 3))
    grads["G1"] = dg1.T @ phi
    grads["H1"] = db1.T @ phi
    dz1 = cache["g1"][:, :, None, None] * da1
    grads["W1"] = conv3x3_weight_grad(dz1, cache["x"])
    dx = conv3x3_input_grad(dz1, P["W1"])
    return pack(grads, C), dx


def loss(y: np.ndarray, t: np.ndarray):
    """Mean over the batch of ||y_b - t_b||^2 / ||t_b||^2 and its gradient in y."""
    B = y.shape[0]
    tn = (t ** 2).sum(axis=(1, 2, 3))
    diff = y - t
    val = float(np.mean((diff ** 2).sum(axis=(1, 2, 3)) / tn))
    dy = 2.0 * diff / (tn[:, None, None, None] * B)
    return val, dy


def adam(params, grad, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) with bias correction; step >= 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad ** 2
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed: int = 0, C: int = C_HIDDEN) -> np.ndarray:
    """He-normal conv weights, zero FiLM maps and bias (drawn on the host, seeded)."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.standard_normal((C, 3, 3, 3)) * np.sqrt(2.0 / 27),
         "G1": np.zeros((C, N_FEAT)), "H1": np.zeros((C, N_FEAT)),
         "W2": rng.standard_normal((C, C, 3, 3)) * np.sqrt(2.0 / (9 * C)),
         "G2": np.zeros((C, N_FEAT)), "H2": np.zeros((C, N_FEAT)),
         "W3": rng.standard_normal((2, C, 3, 3)) * np.sqrt(1.0 / (9 * C)),
         "b3": np.zeros(2)}
    return pack(d, C)


def node_log_coefficient(ax: np.ndarray, ay: np.ndarray) -> np.ndarray:
    """log of the mean of the four face coefficients around each node, centred
    (mean subtracted); the third input channel.  Shape [m][m]."""
    a = 0.25 * (ax[:, :-1] + ax[:, 1:] + ay[:-1, :] + ay[1:, :])
    la = np.log(a)
    return la - la.mean()


def inner_apply(params: np.ndarray, lvls, r: np.ndarray, lam: complex, loga: np.ndarray,
                C: int = C_HIDDEN) -> np.ndarray:
    """The learned inner solve of one block: e1 = V(r), rho = r - B e1,
    e = S_r(e1 + s N(rho/s) / (lambda + d)) with s the root-mean-square of rho
    over both planes, d the diagonal of tau K_a and S_r one red-black
    Gauss-Seidel sweep for B e = r."""
    from . import mg
    m, wx, wy = lvls[0]
    e1 = mg.vcycle(lvls, 0, r, lam)
    rho = r - mg.apply_B(e1, lam, wx, wy)
    s = np.sqrt(np.mean(rho.real ** 2 + rho.imag ** 2) / 2.0)
    if s == 0.0:
        return e1
    x = np.stack([rho.real / s, rho.imag / s, loga])[None]
    y, _ = forward(params, x, features(np.array([lam])), C)
    corr = (y[0, 0] + 1j * y[0, 1]) / (lam + _diag(wx, wy))
    return mg.rbgs(e1 + s * corr, r, lam, wx, wy)


# ---------------------------------------------------------------- residual loss
# The correction y_b / (lambda_b + d) (y_b the network output, d the diagonal
# of tau K_a) is followed by one red-black Gauss-Seidel sweep S for B e = rho
# (normalised units) and scored by the residual it leaves:
#     L_b = ||rho_b - B S(y_b / (lambda_b + d))||^2 / ||rho_b||^2,
# which is the error against the multigrid correction delta (B delta = rho)
# measured in the norm ||B .||.  Arrays are real [B][2][H][W] (Re, Im); lam is
# complex per batch entry; wx [H][W+1], wy [H+1][W] are tau/h^2 face weights.

def _c(a):
    return a[:, 0] + 1j * a[:, 1]


def _r(z):
    return np.stack([z.real, z.imag], axis=1)


def _nbr(e, wx, wy):
    """sum over faces of w_f e_nbr for a batch [B][H][W] (complex), zero outside."""
    H, W = e.shape[-2:]
    s = np.zeros_like(e)
    s[:, :, 1:] += wx[None, :, 1:W] * e[:, :, :-1]
    s[:, :, :-1] += wx[None, :, 1:W] * e[:, :, 1:]
    s[:, 1:, :] += wy[None, 1:H, :] * e[:, :-1, :]
    s[:, :-1, :] += wy[None, 1:H, :] * e[:, 1:, :]
    return s


def _diag(wx, wy):
    return wx[:, :-1] + wx[:, 1:] + wy[:-1, :] + wy[1:, :]


def _colors(H, W):
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    red = (ii + jj) % 2 == 0
    return red, ~red


def sweep(y, rho, lam, wx, wy):
    """One red-black Gauss-Seidel sweep for B e = rho from e = y (batch)."""
    e = _c(y).copy()
    r = _c(rho)
    den = lam[:, None, None] + _diag(wx, wy)[None]
    for mask in _colors(*e.shape[-2:]):
        upd = (r + _nbr(e, wx, wy)) / den
        e[:, mask] = upd[:, mask]
    return _r(e)


def apply_B_batch(e, lam, wx, wy):
    z = _c(e)
    return _r((lam[:, None, None] + _diag(wx, wy)[None]) * z - _nbr(z, wx, wy))


def residual_loss(y, rho, lam, wx, wy):
    """(mean_b ||rho_b - B S(y_b / (lambda_b + d))||^2 / ||rho_b||^2, gradient in y)."""
    Bn = y.shape[0]
    rn = (rho ** 2).sum(axis=(1, 2, 3))
    cdiag = lam[:, None, None] + _diag(wx, wy)[None]
    e = sweep(_r(_c(y) / cdiag), rho, lam, wx, wy)
    q = rho - apply_B_batch(e, lam, wx, wy)
    val = float(np.mean((q ** 2).sum(axis=(1, 2, 3)) / rn))
    # gradient: dL/dq, then through B (B^H), then through the sweep (adjoint)
    dq = _c(2.0 * q / (rn[:, None, None, None] * Bn))
    g = -((np.conj(lam)[:, None, None] + _diag(wx, wy)[None]) * dq - _nbr(dq, wx, wy))
    den_c = np.conj(lam[:, None, None] + _diag(wx, wy)[None])
    red, black = _colors(*g.shape[-2:])
    # black half sweep: black' = (rho + W red')/den -> adds W^T (black grad / conj den) to red
    gb = np.where(black[None], g / den_c, 0.0)
    h = np.where(red[None], g + _nbr(gb, wx, wy), 0.0)
    # red half sweep: red' = (rho + W y_black)/den -> gradient to y at black points
    hr = h / den_c
    dy = np.where(black[None], _nbr(hr, wx, wy), 0.0)
    # through the pointwise division by lambda + d: the adjoint divides by its conjugate
    return val, _r(dy / np.conj(cdiag))
