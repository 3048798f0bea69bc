"""Learned inner solve on the GPU: network arithmetic against the FP64 oracle,
the full learned inner application, training, and what the trained network
gains over the multigrid fallback on data it has not seen.

Tolerances: FP32 forward 1e-5 and input gradient 1e-5 (relative 2-norm, u = 6e-8
times at most 27 * 8 terms per output); parameter gradients 1e-4 (sums over all
pixels of a batch in FP32); learned inner solve 1e-5 relative to the V-cycle part.
"""
import numpy as np
import pytest

from oracle import cnn, heat, mg
import workloads as W
from errnorms import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def params_for(seed):
    p = W.cnn_init_params(seed)
    return p + 0.05 * np.random.default_rng(seed + 100).standard_normal(p.size)


def solver(m1=15, n=8, faces=None, precision="fp64"):
    from paper_2002_01108_amd import Solver
    s = Solver(2, m1, n, precision=precision)
    if faces is not None:
        s.set_coefficient(faces)
    return s


def test_param_count_matches_oracle_layout():
    s = solver()
    assert s.cnn_param_count() == cnn.layout()[1]


@pytest.mark.parametrize("B,H,W", [(3, 7, 9), (2, 37, 41), (1, 1, 1)])
def test_forward_and_backward_match_oracle(B, H, W):
    s = solver()
    p = params_for(1)
    s.cnn_set_params(p.astype(np.float32))
    rng = np.random.default_rng(2)
    x = rng.standard_normal((B, 3, H, W))
    lam = 1 - 0.9 * np.exp(2j * np.pi * rng.uniform(size=B))
    p32 = p.astype(np.float32).astype(np.float64)       # same parameters on both sides
    y_or, cache = cnn.forward(p32, x, cnn.features(lam))
    y = host(s.cnn_forward(dev32(x), lam))
    assert rel(y, y_or) <= 1e-5
    dy = rng.standard_normal(y.shape)
    g_or, dx_or = cnn.backward(p32, cache, dy)
    g, dx = s.cnn_backward(dev32(x), lam, dev32(dy))
    assert rel(host(dx), dx_or) <= 1e-5
    for name, shp, off, size in cnn.layout()[0]:
        assert rel(g[off:off + size], g_or[off:off + size]) <= 1e-4, name


def test_set_params_validation():
    from paper_2002_01108_amd import AaoError
    s = solver()
    with pytest.raises(AaoError):
        s.cnn_set_params(np.zeros(10, np.float32))
    bad = W.cnn_init_params(0).astype(np.float32)
    bad[3] = np.nan
    with pytest.raises(AaoError):
        s.cnn_set_params(bad)
    with pytest.raises(AaoError):
        s.set_inner("cnn")          # no parameters yet
    s.cnn_set_params(W.cnn_init_params(0).astype(np.float32))
    assert np.array_equal(s.cnn_get_params(), W.cnn_init_params(0).astype(np.float32))


def test_learned_inner_solve_matches_oracle():
    m1, n = 31, 16
    faces = W.grf_faces(m1, 2, seed=3)
    p = heat.Problem(m1, 2, n, faces=faces)
    s = solver(m1, n, faces)
    prm = params_for(4).astype(np.float32)
    s.cnn_set_params(prm)
    s.set_inner("cnn")
    rng = np.random.default_rng(5)
    yt = rng.standard_normal((n // 2 + 1, p.m, 2))
    yt[0, :, 1] = 0.0
    yt[-1, :, 1] = 0.0
    got = host(s.step2(dev(yt)))
    got = got[..., 0] + 1j * got[..., 1]
    lam = heat.lambdas(n, p.eps)[: n // 2 + 1]
    lv = mg.levels(faces[0], faces[1], p.tau)
    loga = cnn.node_log_coefficient(*faces)
    prm64 = prm.astype(np.float64)
    for k in range(n // 2 + 1):
        r = (yt[k, :, 0] + 1j * yt[k, :, 1]).reshape(m1, m1)
        want = cnn.inner_apply(prm64, lv, r, lam[k], loga).reshape(-1)
        e1 = mg.vcycle(lv, 0, r, lam[k]).reshape(-1)
        # FP32 network: error relative to the size of its correction, and overall
        assert np.linalg.norm(got[k] - want) <= 1e-5 * np.linalg.norm(want - e1) + 1e-12 * np.linalg.norm(want)


def test_training_pairs_and_loss_match_oracle():
    """First-step residual loss of training on GPU-made pairs equals the oracle's
    loss on oracle-made pairs of the same fields; the first Adam step moves each
    parameter with a clear gradient by about lr against its gradient sign."""
    m1, n, S = 15, 8, 2
    faces = W.grf_faces(m1, 2, seed=6)
    p = heat.Problem(m1, 2, n, faces=faces)
    s = solver(m1, n, faces)
    prm = params_for(7).astype(np.float32)
    s.cnn_set_params(prm)
    rng = np.random.default_rng(8)
    ys = rng.standard_normal((S, n, p.m))
    npairs = s.cnn_make_pairs(dev(ys), target_cycles=30)
    nh = n // 2 + 1
    assert npairs == S * nh
    # oracle pairs
    lam = heat.lambdas(n, p.eps)[:nh]
    lv = mg.levels(faces[0], faces[1], p.tau)
    loga = cnn.node_log_coefficient(*faces)
    X, PHI, LAM = [], [], []
    for sidx in range(S):
        yt = heat.step1(ys[sidx], p.eps)
        for k in range(nh):
            r = yt[k].reshape(m1, m1)
            e1 = mg.vcycle(lv, 0, r, lam[k])
            rho = r - mg.apply_B(e1, lam[k], lv[0][1], lv[0][2])
            sc = np.sqrt(np.mean(rho.real ** 2 + rho.imag ** 2) / 2)
            X.append(np.stack([rho.real / sc, rho.imag / sc, loga]))
            PHI.append(cnn.features(lam[k]))
            LAM.append(lam[k])
    X, PHI, LAM = np.array(X), np.array(PHI), np.array(LAM)
    idx = np.array([[0, 3, 5, 9]])
    loss = s.cnn_train(idx, lr=1e-3)
    prm64 = prm.astype(np.float64)
    b = idx[0]
    y_or, cache = cnn.forward(prm64, X[b], PHI[b])
    l_or, dy_or = cnn.residual_loss(y_or, X[b, :2], LAM[b], lv[0][1], lv[0][2])
    assert loss[0] == pytest.approx(l_or, rel=1e-4)
    g_or, _ = cnn.backward(prm64, cache, dy_or)
    p1 = s.cnn_get_params().astype(np.float64)
    clear = np.abs(g_or) > 1e-2 * np.abs(g_or).max()
    want = prm64 - 1e-3 * np.sign(g_or)
    assert np.allclose(p1[clear], want[clear], atol=2e-5)


def _block_residual(p, lam, yt, z):
    """||yt_k - B_k z_k|| / ||yt_k|| over all kept blocks (oracle operator)."""
    num = den = 0.0
    for k in range(yt.shape[0]):
        rk = yt[k] - (lam[k] * z[k] + p.tau * (p.K @ z[k]))
        num += np.linalg.norm(rk) ** 2
        den += np.linalg.norm(yt[k]) ** 2
    return np.sqrt(num / den)


def test_trained_network_gains_over_multigrid():
    """Train on pairs from seeded random fields, then measure on data the network
    has not seen, against two baselines: the multigrid fallback (one V-cycle)
    and the same learned inner solve with a zero network, i.e. the V-cycle plus
    the extra red-black sweep that wraps the network (the equal-structure
    control, so the gain below is the network's own).  The trained network
    leaves a smaller block residual per inner application than both, FGMRES
    needs no more iterations with it than with either, and every solution
    matches sequential backward Euler."""
    m1, n = 63, 64
    faces = W.grf_faces(m1, 2, seed=2)
    p = heat.Problem(m1, 2, n, faces=faces)
    s = solver(m1, n, faces)
    s.cnn_set_params(W.cnn_init_params(11).astype(np.float32))
    rng = np.random.default_rng(12)
    ys = rng.standard_normal((6, n, p.m))
    npairs = s.cnn_make_pairs(dev(ys), target_cycles=20)
    steps, batch = 1500, 8
    idx = np.random.default_rng(13).integers(0, npairs, size=(steps, batch))
    loss = s.cnn_train(idx, lr=3e-3)
    assert np.mean(loss[-100:]) < 0.5 * np.mean(loss[:20])
    trained = s.cnn_get_params()
    zero = np.zeros_like(trained)

    def use(inner):
        if inner == "mg":
            s.set_inner("mg")
        else:
            s.cnn_set_params(trained if inner == "cnn" else zero)
            s.set_inner("cnn")

    # block residual per inner application on a held-out field and on the first
    # Krylov vector of the held-out solve
    lam = heat.lambdas(n, p.eps)[: n // 2 + 1]
    f = np.random.default_rng(14).standard_normal((n, p.m))
    rhs = p.rhs(f, W.initial_value(m1, 2, "modes", 15))
    for field in (np.random.default_rng(16).standard_normal((n, p.m)),
                  rhs / np.linalg.norm(rhs)):
        yt = heat.step1(field, p.eps)
        yt_ext = np.stack([yt.real, yt.imag], -1)
        r = {}
        for inner in ("mg", "sweep", "cnn"):
            use(inner)
            z = host(s.step2(dev(yt_ext)))
            r[inner] = _block_residual(p, lam, yt, z[..., 0] + 1j * z[..., 1])
        print("block residual per application", r, flush=True)
        assert r["cnn"] < 0.8 * r["sweep"] < 0.8 * r["mg"], r

    exact = p.exact(rhs)
    its = {}
    for inner in ("mg", "sweep", "cnn"):
        use(inner)
        u, info = s.solve(dev(rhs), tol=1e-10, maxit=100)
        assert info["status"] == 0
        assert rel(host(u), exact) <= 1e-8
        its[inner] = info["iters"]
    print("FGMRES iterations", its, flush=True)
    assert its["cnn"] <= its["sweep"] <= its["mg"], its
