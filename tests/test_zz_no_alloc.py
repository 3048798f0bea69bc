"""The allocation-free learned forward (aao_cnn_forward_noalloc) against the
allocating one (aao_cnn_forward), through the C ABI: two calls in a row, the
second with a smaller input (the fixed workspace keeps the first call's
contents), each within the FP32 network tolerance of the other and of the
FP64 oracle; requests beyond the fixed workspace are refused before any
device work."""
import numpy as np
import pytest

from errnorms import rel
from oracle import cnn
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_forward_matches_forward(lib):
    from paper_2002_01108_amd import Solver
    s = Solver(2, 15, 8)
    prm = W.cnn_init_params(3) + 0.05 * np.random.default_rng(4).standard_normal(
        W.cnn_init_params(3).size)
    prm32 = prm.astype(np.float32)
    s.cnn_set_params(prm32)
    rng = np.random.default_rng(5)
    for B, H, Wd in ((9, 63, 63), (3, 17, 29)):          # the second call is smaller
        x = rng.standard_normal((B, 3, H, Wd))
        lam = 1 - 0.9 * np.exp(2j * np.pi * rng.uniform(size=B))
        y_ref = host(s.cnn_forward(dev32(x), lam))
        y = host(s.cnn_forward_noalloc(dev32(x), lam))
        assert y.shape == y_ref.shape
        assert rel(y, y_ref) <= 1e-6
        y_or, _ = cnn.forward(prm32.astype(np.float64), x, cnn.features(lam))
        assert rel(y, y_or) <= 1e-5
        print(f"B={B} {H}x{Wd}: vs forward {rel(y, y_ref):.2e} "
              f"(bitwise {np.array_equal(y, y_ref)}), vs oracle {rel(y, y_or):.2e}", flush=True)


def test_noalloc_forward_rejects_oversize_and_bad_lambda():
    from paper_2002_01108_amd import AaoError, Solver
    s = Solver(2, 15, 8)
    x = torch.zeros((4, 3, 600, 600), dtype=torch.float32, device="cuda")   # 1.44 M pixels
    lam = np.full(4, 0.5 + 0.1j)
    with pytest.raises(AaoError) as e:
        s.cnn_forward_noalloc(x, lam)
    assert e.value.status == -5                     # no parameters yet
    s.cnn_set_params(W.cnn_init_params(0).astype(np.float32))
    with pytest.raises(AaoError) as e:
        s.cnn_forward_noalloc(x, lam)
    assert e.value.status == -1 and "fixed workspace" in str(e.value)
    small = torch.zeros((2, 3, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(AaoError) as e:
        s.cnn_forward_noalloc(small, np.array([0.0, 1.0]))
    assert e.value.status == -1
