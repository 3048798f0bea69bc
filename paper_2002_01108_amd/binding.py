"""ctypes binding of libaao.so (the C ABI in include/aao.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Device arrays are torch tensors on the GPU (float64, contiguous); their data
pointers and torch's current HIP stream are handed to the library.  There is
no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaao.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENAN, ESTATE = 0, 1, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
INNERS = {"dst": 0, "dst_mean": 1, "mg": 2, "cnn": 3}
SIDES = {"right": 0, "left": 1}

# exported symbols and their signatures: (restype, argtypes)
_c_int, _c_double, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_pint, _pdbl = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
_pflt = ctypes.POINTER(ctypes.c_float)
SIGNATURES = {
    "aao_setup": (_c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _c_double, _c_double,
                           ctypes.POINTER(_vp)]),
    "aao_destroy": (None, [_vp]),
    "aao_set_stream": (_c_int, [_vp, _vp]),
    "aao_set_precision": (_c_int, [_vp, _c_int]),
    "aao_set_precision_schedule": (_c_int, [_vp, _c_int, _c_int]),
    "aao_build_rhs": (_c_int, [_vp, _vp, _vp, _vp]),
    "aao_apply_A": (_c_int, [_vp, _vp, _vp]),
    "aao_apply_Pinv": (_c_int, [_vp, _vp, _vp]),
    "aao_step1": (_c_int, [_vp, _vp, _vp]),
    "aao_step2": (_c_int, [_vp, _vp, _vp]),
    "aao_step3": (_c_int, [_vp, _vp, _vp]),
    "aao_solve": (_c_int, [_vp, _vp, _vp, _c_int, _c_double, _c_int, _c_int, _pint, _pdbl,
                           _c_int, _pint, _pdbl]),
    "aao_sync": (_c_int, [_vp]),
    "aao_status_string": (ctypes.c_char_p, [_c_int]),
    "aao_last_error": (ctypes.c_char_p, [_vp]),
    "aao_query": (_c_int, [_vp, _pint]),
    "aao_set_coefficient": (_c_int, [_vp, _pdbl, _pdbl, _pdbl]),
    "aao_set_inner": (_c_int, [_vp, _c_int, _c_int]),
    "aao_set_side": (_c_int, [_vp, _c_int]),
    "aao_set_scheme": (_c_int, [_vp, _c_int]),
    "aao_set_discretisation": (_c_int, [_vp, _c_int]),
    "aao_set_convection": (_c_int, [_vp, _c_double, _pdbl, _pdbl]),
    "aao_boundary_source": (_c_int, [_vp, _vp, _vp]),
    "aao_cnn_param_count": (_c_int, []),
    "aao_cnn_set_params": (_c_int, [_vp, _pflt, _c_int]),
    "aao_cnn_get_params": (_c_int, [_vp, _pflt, _c_int]),
    "aao_cnn_forward": (_c_int, [_vp, _vp, _pdbl, _c_int, _c_int, _c_int, _vp]),
    "aao_cnn_forward_noalloc": (_c_int, [_vp, _vp, _pdbl, _c_int, _c_int, _c_int, _vp]),
    "aao_cnn_backward": (_c_int, [_vp, _vp, _pdbl, _c_int, _c_int, _c_int, _vp, _vp, _pflt]),
    "aao_cnn_make_pairs": (_c_int, [_vp, _vp, _c_int, _c_int]),
    "aao_cnn_num_pairs": (_c_int, [_vp, _pint]),
    "aao_cnn_train": (_c_int, [_vp, _c_int, _c_int, ctypes.c_float, _pint, _pflt]),
    "aao_profile": (_c_int, [_vp, _c_int]),
    "aao_profile_read": (_c_int, [_vp, _pdbl, _pint]),
}
KERNEL_CLASSES = ["apply_L", "time_fwd", "time_inv", "dst", "divide", "krylov"]

_lib = None


class AaoError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{status_string(status)}: {msg}")


def load(path: str = LIB_PATH):
    """Load libaao.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2002_01108_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return load().aao_status_string(st).decode()


def _dptr(t, numel, device, dtype, what):
    """Data pointer of a contiguous GPU tensor of `dtype` with exactly `numel`
    elements on `device`; the library trusts these sizes, so they are checked
    here (a short array would be read or written past its end on the GPU)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a GPU torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what}: expected a contiguous {dtype} tensor")
    if t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
    if t.device.index != device:
        raise ValueError(f"{what}: on cuda:{t.device.index}, the context is on cuda:{device}")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One context of the library: grid, time steps, T, eps and precision."""

    def __init__(self, dim: int, m1: int, n: int, T: float = 1.0, eps: float | None = None,
                 precision: str = "fp64", m2: int | None = None, m3: int | None = None,
                 stream=None):
        import torch
        self.lib = load()
        self.dim, self.m1, self.n, self.T = dim, m1, n, T
        self.m2 = m1 if m2 is None else m2
        self.m3 = m1 if m3 is None else m3
        self.tau = T / n
        self.eps = min(0.5, (self.tau) ** 0.5) if eps is None else eps
        dims = [m1, self.m2, self.m3][:dim]
        self.m = int(np.prod(dims))
        self.device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        st = self.lib.aao_setup(dim, m1, self.m2, self.m3, n, T, self.eps, ctypes.byref(h))
        if st != OK:
            raise AaoError(st, "aao_setup")
        self._h = h
        s = stream if stream is not None else torch.cuda.current_stream()
        self._check(self.lib.aao_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)))
        self.set_precision(precision)

    def _vec(self, t, numel=None, what="space-time array"):
        """float64 device array of n*m elements (or `numel`) on this context's GPU."""
        import torch
        return _dptr(t, self.n * self.m if numel is None else numel, self.device, torch.float64,
                     what)

    def _fvec(self, t, numel, what):
        import torch
        return _dptr(t, numel, self.device, torch.float32, what)

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise AaoError(st, self.lib.aao_last_error(self._h).decode())
        return st

    def set_precision(self, precision: str):
        self.precision = precision
        self._check(self.lib.aao_set_precision(self._h, PRECISIONS[precision]))

    def set_precision_schedule(self, first: str = "fp32", steps: int = 1):
        """The first `steps` Arnoldi steps of each solve apply P^{-1} in `first`,
        the later ones in the context's precision (include/aao.h); steps = 0
        switches the schedule off."""
        self._check(self.lib.aao_set_precision_schedule(self._h, PRECISIONS[first], int(steps)))

    def set_coefficient(self, faces=None):
        """Face coefficients (host numpy arrays, see include/aao.h); None: a = 1."""
        if faces is None:
            self._check(self.lib.aao_set_coefficient(self._h, None, None, None))
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in faces]
        ms = [self.m1, self.m2, self.m3][: self.dim]
        if len(arrs) != self.dim:
            raise ValueError(f"expected {self.dim} face arrays, got {len(arrs)}")
        for d, a in enumerate(arrs):
            want = int(np.prod([v + (e == d) for e, v in enumerate(ms)]))
            if a.size != want:
                raise ValueError(f"face array {d}: {a.size} values, expected {want}")
        self._faces = arrs   # keep alive during the call
        ptrs = [a.ctypes.data_as(_pdbl) for a in arrs] + [None] * (3 - len(arrs))
        self._check(self.lib.aao_set_coefficient(self._h, *ptrs))

    def set_convection(self, nu=None, wind=None):
        """-nu Laplace + w . grad with upwinding on the unit square; wind =
        (wx, wy) host arrays [m2][m1] at the interior nodes (include/aao.h).
        No arguments: back to K = -Laplace."""
        if wind is None:
            self._check(self.lib.aao_set_convection(self._h, 0.0, None, None))
            return
        wx, wy = (np.ascontiguousarray(a, dtype=np.float64) for a in wind)
        for name, a in (("wx", wx), ("wy", wy)):
            if a.size != self.m1 * self.m2:
                raise ValueError(f"{name}: {a.size} values, expected {self.m1 * self.m2}")
        self._check(self.lib.aao_set_convection(self._h, float(nu), wx.ctypes.data_as(_pdbl),
                                                wy.ctypes.data_as(_pdbl)))

    def set_inner(self, inner: str = "dst", cycles: int = 1):
        self._check(self.lib.aao_set_inner(self._h, INNERS[inner], cycles))

    def set_scheme(self, order: int = 1):
        """Time discretisation: 1 = backward Euler, 2 = BDF2 with a
        backward-Euler first step (include/aao.h)."""
        self._check(self.lib.aao_set_scheme(self._h, int(order)))

    def set_discretisation(self, disc: str = "fd"):
        """'fd' (finite differences, M = I) or 'q1' (bilinear finite elements,
        2D square grids; include/aao.h)."""
        self._check(self.lib.aao_set_discretisation(self._h, {"fd": 0, "q1": 1}[disc]))

    def set_side(self, side: str = "right"):
        """'right' (flexible GMRES, true-residual stopping) or 'left' (GMRES on
        P^{-1} L u = P^{-1} rhs, preconditioned-residual stopping)."""
        self._check(self.lib.aao_set_side(self._h, SIDES[side]))

    # ------------------------------------------------------------ learned correction
    def cnn_param_count(self) -> int:
        return int(self.lib.aao_cnn_param_count())

    def cnn_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.aao_cnn_set_params(self._h, p.ctypes.data_as(_pflt), p.size))

    def cnn_get_params(self):
        p = np.zeros(self.cnn_param_count(), dtype=np.float32)
        self._check(self.lib.aao_cnn_get_params(self._h, p.ctypes.data_as(_pflt), p.size))
        return p

    @staticmethod
    def _lam(lam):
        lam = np.asarray(lam, dtype=np.complex128).reshape(-1)
        return np.ascontiguousarray(np.stack([lam.real, lam.imag], -1))

    def cnn_forward(self, x, lam):
        """x: GPU float32 [B][3][H][W]; lam: B complex values. Returns y [B][2][H][W]."""
        import torch
        B, _, H, W = x.shape
        y = torch.empty((B, 2, H, W), dtype=torch.float32, device=x.device)
        la = self._lam(lam)
        self._check(self.lib.aao_cnn_forward(self._h, self._fvec(x, B * 3 * H * W, "x"),
                                             la.ctypes.data_as(_pdbl), B, H, W,
                                             self._fvec(y, B * 2 * H * W, "y")))
        return y

    def cnn_forward_noalloc(self, x, lam, out=None):
        """As cnn_forward, through the entry point that allocates nothing (its
        workspace is the library's fixed per-GPU array); out: optional
        preallocated float32 [B][2][H][W]."""
        import torch
        B, _, H, W = x.shape
        y = torch.empty((B, 2, H, W), dtype=torch.float32, device=x.device) if out is None else out
        la = self._lam(lam)
        self._check(self.lib.aao_cnn_forward_noalloc(
            self._h, self._fvec(x, B * 3 * H * W, "x"), la.ctypes.data_as(_pdbl), B, H, W,
            self._fvec(y, B * 2 * H * W, "y")))
        return y

    def cnn_backward(self, x, lam, dy):
        """(parameter gradient numpy float32, input gradient GPU tensor)."""
        import torch
        B, _, H, W = x.shape
        dx = torch.empty_like(x)
        g = np.zeros(self.cnn_param_count(), dtype=np.float32)
        la = self._lam(lam)
        self._check(self.lib.aao_cnn_backward(
            self._h, self._fvec(x, B * 3 * H * W, "x"), la.ctypes.data_as(_pdbl), B, H, W,
            self._fvec(dy, B * 2 * H * W, "dy"), self._fvec(dx, B * 3 * H * W, "dx"),
            g.ctypes.data_as(_pflt)))
        return g, dx

    def cnn_make_pairs(self, y, target_cycles: int = 12):
        """y: GPU float64 [S][n][m] space-time fields."""
        S = y.shape[0]
        self._check(self.lib.aao_cnn_make_pairs(self._h, self._vec(y, S * self.n * self.m, "y"),
                                                S, target_cycles))
        cnt = ctypes.c_int(0)
        self._check(self.lib.aao_cnn_num_pairs(self._h, ctypes.byref(cnt)))
        return cnt.value

    def cnn_train(self, idx, lr: float = 3e-3):
        """idx: int array [steps][batch] of pair indices. Returns the loss per step."""
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        steps, batch = idx.shape
        loss = np.zeros(steps, dtype=np.float32)
        self._check(self.lib.aao_cnn_train(self._h, steps, batch, lr, idx.ctypes.data_as(_pint),
                                           loss.ctypes.data_as(_pflt)))
        return loss

    def query(self):
        out = (ctypes.c_int * 9)()
        self._check(self.lib.aao_query(self._h, out))
        return list(out)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.aao_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ operators
    def new(self, *shape):
        import torch
        shape = shape or (self.n, self.m)
        return torch.empty(shape, dtype=torch.float64, device="cuda")

    def build_rhs(self, f, u0, out=None):
        out = self.new() if out is None else out
        self._check(self.lib.aao_build_rhs(self._h, self._vec(f, what="f"),
                                           self._vec(u0, self.m, "u0"), self._vec(out, what="out")))
        return out

    def boundary_source(self, gb, f):
        """f += boundary couplings x Dirichlet values gb (device [n][2 m2 + 2 m1]:
        west, east, south, north walls per time level); f updated in place."""
        nb = self.n * 2 * (self.m1 + self.m2)
        self._check(self.lib.aao_boundary_source(self._h, self._vec(gb, nb, "gb"),
                                                 self._vec(f, what="f")))
        return f

    def apply_A(self, x, out=None):
        out = self.new() if out is None else out
        self._check(self.lib.aao_apply_A(self._h, self._vec(x, what="x"),
                                         self._vec(out, what="out")))
        return out

    def apply_Pinv(self, x, out=None):
        out = self.new() if out is None else out
        self._check(self.lib.aao_apply_Pinv(self._h, self._vec(x, what="x"),
                                            self._vec(out, what="out")))
        return out

    def step1(self, y):
        out = self.new(self.n // 2 + 1, self.m, 2)
        self._check(self.lib.aao_step1(self._h, self._vec(y, what="y"),
                                       self._vec(out, out.numel(), "out")))
        return out

    def step2(self, yt):
        out = self.new(self.n // 2 + 1, self.m, 2)
        self._check(self.lib.aao_step2(self._h, self._vec(yt, out.numel(), "yt"),
                                       self._vec(out, out.numel(), "out")))
        return out

    def step3(self, zt):
        out = self.new()
        nzt = (self.n // 2 + 1) * self.m * 2
        self._check(self.lib.aao_step3(self._h, self._vec(zt, nzt, "zt"), self._vec(out, what="out")))
        return out

    def solve(self, rhs, tol: float = 1e-8, maxit: int = 100, restart: int = 50, u=None,
              use_guess: bool = False):
        """Returns (u, info) with info = dict(status, iters, hist, final_res)."""
        u = self.new() if u is None else u
        iters = ctypes.c_int(0)
        cap = max(maxit, 1)
        hist = (ctypes.c_double * cap)()
        hlen = ctypes.c_int(0)
        fres = ctypes.c_double(float("nan"))
        st = self.lib.aao_solve(self._h, self._vec(rhs, what="rhs"), self._vec(u, what="u"),
                                int(use_guess), tol, maxit, restart,
                                ctypes.byref(iters), hist, cap, ctypes.byref(hlen),
                                ctypes.byref(fres))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return u, {"status": st, "iters": iters.value, "hist": list(hist[: hlen.value]),
                   "final_res": fres.value}

    def sync(self):
        self._check(self.lib.aao_sync(self._h))

    def profile(self, classes=None):
        """Start event timing of the named kernel classes (None: stop)."""
        mask = 0
        for name in classes or ():
            mask |= 1 << KERNEL_CLASSES.index(name)
        self._check(self.lib.aao_profile(self._h, mask))

    def profile_read(self):
        """{class: (total_ms, launches)} since profile() was called."""
        nc = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * nc)()
        cnt = (ctypes.c_int * nc)()
        self._check(self.lib.aao_profile_read(self._h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}
