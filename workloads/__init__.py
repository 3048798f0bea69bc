"""Seeded synthetic inputs for the all-at-once heat-equation solve.

This module is shared by the CPU oracle and the GPU path.  It draws and samples
inputs only: the source f, the initial value u0, the diffusion coefficient a on
cell faces, the manufactured solution of the paper's variable-coefficient
example (Section 5, Example 2), and the wind and hot-wall boundary data of its
convection-diffusion example (Section 5, Example 3).  It holds none of the method's arithmetic (no
operator, transform, preconditioner or Krylov step).

Conventions
-----------
* Domain (0,1)^d, `m1` interior points per dimension, spacing h = 1/(m1+1),
  interior node i (0-based) at x = (i+1) h.  Homogeneous Dirichlet data.
* A space-time array has shape [n][m3][m2][m1] (x fastest); time level k
  (0-based) is t_{k+1} = (k+1) tau, tau = T/n (Section 2, eq. (stepsystem)).
* Face arrays (coefficient a at face midpoints), x-faces between node i-1 and
  node i sit at x = (i+1/2) h for i = 0..m1:
    1D: ax[m1+1]
    2D: ax[m2][m1+1], ay[m2+1][m1]
    3D: ax[m3][m2][m1+1], ay[m3][m2+1][m1], az[m3+1][m2][m1]
* Random streams: numpy PCG64; f from `seed`, u0 from `seed+1`, a from `seed+2`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One heat-equation workload: grid, time steps, horizon and epsilon."""
    name: str
    dim: int
    m1: int
    n: int
    T: float = 1.0
    eps: float | None = None          # None -> sqrt(tau) capped at 0.5
    u0_kind: str = "modes"            # "sine" | "modes" | "zero"
    coefficient: str = "const"        # "const" | "grf" | "wind"
    precision: str = "fp64"           # preconditioner arithmetic
    inner: str = "dst"
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.m1,) * self.dim

    @property
    def m(self) -> int:
        return self.m1 ** self.dim

    @property
    def tau(self) -> float:
        return self.T / self.n

    @property
    def epsilon(self) -> float:
        if self.eps is not None:
            return self.eps
        return min(0.5, math.sqrt(self.tau))

    @property
    def dof(self) -> int:
        return self.n * self.m


# The five workloads: 1D/2D/3D constant coefficient and the 2D variable one.
WORKLOADS = {
    "heat1d_63x64": Workload("heat1d_63x64", 1, 63, 64, u0_kind="sine"),
    "heat2d_255x256": Workload("heat2d_255x256", 2, 255, 256, u0_kind="modes"),
    "heat2d_511x512": Workload("heat2d_511x512", 2, 511, 512, u0_kind="modes",
                               precision="fp32"),
    "heat3d_127x256": Workload("heat3d_127x256", 3, 127, 256, u0_kind="zero",
                               precision="fp32"),
    "varheat2d_255x256": Workload("varheat2d_255x256", 2, 255, 256, u0_kind="modes",
                                  coefficient="grf", inner="cnn"),
    # Section 5, Example 3 on (-1, 1)^2: J+1 = 256, N = 256, eps = 0.5 tau
    "cd2d_255x256": Workload("cd2d_255x256", 2, 255, 256, eps=0.5 / 256, u0_kind="zero",
                             coefficient="wind", inner="mg"),
}

# Section 5, Example 3: diffusion 1/200 on (-1, 1)^2, circulating wind, a hot
# wall x = 1 whose temperature rises as 1 - exp(-10 t), zero elsewhere and at t = 0.
CD_NU = 1.0 / 200.0


def cd_nodes(m1: int) -> np.ndarray:
    """Interior node coordinates on (-1, 1): -1 + (i+1) h, h = 2/(m1+1)."""
    return -1.0 + (2.0 / (m1 + 1)) * np.arange(1, m1 + 1)


def cd_wind(m1: int):
    """(w1, w2) = (2y(1-x^2), -2x(1-y^2)) at the interior nodes, [m1][m1] (y, x)."""
    x = cd_nodes(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    return 2.0 * Y * (1.0 - X * X), -2.0 * X * (1.0 - Y * Y)


def cd_hot_wall(m1: int, n: int, T: float = 1.0) -> np.ndarray:
    """Boundary values [n][4 m1] at t_k = (k+1) T/n next to the west, east,
    south and north walls (m1 each): 1 - exp(-10 t) on the east wall x = 1,
    zero on the others."""
    g = np.zeros((n, 4 * m1))
    t = (np.arange(n) + 1) * (T / n)
    g[:, m1:2 * m1] = (1.0 - np.exp(-10.0 * t))[:, None]
    return g


def node_coords(m1: int) -> np.ndarray:
    """Interior node coordinates (i+1) h, i = 0..m1-1."""
    h = 1.0 / (m1 + 1)
    return (np.arange(m1, dtype=np.float64) + 1.0) * h


def source(n: int, m1: int, dim: int, seed: int = 0) -> np.ndarray:
    """f ~ N(0,1) iid per interior node and time level t_1..t_n; shape [n][m]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = m1 ** dim
    out = np.empty((n, m), dtype=np.float64)
    for k in range(n):            # row by row keeps peak memory low for big grids
        out[k] = rng.standard_normal(m)
    return out


def initial_value(m1: int, dim: int, kind: str, seed: int = 1, modes: int = 16) -> np.ndarray:
    """u0 on interior nodes, flattened x-fastest.

    sine  : product of sin(pi x_d)
    modes : sum of `modes` products sin(k1 pi x) sin(k2 pi y) [sin(k3 pi z)] with
            distinct wavenumber tuples drawn from {1..16}^dim and N(0,1) weights
    zero  : 0
    """
    x = node_coords(m1)
    if kind == "zero":
        return np.zeros(m1 ** dim)
    if kind == "sine":
        s = np.sin(math.pi * x)
        u = s
        for _ in range(dim - 1):
            u = np.multiply.outer(s, u)
        return np.ascontiguousarray(u).reshape(-1)
    if kind != "modes":
        raise ValueError(kind)
    rng = np.random.Generator(np.random.PCG64(seed))
    cand = 16 ** dim
    pick = rng.choice(cand, size=modes, replace=False)
    weights = rng.standard_normal(modes)
    u = np.zeros((m1,) * dim)
    for p, c in zip(pick, weights):
        ks = []
        q = int(p)
        for _ in range(dim):
            ks.append(q % 16 + 1)
            q //= 16
        term = np.sin(ks[0] * math.pi * x)          # along x (fastest)
        for d in range(1, dim):
            term = np.multiply.outer(np.sin(ks[d] * math.pi * x), term)
        u += c * term
    return u.reshape(-1)


def constant_faces(m1: int, dim: int, value: float = 1.0):
    """Face arrays for a constant coefficient (see module docstring for shapes)."""
    return tuple(np.full(s, value) for s in face_shapes(m1, dim))


def face_shapes(m1: int, dim: int):
    """Shapes of (ax[, ay[, az]]) for an m1^dim grid, slowest index first."""
    shapes = []
    for d in range(dim):             # d = 0: x, 1: y, 2: z
        s = [m1] * dim               # order [z][y][x] -> index dim-1-d is axis d
        s[dim - 1 - d] = m1 + 1
        shapes.append(tuple(s))
    return shapes


def grf_faces(m1: int, dim: int = 2, seed: int = 2, corr_len: float = 0.1,
              contrast: float = 100.0):
    """a = exp(g) on faces, g a Gaussian random field with Gaussian covariance.

    The field is synthesised spectrally on a periodic grid of spacing h/2 over
    [0,2)^dim (twice the domain, so the wrap-around does not couple opposite
    walls), sampled at face midpoints, affinely mapped to [-1,1] over the
    sampled faces, and exponentiated so that max(a)/min(a) == contrast.
    """
    if dim != 2:
        raise NotImplementedError("the variable-coefficient workload is 2D")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / (m1 + 1)
    ng = 4 * (m1 + 1)
    dx = h / 2.0
    noise = rng.standard_normal((ng, ng))
    kk = 2.0 * math.pi * np.fft.fftfreq(ng, d=dx)
    k2 = kk[:, None] ** 2 + kk[None, :] ** 2
    amp = np.exp(-0.25 * corr_len ** 2 * k2)        # sqrt of the Gaussian spectrum
    g = np.real(np.fft.ifft2(np.fft.fft2(noise) * amp))
    # half-spacing grid index p <-> coordinate p*dx; node i -> 2(i+1), face f -> 2f+1
    nodes = 2 * (np.arange(m1) + 1)
    faces = 2 * np.arange(m1 + 1) + 1
    gx = g[np.ix_(nodes, faces)]          # [y=node][x=face]
    gy = g[np.ix_(faces, nodes)]          # [y=face][x=node]
    lo = min(gx.min(), gy.min())
    hi = max(gx.max(), gy.max())
    half_log = 0.5 * math.log(contrast)

    def mapped(v):
        return np.exp((2.0 * (v - lo) / (hi - lo) - 1.0) * half_log)

    return mapped(gx), mapped(gy)


# Manufactured solution of the variable-coefficient example (Section 5, Example 2):
# u = exp(-t) x(1-x) y(1-y) with a = sin(pi x y).  The printed source term matches
# this u only for the unscaled coefficient sin(pi x y), which is the reading used.

def manufactured_u(m1: int, t: float) -> np.ndarray:
    x = node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")      # [y][x]
    return (math.exp(-t) * X * (1 - X) * Y * (1 - Y)).reshape(-1)


def manufactured_f(m1: int, t: float) -> np.ndarray:
    x = node_coords(m1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    s = np.sin(math.pi * X * Y)
    c = np.cos(math.pi * X * Y)
    e = math.exp(-t)
    f = (e * X * (1 - X) * (2 * s - Y * (1 - Y) - math.pi * c * X * (1 - 2 * Y))
         + e * Y * (1 - Y) * (2 * s - math.pi * c * Y * (1 - 2 * X)))
    return f.reshape(-1)


def manufactured_faces(m1: int):
    """a = sin(pi x y) at face midpoints, shapes ax[m1][m1+1], ay[m1+1][m1]."""
    h = 1.0 / (m1 + 1)
    x = node_coords(m1)
    xf = (np.arange(m1 + 1) + 0.5) * h
    ax = np.sin(math.pi * np.multiply.outer(x, xf))     # [y node][x face]
    ay = np.sin(math.pi * np.multiply.outer(xf, x))     # [y face][x node]
    return ax, ay


def make(workload: Workload | str, seed: int = 0):
    """(f [n][m], u0 [m], faces or None) for a named or given workload."""
    w = WORKLOADS[workload] if isinstance(workload, str) else workload
    f = np.zeros((w.n, w.m)) if w.coefficient == "wind" else source(w.n, w.m1, w.dim, seed)
    u0 = initial_value(w.m1, w.dim, w.u0_kind, seed + 1)
    faces = grf_faces(w.m1, w.dim, seed + 2) if w.coefficient == "grf" else None
    return f, u0, faces


def cnn_init_params(seed: int = 0, C: int = 8) -> np.ndarray:
    """Initial parameters of the learned inner solve, drawn seeded on the host in
    the library's flat layout W1[C][3][3][3] G1[C][4] H1[C][4] W2[C][C][3][3]
    G2[C][4] H2[C][4] W3[2][C][3][3] b3[2]: He-normal convolution weights, zero
    FiLM maps and bias (FP64; the library stores FP32)."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal(C * 27) * np.sqrt(2.0 / 27)
    w2 = rng.standard_normal(C * C * 9) * np.sqrt(2.0 / (9 * C))
    w3 = rng.standard_normal(2 * C * 9) * np.sqrt(1.0 / (9 * C))
    film = np.zeros(2 * C * 4)
    return np.concatenate([w1, film, w2, film, w3, np.zeros(2)])
