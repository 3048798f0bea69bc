"""Error measure shared by the parity tests.

rel(a, b) is the larger of the relative 2-norm error ||a - b|| / ||b|| and
the normalised max-abs error max|a - b| / max|b|.  The 2-norm alone can hide
an error confined to a few entries (a tile edge, a padding row) under the
norm of millions of correct ones; the max-abs term exposes it.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = a - b
    nb = np.linalg.norm(b)
    mb = np.max(np.abs(b)) if b.size else 0.0
    r2 = np.linalg.norm(d) / (nb if nb > 0 else 1.0)
    rm = (np.max(np.abs(d)) if d.size else 0.0) / (mb if mb > 0 else 1.0)
    return float(max(r2, rm))


def trel(a, b):
    """rel for two torch tensors on the same device (no host copy)."""
    import torch
    d = a - b
    nb = float(torch.linalg.vector_norm(b))
    mb = float(b.abs().max()) if b.numel() else 0.0
    r2 = float(torch.linalg.vector_norm(d)) / (nb if nb > 0 else 1.0)
    rm = (float(d.abs().max()) if d.numel() else 0.0) / (mb if mb > 0 else 1.0)
    return max(r2, rm)
