"""Layout helpers for comparing the HIP library's state with the oracle's.

These only reshape and re-interpret buffers (interleaved complex, the packed
form of C); no coding or learning arithmetic lives here.
"""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


def spectra(flat: np.ndarray, lead: tuple, ph: int, pw: int) -> np.ndarray:
    """Interleaved complex [*lead][Pf] -> complex array (*lead, ph, pw//2+1)."""
    z = flat[0::2] + 1j * flat[1::2]
    return z.reshape(lead + (ph, pw // 2 + 1))


def unpack_cinv(flat: np.ndarray, K: int, ph: int, pw: int) -> np.ndarray:
    """Packed C [Pf][K][K] (Re above/on the diagonal, Im below) -> (ph, wc, K, K) complex."""
    R = flat.reshape(-1, K, K)
    up = np.triu(R)
    re = up + np.triu(R, 1).transpose(0, 2, 1)
    lo = np.tril(R, -1)                      # lo[j][i] = Im C_ij for i < j
    im = lo.transpose(0, 2, 1) - lo
    return (re + 1j * im).reshape(ph, pw // 2 + 1, K, K)


def pack_cinv(C: np.ndarray) -> np.ndarray:
    """(..., K, K) Hermitian complex -> packed [Pf][K][K] reals."""
    K = C.shape[-1]
    C = C.reshape(-1, K, K)
    R = np.triu(C.real) + np.tril(C.imag.transpose(0, 2, 1), -1)
    return R.reshape(-1)


def interleave(z: np.ndarray) -> np.ndarray:
    out = np.empty(z.size * 2)
    out[0::2] = z.real.ravel()
    out[1::2] = z.imag.ravel()
    return out
