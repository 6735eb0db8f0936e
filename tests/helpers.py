"""Shared test helpers: comparison metrics and device selection."""
import numpy as np


def rel(a, b) -> float:
    """Norm-wise relative error ||a - b||_2 / ||b||_2 over all entries."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gauge(f, g, T, M, b=None):
    """Fix the (f + c, g - c) freedom of the cross potentials: <a,f> = <b,g>."""
    a = np.full(T, 1.0 / T)
    b = np.full(M, 1.0 / M) if b is None else b
    c = 0.5 * (b @ np.asarray(g, np.float64) - a @ np.asarray(f, np.float64))
    return np.asarray(f, np.float64) + c, np.asarray(g, np.float64) - c
