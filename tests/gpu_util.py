"""Helpers for GPU tests (no solver arithmetic here)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)
