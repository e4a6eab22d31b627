"""Helpers for GPU tests (no solver arithmetic here)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def excess(a, b, rtol, floor):
    """Element-wise gate: max_j |a_j - b_j| / (rtol |b_j| + floor max_k |b_k|).
    A value <= 1 passes; the floor keeps entries near zero (rates at the lower
    end of the box, prices of slack links) from needing relative accuracy that
    their absolute rounding cannot give."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    scale = np.max(np.abs(b))
    den = rtol * np.abs(b) + floor * (scale if scale > 0 else 1.0)
    return float(np.max(np.abs(a - b) / den))


# element-wise gates (rtol, floor as a fraction of the largest entry)
F64_ELEM = (1e-10, 1e-12)
F32_ELEM = (1e-4, 1e-7)
# over a whole solve (thousands of iterations) single entries of the exact
# iteration itself move by more than 1e-4: on the medium workload at its
# 2380-iteration solve, the FP64 oracle run on data perturbed by one FP32 ulp
# (c, w times 1 +- 2^-24) differs from the unperturbed run by up to 3.2e-4
# relative in x (normwise 1.9e-7), so the element-wise gate is 10x looser
F32_ELEM_SOLVE = (1e-3, 1e-6)


def close(a, b, bits):
    """Both parity gates at once: normwise (1e-10 for FP64, 1e-5 for FP32)
    and element-wise (F64_ELEM / F32_ELEM)."""
    tol, elem = (1e-10, F64_ELEM) if bits == 64 else (1e-5, F32_ELEM)
    return rel(a, b) <= tol and excess(a, b, *elem) <= 1.0
