"""FP64 CPU oracle for proximal message passing on NUM -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The HIP library never imports, links or calls it.

`run` drives the literal per-terminal PMP in `pmp_oracle.c` (built with gcc
into `oracle/_build/liboracle.so`); `optimality` holds the converged-run
checker and the closed-form optima that pin it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("utility", ctypes.c_void_p), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("alpha", ctypes.c_double),
                ("mu", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eps_abs", ctypes.c_double), ("adapt_every", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("stop", ctypes.c_int32), ("threads", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("r_norm", ctypes.c_double),
                ("s_norm", ctypes.c_double), ("eps_tol", ctypes.c_double),
                ("rho", ctypes.c_double), ("converged", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Params)] + \
            [ctypes.c_void_p] * 15 + [ctypes.POINTER(_Result)]
        for name in ("orc_prox_log", "orc_prox_linear", "orc_prox_alpha2"):
            f = getattr(lib, name)
            f.restype = ctypes.c_double
            f.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.orc_prox_slack.restype = ctypes.c_double
        lib.orc_prox_slack.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def prox_log(S, L, w, rho, lo=0.0, hi=math.inf):
    return _load().orc_prox_log(S, L, w, rho, lo, hi)


def prox_linear(S, L, w, rho, lo=0.0, hi=math.inf):
    return _load().orc_prox_linear(S, L, w, rho, lo, hi)


def prox_alpha2(S, L, w, rho, lo=0.0, hi=math.inf):
    return _load().orc_prox_alpha2(S, L, w, rho, lo, hi)


def prox_slack(zeta, c):
    return _load().orc_prox_slack(zeta, c)


def run(inst, iters, rho0=1.0, alpha=1.6, mu=2.0, gamma=1.1, eps_abs=1e-4,
        adapt_every=50, check_every=10, stop=False, threads=0, history=False,
        branches=False, state=None, keep_state=False):
    """Run the literal PMP on `inst` for `iters` iterations (or until the stop
    rule fires, when `stop`).  Returns a dict with x, lam (= rho u), slack,
    iterations, r_norm, s_norm, eps_tol, rho, converged, zsum_worst, with
    `history` per-iteration hist_r / hist_s / hist_rho and the norms
    hist_pnorm / hist_znorm / hist_unorm of p, z and rho u, and with
    `branches` the digest of every prox branch taken (clip of each rate,
    slack projection of each link) over the run.  `state` (from an earlier
    run with keep_state=True, same R) starts from that iterate and its rho:
    a warm start; keep_state=True returns the final iterate as "state"."""
    lib = _load()
    row_ptr = np.ascontiguousarray(inst.row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(inst.col_idx, dtype=np.int32)
    c = np.ascontiguousarray(inst.c, dtype=np.float64)
    w = np.ascontiguousarray(inst.w, dtype=np.float64)
    util = np.ascontiguousarray(inst.utility, dtype=np.uint8)
    prob = _Problem(inst.m, inst.n, int(row_ptr[-1]), _ptr(row_ptr), _ptr(col_idx),
                    _ptr(c), _ptr(w), _ptr(util), float(inst.lo), float(inst.hi))
    prm = _Params(rho0, alpha, mu, gamma, eps_abs, adapt_every, check_every,
                  int(iters), int(bool(stop)), int(threads))
    J = int(row_ptr[-1]) + inst.m
    st_in = None
    if state is not None:
        st_in = np.ascontiguousarray(state, dtype=np.float64)
        if st_in.size != 3 * J + inst.m + 1:
            raise ValueError("state does not match this pattern")
    st_out = np.zeros(3 * J + inst.m + 1) if keep_state else None
    x = np.zeros(inst.n)
    lam = np.zeros(inst.m)
    slack = np.zeros(inst.m)
    hr = hs = hrho = hpn = hzn = hun = None
    if history:
        hr, hs, hrho, hpn, hzn, hun = (np.zeros(max(1, iters)) for _ in range(6))
    zw = ctypes.c_double(0.0)
    dig = ctypes.c_uint64(0)
    secs = ctypes.c_double(0.0)
    nthr = ctypes.c_int32(0)
    res = _Result()
    vp = lambda o: ctypes.cast(ctypes.byref(o), ctypes.c_void_p)
    rc = lib.orc_run(ctypes.byref(prob), ctypes.byref(prm), _ptr(x), _ptr(lam),
                     _ptr(slack), _ptr(hr), _ptr(hs), _ptr(hrho), _ptr(hpn), _ptr(hzn),
                     _ptr(hun), vp(zw), vp(secs),
                     vp(nthr), vp(dig) if branches else None, _ptr(st_in), _ptr(st_out),
                     ctypes.byref(res))
    if rc != 0:
        raise RuntimeError(f"orc_run failed with code {rc}")
    out = {"x": x, "lam": lam, "slack": slack, "iterations": int(res.iterations),
           "r_norm": res.r_norm, "s_norm": res.s_norm, "eps_tol": res.eps_tol,
           "rho": res.rho, "converged": bool(res.converged), "zsum_worst": zw.value,
           "loop_seconds": secs.value, "threads": int(nthr.value)}
    if branches:
        out["branch_digest"] = int(dig.value)
    if keep_state:
        out["state"] = st_out
    if history:
        k = int(res.iterations)
        out.update(hist_r=hr[:k], hist_s=hs[:k], hist_rho=hrho[:k], hist_pnorm=hpn[:k],
                   hist_znorm=hzn[:k], hist_unorm=hun[:k])
    return out
