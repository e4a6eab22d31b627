"""Python binding of the PMP C ABI (include/pmp.h).

Argument marshalling only: every step of the solver runs in libpmp.so's HIP
kernels.  PyTorch supplies device memory (the workspace and the problem
arrays) and the stream.  The functions keep the C names; `Solver` bundles
them for one instance.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PMP_OK, PMP_ERR_INVALID, PMP_ERR_SHAPE, PMP_ERR_NOMEM, PMP_ERR_HIP, PMP_ERR_NUMERIC, \
    PMP_NOT_CONVERGED, PMP_ERR_STATE = range(8)
PMP_F32, PMP_F64 = 0, 1
PMP_MEM_HOST, PMP_MEM_DEVICE = 0, 1
PMP_LAYOUT_AUTO, PMP_LAYOUT_GATHER, PMP_LAYOUT_BINNED = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpmp.so")
_lib = None


class PMPError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


class pmp_problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("utility", ctypes.c_void_p), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("dtype", ctypes.c_int), ("memory", ctypes.c_int)]


class pmp_params(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("alpha", ctypes.c_double),
                ("mu", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eps_abs", ctypes.c_double), ("adapt_every", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("eps_rel", ctypes.c_double)]


class pmp_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("r_norm", ctypes.c_double),
                ("s_norm", ctypes.c_double), ("eps_tol", ctypes.c_double),
                ("rho", ctypes.c_double), ("status", ctypes.c_int)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "pmp_params_default": [ctypes.POINTER(pmp_params)],
    "pmp_workspace_size": [ctypes.POINTER(pmp_problem), ctypes.POINTER(pmp_params),
                           ctypes.POINTER(ctypes.c_size_t)],
    "pmp_setup": [ctypes.POINTER(pmp_problem), ctypes.POINTER(pmp_params), _P,
                  ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "pmp_iterate": [_P, ctypes.c_int32],
    "pmp_residuals": [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                      ctypes.POINTER(ctypes.c_int64)],
    "pmp_solve": [_P, ctypes.POINTER(pmp_result)],
    "pmp_get_solution": [_P, _P, _P, _P],
    "pmp_state_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "pmp_get_state": [_P, _P],
    "pmp_set_state": [_P, _P],
    "pmp_update_capacity": [_P, _P],
    "pmp_device_views": [_P] + [ctypes.POINTER(_P)] * 6,
    "pmp_update_params": [_P, ctypes.POINTER(pmp_params)],
    "pmp_history": [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "pmp_time_kernels": [_P, ctypes.c_int32, _P],
    "pmp_update_weights": [_P, _P],
    "pmp_adjoint_workspace_size": [_P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_size_t)],
    "pmp_forward_ckpt": [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t,
                         ctypes.POINTER(ctypes.c_double)],
    "pmp_backward": [_P, _P, _P],
    "pmp_get_layout": [_P, ctypes.POINTER(ctypes.c_int32)],
    "pmp_get_path_prices": [_P, _P],
    "pmp_prune_workspace_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "pmp_prune": [_P, _P, _P, ctypes.c_size_t, _P, _P, _P, _P, _P, _P, _P, _P,
                  ctypes.POINTER(ctypes.c_int64)],
    "pmp_prune_noalloc": [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                          ctypes.POINTER(ctypes.c_int64)],
    "pmp_destroy": [_P],
}


def exported_symbols():
    """Names the C ABI exports (include/pmp.h)."""
    return sorted(list(_SIGNATURES) + ["pmp_status_string", "pmp_last_error"])


def load_library(require_torch: bool = True):
    """Load libpmp.so.  torch is imported first so that the library binds to
    the HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    if require_torch:
        import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.pmp_status_string.argtypes = [ctypes.c_int]
    lib.pmp_status_string.restype = ctypes.c_char_p
    lib.pmp_last_error.argtypes = []
    lib.pmp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, where, allow=(PMP_OK,)):
    if status not in allow:
        lib = load_library()
        raise PMPError(status, where, lib.pmp_last_error().decode())
    return status


def params_default(**overrides) -> pmp_params:
    p = pmp_params()
    _check(load_library().pmp_params_default(ctypes.byref(p)), "pmp_params_default")
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _device_array(torch, a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(dtype=dtype, device=device).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device=device)


class PrunedInstance:
    """A problem whose arrays are device tensors (the output of pruning)."""

    def __init__(self, m, n, row_ptr, col_idx, c, w, utility, lo, hi):
        self.m, self.n = m, n
        self.row_ptr, self.col_idx = row_ptr, col_idx
        self.c, self.w, self.utility = c, w, utility
        self.lo, self.hi = lo, hi
        self.nnz = int(col_idx.numel())


class Solver:
    """One NUM instance resident on the GPU.

    `inst` has m, n, row_ptr, col_idx (int32 CSR of R), c, w, utility, lo,
    hi (see paper_2509_10722_amd.instances.Instance).  dtype is torch.float32
    or torch.float64.  With memory="device" the arrays are first placed in
    device tensors (the boundary then reads device memory); with "host" the
    library copies them from host memory.
    """

    def __init__(self, inst, dtype=None, params=None, device="cuda", memory="device", **kw):
        import torch
        lib = load_library()
        self.torch = torch
        self.dtype = dtype or torch.float32
        self.device = torch.device(device)
        self.m, self.n = int(inst.m), int(inst.n)
        self.nnz = int(inst.row_ptr[-1])
        self.lo, self.hi = float(inst.lo), float(inst.hi)
        npdt = np.float32 if self.dtype == torch.float32 else np.float64
        self.params = params or params_default(**kw)
        dt = PMP_F32 if self.dtype == torch.float32 else PMP_F64
        if memory == "device":
            arrs = [_device_array(torch, inst.row_ptr, torch.int32, self.device),
                    _device_array(torch, inst.col_idx, torch.int32, self.device),
                    _device_array(torch, inst.c, self.dtype, self.device),
                    _device_array(torch, inst.w, self.dtype, self.device),
                    _device_array(torch, inst.utility, torch.uint8, self.device)]
            ptrs = [a.data_ptr() for a in arrs]
            mem = PMP_MEM_DEVICE
        else:
            arrs = [np.ascontiguousarray(inst.row_ptr, dtype=np.int32),
                    np.ascontiguousarray(inst.col_idx, dtype=np.int32),
                    np.ascontiguousarray(inst.c, dtype=npdt),
                    np.ascontiguousarray(inst.w, dtype=npdt),
                    np.ascontiguousarray(inst.utility, dtype=np.uint8)]
            ptrs = [a.ctypes.data for a in arrs]
            mem = PMP_MEM_HOST
        self.problem = pmp_problem(self.m, self.n, self.nnz, *ptrs, float(inst.lo),
                                   float(inst.hi), dt, mem)
        nbytes = ctypes.c_size_t()
        _check(lib.pmp_workspace_size(ctypes.byref(self.problem), ctypes.byref(self.params),
                                      ctypes.byref(nbytes)), "pmp_workspace_size")
        self.workspace = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.pmp_setup(ctypes.byref(self.problem), ctypes.byref(self.params),
                             self.workspace.data_ptr(), nbytes.value, self.stream.cuda_stream,
                             ctypes.byref(h)), "pmp_setup")
        self.handle = h
        del arrs
        self.lib = lib

    # -- C calls -----------------------------------------------------------
    def iterate(self, k: int):
        _check(self.lib.pmp_iterate(self.handle, int(k)), "pmp_iterate")

    def residuals(self):
        r, s, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.pmp_residuals(self.handle, ctypes.byref(r), ctypes.byref(s),
                                      ctypes.byref(it)), "pmp_residuals")
        return r.value, s.value, it.value

    def solve(self):
        res = pmp_result()
        st = self.lib.pmp_solve(self.handle, ctypes.byref(res))
        _check(st, "pmp_solve", allow=(PMP_OK, PMP_NOT_CONVERGED))
        return {"iterations": res.iterations, "r_norm": res.r_norm, "s_norm": res.s_norm,
                "eps_tol": res.eps_tol, "rho": res.rho, "converged": st == PMP_OK}

    def solution(self):
        t = self.torch
        x = t.empty(self.n, dtype=self.dtype, device=self.device)
        lam = t.empty(self.m, dtype=self.dtype, device=self.device)
        slack = t.empty(self.m, dtype=self.dtype, device=self.device)
        _check(self.lib.pmp_get_solution(self.handle, x.data_ptr() if self.n else None,
                                         lam.data_ptr(), slack.data_ptr()), "pmp_get_solution")
        return x, lam, slack

    def state_size(self):
        b = ctypes.c_size_t()
        _check(self.lib.pmp_state_size(self.handle, ctypes.byref(b)), "pmp_state_size")
        return b.value

    def get_state(self):
        buf = self.torch.empty(self.state_size(), dtype=self.torch.uint8, device=self.device)
        _check(self.lib.pmp_get_state(self.handle, buf.data_ptr()), "pmp_get_state")
        return buf

    def set_state(self, buf):
        _check(self.lib.pmp_set_state(self.handle, buf.data_ptr()), "pmp_set_state")

    def update_capacity(self, c_new):
        c = self.torch.as_tensor(c_new).to(dtype=self.dtype, device=self.device).contiguous()
        _check(self.lib.pmp_update_capacity(self.handle, c.data_ptr()), "pmp_update_capacity")

    def path_prices(self):
        """pi[n] = sum of the link prices rho u along each route (Section VI-B)."""
        pi = self.torch.empty(max(1, self.n), dtype=self.dtype, device=self.device)
        _check(self.lib.pmp_get_path_prices(self.handle, pi.data_ptr()), "pmp_get_path_prices")
        return pi[:self.n]

    def prune(self, failed, params=None, noalloc=False):
        """Link failure (Section V-D): drop the links flagged in failed[m] and
        every stream routed over one of them, on the device.  Returns
        (solver of the pruned instance warm-started from this iterate,
        link_map, stream_map) with the maps giving old indices; the pruned
        problem's device arrays are kept as `solver.instance`.  With
        noalloc=True the compaction runs through pmp_prune_noalloc (its
        scratch in the library's fixed array instead of a workspace)."""
        t = self.torch
        f = t.as_tensor(failed).to(dtype=t.uint8, device=self.device).contiguous()
        if f.numel() != self.m:
            raise ValueError(f"failed must have m = {self.m} entries")
        if not noalloc:
            nb = ctypes.c_size_t()
            _check(self.lib.pmp_prune_workspace_size(self.handle, ctypes.byref(nb)),
                   "pmp_prune_workspace_size")
            ws = t.empty(max(1, nb.value), dtype=t.uint8, device=self.device)
        i32 = dict(dtype=t.int32, device=self.device)
        row_ptr = t.empty(self.m + 1, **i32)
        col_idx = t.empty(max(1, self.nnz), **i32)
        c = t.empty(self.m, dtype=self.dtype, device=self.device)
        w = t.empty(max(1, self.n), dtype=self.dtype, device=self.device)
        util = t.empty(max(1, self.n), dtype=t.uint8, device=self.device)
        link_map = t.empty(self.m, **i32)
        stream_map = t.empty(max(1, self.n), **i32)
        state = t.empty(self.state_size(), dtype=t.uint8, device=self.device)
        sizes = (ctypes.c_int64 * 3)()
        outs = (row_ptr.data_ptr(), col_idx.data_ptr(), c.data_ptr(), w.data_ptr(),
                util.data_ptr(), link_map.data_ptr(), stream_map.data_ptr(), state.data_ptr(),
                sizes)
        if noalloc:
            _check(self.lib.pmp_prune_noalloc(self.handle, f.data_ptr(), *outs),
                   "pmp_prune_noalloc")
        else:
            _check(self.lib.pmp_prune(self.handle, f.data_ptr(), ws.data_ptr(), nb.value, *outs),
                   "pmp_prune")
        m2, n2, nnz2 = (int(v) for v in sizes)
        pruned = PrunedInstance(m2, n2, row_ptr[:m2 + 1], col_idx[:nnz2], c[:m2], w[:n2],
                                util[:n2], self.lo, self.hi)
        solver = Solver(pruned, dtype=self.dtype, params=params or self.params,
                        device=self.device)
        solver.instance = pruned
        solver.set_state(state)
        return solver, link_map[:m2], stream_map[:n2]

    def update_params(self, **kw):
        for k, v in kw.items():
            setattr(self.params, k, v)
        _check(self.lib.pmp_update_params(self.handle, ctypes.byref(self.params)),
               "pmp_update_params")

    def history(self, capacity=4096):
        out = np.zeros((capacity, 4))
        cnt = ctypes.c_int32()
        _check(self.lib.pmp_history(self.handle, out.ctypes.data, capacity, ctypes.byref(cnt)),
               "pmp_history")
        return out[: cnt.value]

    def time_kernels(self, k):
        ms = np.zeros(4)
        _check(self.lib.pmp_time_kernels(self.handle, int(k), ms.ctypes.data), "pmp_time_kernels")
        return {"stream": ms[0], "link": ms[1], "stream_check": ms[2], "link_check": ms[3]}

    def reset(self):
        """Back to the all-zero start with rho = rho0 (a fresh solve)."""
        buf = self.torch.zeros(self.state_size(), dtype=self.torch.uint8, device=self.device)
        tail = np.zeros(2, dtype=np.float64)
        tail[0] = self.params.rho0
        buf[-16:-8] = self.torch.from_numpy(tail[:1].view(np.uint8).copy()).to(self.device)
        self.set_state(buf)

    def update_weights(self, w_new):
        w = self.torch.as_tensor(w_new).to(dtype=self.dtype, device=self.device).contiguous()
        _check(self.lib.pmp_update_weights(self.handle, w.data_ptr()), "pmp_update_weights")

    def forward_ckpt(self, K, s):
        """K iterations from the current state with checkpoints every s;
        returns J = sum_j U_j(x_j^K)."""
        b = ctypes.c_size_t()
        _check(self.lib.pmp_adjoint_workspace_size(self.handle, int(K), int(s), ctypes.byref(b)),
               "pmp_adjoint_workspace_size")
        self.adj_ws = self.torch.empty(b.value, dtype=self.torch.uint8, device=self.device)
        J = ctypes.c_double()
        _check(self.lib.pmp_forward_ckpt(self.handle, int(K), int(s), self.adj_ws.data_ptr(),
                                         b.value, ctypes.byref(J)), "pmp_forward_ckpt")
        return J.value

    def backward(self):
        """(dJ/dc, dJ/dw) of the last forward_ckpt."""
        gc = self.torch.empty(self.m, dtype=self.dtype, device=self.device)
        gw = self.torch.empty(max(self.n, 1), dtype=self.dtype, device=self.device)
        _check(self.lib.pmp_backward(self.handle, gc.data_ptr(), gw.data_ptr()), "pmp_backward")
        return gc, gw[: self.n]

    def layout_in_use(self):
        """'binned' or 'gather': the layout the library chose at setup."""
        v = ctypes.c_int32()
        _check(self.lib.pmp_get_layout(self.handle, ctypes.byref(v)), "pmp_get_layout")
        return "binned" if v.value == PMP_LAYOUT_BINNED else "gather"

    def views(self):
        """Zero-copy tensors over the internal x, u, a, b, zs, v."""
        ptrs = [ctypes.c_void_p() for _ in range(6)]
        _check(self.lib.pmp_device_views(self.handle, *[ctypes.byref(p) for p in ptrs]),
               "pmp_device_views")
        sizes = [self.n, self.m, self.n, self.m, self.m, self.m]
        names = ["x", "u", "a", "b", "zs", "v"]
        out = {}
        esz = 4 if self.dtype == self.torch.float32 else 8
        for nm, p, sz in zip(names, ptrs, sizes):
            out[nm] = _tensor_from_ptr(self.torch, p.value, sz, self.dtype, self.device,
                                       self.workspace, esz)
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pmp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tensor_from_ptr(torch, ptr, count, dtype, device, workspace, esz):
    """View `count` elements at device address `ptr` inside `workspace`."""
    base = workspace.data_ptr()
    off = ptr - base
    if off < 0 or off + count * esz > workspace.numel():
        raise ValueError("pointer outside the workspace")
    return workspace[off: off + count * esz].view(dtype)


def _autograd_function():
    import torch

    class PMPFunction(torch.autograd.Function):
        """J(c, w) = sum_j U_j(x_j^K) after K PMP iterations from the all-zero
        start, with a hand-written reverse pass (pmp_backward) behind autograd.
        Inputs c [m] and w [n] are device tensors of the solver's dtype."""

        @staticmethod
        def forward(ctx, c, w, solver, K, s):
            solver.update_capacity(c.detach())
            solver.update_weights(w.detach())
            solver.reset()
            J = solver.forward_ckpt(K, s)
            ctx.solver = solver
            return torch.tensor(J, dtype=torch.float64, device=c.device)

        @staticmethod
        def backward(ctx, gJ):
            gc, gw = ctx.solver.backward()
            g = gJ.to(gc.dtype)
            return g * gc, g * gw, None, None, None

    return PMPFunction


_PMPFunction = None


def pmp_objective(c, w, solver, K, s=25):
    """Differentiable J(c, w) (see PMPFunction)."""
    global _PMPFunction
    if _PMPFunction is None:
        _PMPFunction = _autograd_function()
    return _PMPFunction.apply(c, w, solver, K, s)


class pmp_batch_options(ctypes.Structure):
    _fields_ = [("class_m", ctypes.c_int32 * 2), ("tile_cap", ctypes.c_int32 * 3),
                ("reorder_streams", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("heavy_chunk", ctypes.c_int32),
                ("wait_log2", ctypes.c_int32)]


_BATCH_SIGNATURES = {
    "pmp_batch_options_default": [ctypes.POINTER(pmp_batch_options)],
    "pmp_batch_workspace_size": [ctypes.c_int32, ctypes.POINTER(pmp_problem),
                                 ctypes.POINTER(pmp_params), ctypes.POINTER(pmp_batch_options),
                                 ctypes.POINTER(ctypes.c_size_t)],
    "pmp_batch_setup": [ctypes.c_int32, ctypes.POINTER(pmp_problem), ctypes.POINTER(pmp_params),
                        ctypes.POINTER(pmp_batch_options), _P, ctypes.c_size_t, _P,
                        ctypes.POINTER(_P)],
    "pmp_batch_solve": [_P, ctypes.c_int32, ctypes.POINTER(pmp_result)],
    "pmp_batch_get_solution": [_P, ctypes.c_int32, _P, _P, _P],
    "pmp_batch_reset": [_P],
    "pmp_batch_profile": [_P, _P],
    "pmp_batch_destroy": [_P],
}
_SIGNATURES.update(_BATCH_SIGNATURES)


def batch_options_default(**caps) -> pmp_batch_options:
    o = pmp_batch_options()
    _check(load_library().pmp_batch_options_default(ctypes.byref(o)), "pmp_batch_options_default")
    if "tile_cap" in caps:
        for i, v in enumerate(caps["tile_cap"]):
            o.tile_cap[i] = int(v)
    if "class_m" in caps:
        for i, v in enumerate(caps["class_m"]):
            o.class_m[i] = int(v)
    if "reorder_streams" in caps:
        o.reorder_streams = int(caps["reorder_streams"])
    for key in ("wg_per_cu", "profile", "heavy_chunk", "wait_log2"):
        if key in caps:
            setattr(o, key, int(caps[key]))
    return o


class BatchSolver:
    """Many instances solved together by one persistent kernel launch per
    solve (pmp_batch_*).  Instances are host-resident Instance objects."""

    def __init__(self, insts, dtype=None, params=None, options=None, device="cuda", **kw):
        import torch
        lib = load_library()
        self.torch = torch
        self.lib = lib
        self.dtype = dtype or torch.float32
        self.device = torch.device(device)
        npdt = np.float32 if self.dtype == torch.float32 else np.float64
        dt = PMP_F32 if self.dtype == torch.float32 else PMP_F64
        self.params = params or params_default(**kw)
        self.options = options or batch_options_default()
        self.count = len(insts)
        self.sizes = [(int(i.m), int(i.n)) for i in insts]
        keep = []
        probs = (pmp_problem * self.count)()
        for k, inst in enumerate(insts):
            arrs = [np.ascontiguousarray(inst.row_ptr, dtype=np.int32),
                    np.ascontiguousarray(inst.col_idx, dtype=np.int32),
                    np.ascontiguousarray(inst.c, dtype=npdt),
                    np.ascontiguousarray(inst.w, dtype=npdt),
                    np.ascontiguousarray(inst.utility, dtype=np.uint8)]
            keep.append(arrs)
            probs[k] = pmp_problem(int(inst.m), int(inst.n), int(inst.row_ptr[-1]),
                                   *[a.ctypes.data for a in arrs], float(inst.lo), float(inst.hi),
                                   dt, PMP_MEM_HOST)
        nbytes = ctypes.c_size_t()
        _check(lib.pmp_batch_workspace_size(self.count, probs, ctypes.byref(self.params),
                                            ctypes.byref(self.options), ctypes.byref(nbytes)),
               "pmp_batch_workspace_size")
        self.workspace = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.pmp_batch_setup(self.count, probs, ctypes.byref(self.params),
                                   ctypes.byref(self.options), self.workspace.data_ptr(),
                                   nbytes.value, self.stream.cuda_stream, ctypes.byref(h)),
               "pmp_batch_setup")
        self.handle = h
        del keep

    def solve(self, max_iter):
        res = (pmp_result * self.count)()
        st = self.lib.pmp_batch_solve(self.handle, int(max_iter), res)
        _check(st, "pmp_batch_solve", allow=(PMP_OK, PMP_NOT_CONVERGED))
        return [{"iterations": r.iterations, "r_norm": r.r_norm, "s_norm": r.s_norm,
                 "eps_tol": r.eps_tol, "rho": r.rho, "converged": r.status == PMP_OK}
                for r in res]

    def solution(self, k):
        m, n = self.sizes[k]
        t = self.torch
        x = t.empty(max(n, 1), dtype=self.dtype, device=self.device)
        lam = t.empty(m, dtype=self.dtype, device=self.device)
        slack = t.empty(m, dtype=self.dtype, device=self.device)
        _check(self.lib.pmp_batch_get_solution(self.handle, int(k), x.data_ptr(), lam.data_ptr(),
                                               slack.data_ptr()), "pmp_batch_get_solution")
        return x[:n], lam, slack

    def profile(self):
        """Per-phase times (ms, averaged over workgroups) of the last solve's
        kernel; needs options.profile = 1."""
        ms = np.zeros(6)
        _check(self.lib.pmp_batch_profile(self.handle, ms.ctypes.data), "pmp_batch_profile")
        return dict(zip(("stream_tiles", "stream_barrier", "link_tiles", "link_barrier",
                         "finalize", "rescale"), ms.tolist()))

    def reset(self):
        _check(self.lib.pmp_batch_reset(self.handle), "pmp_batch_reset")

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pmp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
