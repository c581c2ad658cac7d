"""Thin ctypes binding of libdpgmi.so (include/dpg.h).

Argument marshalling only: every step of the local solve runs in the HIP
library.  torch is used for device memory and streams.  Loading fails loudly
when the library has not been built (``python -m paper_2609_03155_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpgmi.so")

DPG_OK, DPG_ERR_ARG, DPG_ERR_ALLOC, DPG_ERR_HIP, DPG_ERR_UNSUPPORTED, DPG_ERR_CELL = 0, -1, -2, -3, -4, -5
DPG_FP64, DPG_SPLIT_FP32 = 0, 1
FACE_INTERIOR, FACE_PEC, FACE_PORT, FACE_ROBIN0 = 0, 1, 2, 3

EXPORTS = ("dpg_local_dims", "dpg_plan_create", "dpg_plan_destroy", "dpg_plan_offsets", "dpg_plan_layout",
           "dpg_local_solve", "dpg_local_solve_range", "dpg_plan_set_concurrency", "dpg_plan_autotune",
           "dpg_plan_tuning", "dpg_plan_tiles", "dpg_plan_set_tiles", "dpg_graph_create", "dpg_graph_launch", "dpg_graph_destroy", "dpg_form_local",
           "dpg_form_augmented",
           "dpg_plan_trace_offsets", "dpg_condense", "dpg_trace_numbering", "dpg_trace_system_create",
           "dpg_trace_system_destroy", "dpg_trace_system_info", "dpg_trace_system_numbering", "dpg_trace_system_csr",
           "dpg_assemble", "dpg_csr_matvec", "dpg_cg_solve", "dpg_trace_system_cg", "dpg_trace_system_scatter",
           "dpg_reconstruct", "dpg_dorfler_mark_workspace_size", "dpg_dorfler_mark", "dpg_dorfler_mark_noalloc", "dpg_power_dissipation",
           "dpg_plan_set_profiling", "dpg_plan_profile", "dpg_sync", "dpg_status_string", "dpg_last_error")
KERNEL_CLASSES = ("scale", "form_SM", "form_IF", "form_pad", "form_B", "form_load", "resid", "chol_diag",
                  "chol_panel", "herk")


class dpg_port(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("m", C.c_int32), ("n", C.c_int32),
                ("eps_re", C.c_double), ("eps_im", C.c_double), ("mu_re", C.c_double), ("mu_im", C.c_double)]


class dpg_problem(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_vertices", C.c_int64), ("vertices", C.c_void_p),
                ("cells", C.c_void_p), ("eps", C.c_void_p), ("mu", C.c_void_p), ("face_kind", C.c_void_p),
                ("zinv", C.c_void_p), ("freq_hz", C.c_double), ("length_m", C.c_double), ("alpha", C.c_double),
                ("port", dpg_port)]


class DPGError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DPGError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_03155_amd.build`")
        L = C.CDLL(LIB_PATH)
        i32, i64, vp, dp_ = C.c_int32, C.c_int64, C.c_void_p, C.c_double
        L.dpg_local_dims.argtypes = [i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.dpg_plan_create.argtypes = [i32, vp, i64, i32, i64, C.POINTER(vp)]
        L.dpg_plan_destroy.argtypes = [vp]
        L.dpg_plan_offsets.argtypes = [vp, vp, vp]
        L.dpg_plan_layout.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.dpg_local_solve.argtypes = [vp, C.POINTER(dpg_problem), vp, vp, vp, vp, vp, i32, vp]
        L.dpg_local_solve_range.argtypes = [vp, C.POINTER(dpg_problem), i64, i64, vp, vp, vp, vp, vp, i32, vp]
        L.dpg_plan_set_concurrency.argtypes = [vp, i32]
        L.dpg_plan_autotune.argtypes = [vp, C.POINTER(dpg_problem), vp, vp, vp, vp, vp, i32, vp, C.POINTER(dp_)]
        L.dpg_plan_tuning.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i32)]
        L.dpg_plan_tiles.argtypes = [vp, i32, C.POINTER(i32)]
        L.dpg_plan_set_tiles.argtypes = [vp, i32, i32]
        L.dpg_graph_create.argtypes = [vp, C.POINTER(dpg_problem), i64, i64, vp, vp, vp, vp, vp, i32, C.POINTER(vp)]
        L.dpg_graph_launch.argtypes = [vp, vp]
        L.dpg_graph_destroy.argtypes = [vp]
        L.dpg_form_local.argtypes = [vp, C.POINTER(dpg_problem), i64, i64, vp, vp, vp, vp, vp]
        L.dpg_form_augmented.argtypes = [vp, C.POINTER(dpg_problem), i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.dpg_plan_trace_offsets.argtypes = [vp, vp, vp]
        L.dpg_condense.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.dpg_trace_numbering.argtypes = [vp, vp, vp, i64, vp, C.POINTER(i64)]
        L.dpg_trace_system_create.argtypes = [vp, vp, vp, C.POINTER(vp)]
        L.dpg_trace_system_destroy.argtypes = [vp]
        L.dpg_trace_system_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.dpg_trace_system_numbering.argtypes = [vp, vp]
        L.dpg_trace_system_csr.argtypes = [vp, C.POINTER(vp), C.POINTER(vp)]
        L.dpg_assemble.argtypes = [vp, vp, vp, vp, vp, vp]
        L.dpg_csr_matvec.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        L.dpg_cg_solve.argtypes = [i64, vp, vp, vp, vp, vp, dp_, i64, C.POINTER(i64), C.POINTER(dp_), vp]
        L.dpg_trace_system_cg.argtypes = [vp, vp, vp, vp, dp_, i64, C.POINTER(i64), C.POINTER(dp_), vp]
        L.dpg_trace_system_scatter.argtypes = [vp, vp, vp, vp]
        L.dpg_reconstruct.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.dpg_dorfler_mark_workspace_size.argtypes = [i64, C.POINTER(C.c_size_t)]
        L.dpg_dorfler_mark.argtypes = [i64, vp, dp_, dp_, vp, vp, C.c_size_t, vp]
        L.dpg_dorfler_mark_noalloc.argtypes = [i64, vp, dp_, dp_, vp, vp]
        L.dpg_power_dissipation.argtypes = [vp, C.POINTER(dpg_problem), vp, vp, vp]
        L.dpg_plan_set_profiling.argtypes = [vp, i32]
        L.dpg_plan_profile.argtypes = [vp, vp, vp]
        L.dpg_sync.argtypes = [vp, vp, i64, C.POINTER(i64), C.POINTER(i64)]
        L.dpg_status_string.argtypes = [i32]
        L.dpg_status_string.restype = C.c_char_p
        L.dpg_last_error.argtypes = []
        L.dpg_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("dpg_status_string", "dpg_last_error"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != DPG_OK:
        msg = f"{what}: {lib().dpg_status_string(rc).decode()} ({rc})"
        if rc == DPG_ERR_HIP:
            msg += f" [{lib().dpg_last_error().decode()}]"
        raise DPGError(msg)


def dpg_local_dims(p: int, dp: int):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().dpg_local_dims(p, dp, C.byref(a), C.byref(b), C.byref(c)), "dpg_local_dims")
    return a.value, b.value, c.value


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


@dataclass
class DeviceProblem:
    """Device-resident problem arrays (torch CUDA tensors) and scalars."""
    vertices: "object"
    cells: "object"
    eps: "object"        # complex128 [n]
    mu: "object"         # complex128 [n]
    face_kind: "object"  # int8 [n,6]
    zinv: "object"       # complex128 [n,6]
    freq_hz: float
    port: dict
    length_m: float = 1.0
    alpha: float = 1.0

    @staticmethod
    def from_workload(w, device="cuda:0") -> "DeviceProblem":
        import torch
        dev = torch.device(device)
        return DeviceProblem(
            vertices=torch.from_numpy(np.ascontiguousarray(w.vertices, np.float64)).to(dev),
            cells=torch.from_numpy(np.ascontiguousarray(w.cells, np.int64)).to(dev),
            eps=torch.from_numpy(np.ascontiguousarray(w.eps, np.complex128)).to(dev),
            mu=torch.from_numpy(np.ascontiguousarray(w.mu, np.complex128)).to(dev),
            face_kind=torch.from_numpy(np.ascontiguousarray(w.face_kind, np.int8)).to(dev),
            zinv=torch.from_numpy(np.ascontiguousarray(w.zinv, np.complex128)).to(dev),
            freq_hz=float(w.freq_hz), port=dict(w.port))

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    def cstruct(self) -> dpg_problem:
        p = self.port
        eps, mu = complex(p.get("eps", 1.0)), complex(p.get("mu", 1.0))
        port = dpg_port(float(p["a"]), float(p["b"]), int(p["m"]), int(p["n"]), eps.real, eps.imag, mu.real,
                        mu.imag)
        return dpg_problem(self.n_cells, int(self.vertices.shape[0]), _ptr(self.vertices), _ptr(self.cells),
                           _ptr(self.eps), _ptr(self.mu), _ptr(self.face_kind), _ptr(self.zinv),
                           float(self.freq_hz), float(self.length_m), float(self.alpha), port)


class Plan:
    """dpg_plan_create / dpg_plan_destroy with the plan's output offsets."""

    def __init__(self, degree, dp: int, device: int = 0, max_workspace_bytes: int = 0):
        deg = np.ascontiguousarray(np.asarray(degree, dtype=np.int8))
        self.n_cells = int(deg.shape[0])
        self.dp = int(dp)
        self.degree = deg
        h = C.c_void_p()
        _check(lib().dpg_plan_create(int(device), deg.ctypes.data, self.n_cells, self.dp,
                                     int(max_workspace_bytes), C.byref(h)), "dpg_plan_create")
        self._h = h
        self.K_off = np.zeros(self.n_cells + 1, np.int64)
        self.v_off = np.zeros(self.n_cells + 1, np.int64)
        _check(lib().dpg_plan_offsets(self._h, self.K_off.ctypes.data, self.v_off.ctypes.data), "dpg_plan_offsets")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dpg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self, p: int):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().dpg_plan_layout(self._h, int(p), C.byref(a), C.byref(b), C.byref(c)), "dpg_plan_layout")
        return a.value, b.value, c.value

    def set_profiling(self, enable: bool):
        _check(lib().dpg_plan_set_profiling(self._h, int(bool(enable))), "dpg_plan_set_profiling")

    def profile(self):
        """{kernel class: (total ms, launches)} since the previous call."""
        ms = np.zeros(len(KERNEL_CLASSES), np.float64)
        n = np.zeros(len(KERNEL_CLASSES), np.int64)
        _check(lib().dpg_plan_profile(self._h, ms.ctypes.data, n.ctypes.data), "dpg_plan_profile")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def alloc_outputs(self, device="cuda:0"):
        import torch
        dev = torch.device(device)
        K = torch.empty(int(self.K_off[-1]), dtype=torch.complex128, device=dev)
        l = torch.empty(int(self.v_off[-1]), dtype=torch.complex128, device=dev)
        eta = torch.empty(self.n_cells, dtype=torch.float64, device=dev)
        info = torch.empty(self.n_cells, dtype=torch.int32, device=dev)
        return K, l, eta, info

    def local_solve(self, prob: DeviceProblem, x, K, l, eta, info, precision: int = DPG_FP64, stream=None):
        """dpg_local_solve: enqueue the local solve of every cell on `stream`."""
        s = prob.cstruct()
        _check(lib().dpg_local_solve(self._h, C.byref(s), _ptr(x), _ptr(K), _ptr(l), _ptr(eta), _ptr(info),
                                     int(precision), _stream(stream)), "dpg_local_solve")

    def local_solve_range(self, prob: DeviceProblem, first: int, count: int, x, K, l, eta, info,
                          precision: int = DPG_FP64, stream=None):
        """dpg_local_solve_range: cells first..first+count-1, outputs relative to the range."""
        s = prob.cstruct()
        _check(lib().dpg_local_solve_range(self._h, C.byref(s), int(first), int(count), _ptr(x), _ptr(K), _ptr(l),
                                           _ptr(eta), _ptr(info), int(precision), _stream(stream)),
               "dpg_local_solve_range")

    def set_concurrency(self, enable: bool):
        _check(lib().dpg_plan_set_concurrency(self._h, int(bool(enable))), "dpg_plan_set_concurrency")

    def autotune(self, prob: DeviceProblem, x, K, l, eta, info, precision: int = DPG_FP64, stream=None) -> float:
        """dpg_plan_autotune: returns the time (ms) of a solve with the chosen batching."""
        s = prob.cstruct()
        ms = C.c_double()
        _check(lib().dpg_plan_autotune(self._h, C.byref(s), _ptr(x), _ptr(K), _ptr(l), _ptr(eta), _ptr(info),
                                       int(precision), _stream(stream), C.byref(ms)), "dpg_plan_autotune")
        return ms.value

    def tuning(self, p: int):
        """(cells per launch sequence of degree p, concurrent schedule on?)"""
        a, b = C.c_int64(), C.c_int32()
        _check(lib().dpg_plan_tuning(self._h, int(p), C.byref(a), C.byref(b)), "dpg_plan_tuning")
        return a.value, bool(b.value)

    def tiles(self, p: int) -> int:
        """dpg_plan_tiles: column tiles per chunk of degree p's sum-factorised formation."""
        a = C.c_int32()
        _check(lib().dpg_plan_tiles(self._h, int(p), C.byref(a)), "dpg_plan_tiles")
        return a.value

    def set_tiles(self, p: int, form_col_tiles: int):
        """dpg_plan_set_tiles."""
        _check(lib().dpg_plan_set_tiles(self._h, int(p), int(form_col_tiles)), "dpg_plan_set_tiles")

    def graph(self, prob: DeviceProblem, x, K, l, eta, info, precision: int = DPG_FP64, first: int = 0,
              count: int = None) -> "Graph":
        """dpg_graph_create: the solve of cells first..first+count-1 as a replayable HIP graph."""
        if count is None:
            count = self.n_cells - first
        s = prob.cstruct()
        h = C.c_void_p()
        _check(lib().dpg_graph_create(self._h, C.byref(s), int(first), int(count), _ptr(x), _ptr(K), _ptr(l),
                                      _ptr(eta), _ptr(info), int(precision), C.byref(h)), "dpg_graph_create")
        return Graph(h, (self, prob, x, K, l, eta, info))

    def trace_offsets(self):
        """(A_off, b_off): offsets of the condensed cell matrices and right-hand sides."""
        A_off = np.zeros(self.n_cells + 1, np.int64)
        b_off = np.zeros(self.n_cells + 1, np.int64)
        _check(lib().dpg_plan_trace_offsets(self._h, A_off.ctypes.data, b_off.ctypes.data), "dpg_plan_trace_offsets")
        return A_off, b_off

    def condense(self, K, l, stream=None):
        """dpg_condense: (A, b, info) device tensors from a solve's K_e, l_e."""
        import torch
        A_off, b_off = self.trace_offsets()
        dev = K.device
        A = torch.empty(max(int(A_off[-1]), 1), dtype=torch.complex128, device=dev)
        b = torch.empty(max(int(b_off[-1]), 1), dtype=torch.complex128, device=dev)
        info = torch.empty(max(self.n_cells, 1), dtype=torch.int32, device=dev)
        _check(lib().dpg_condense(self._h, _ptr(K), _ptr(l), _ptr(A), _ptr(b), _ptr(info), _stream(stream)),
               "dpg_condense")
        return A, b, info

    def reconstruct(self, K, l, t_local, x=None, stream=None):
        """dpg_reconstruct: (x, info) with x = [u_K ; t_K] per cell (the layout
        of a solve's x) from a solve's K_e, l_e and the local traces."""
        import torch
        dev = K.device
        if x is None:
            x = torch.empty(max(int(self.v_off[-1]), 1), dtype=torch.complex128, device=dev)
        info = torch.empty(max(self.n_cells, 1), dtype=torch.int32, device=dev)
        _check(lib().dpg_reconstruct(self._h, _ptr(K), _ptr(l), _ptr(t_local), _ptr(x), _ptr(info), _stream(stream)),
               "dpg_reconstruct")
        return x, info

    def power_dissipation(self, prob: DeviceProblem, x, out=None, stream=None):
        """dpg_power_dissipation: [n_cells, 3] float64 device tensor of the cell
        integrals of the dissipated power density, |E|^2 and |H|^2."""
        import torch
        if out is None:
            out = torch.empty((max(self.n_cells, 1), 3), dtype=torch.float64, device=x.device)
        s = prob.cstruct()
        _check(lib().dpg_power_dissipation(self._h, C.byref(s), _ptr(x), _ptr(out), _stream(stream)),
               "dpg_power_dissipation")
        return out

    def range_sizes(self, first: int, count: int):
        """(K elements, l/x elements) of the outputs of a range solve."""
        return (int(self.K_off[first + count] - self.K_off[first]), int(self.v_off[first + count] - self.v_off[first]))

    def form_local(self, prob: DeviceProblem, first: int, count: int, stream=None):
        """dpg_form_local: unscaled G, B_f, l of cells first..first+count-1 (same degree)."""
        import torch
        p = int(self.degree[first])
        nt, nu, ntr = dpg_local_dims(p, self.dp)
        k = nu + ntr
        dev = prob.vertices.device
        G = torch.empty((count, nt, nt), dtype=torch.complex128, device=dev)
        Bf = torch.empty((count, k, nt), dtype=torch.complex128, device=dev)
        lv = torch.empty((count, nt), dtype=torch.complex128, device=dev)
        info = torch.zeros(count, dtype=torch.int32, device=dev)
        s = prob.cstruct()
        _check(lib().dpg_form_local(self._h, C.byref(s), int(first), int(count), _ptr(G), _ptr(Bf), _ptr(lv),
                                    _ptr(info), _stream(stream)), "dpg_form_local")
        # column-major per cell: G[c][col][row] -> transpose to [row][col]
        return G.transpose(1, 2), Bf.transpose(1, 2), lv, info

    def form_augmented(self, prob: DeviceProblem, first: int, count: int, x=None, stream=None):
        """dpg_form_augmented: the Jacobi-scaled D G D, D B_f, D l, D r and d of
        cells first..first+count-1 (same degree); x holds the range's
        coefficients (or None: r = 0)."""
        import torch
        p = int(self.degree[first])
        nt, nu, ntr = dpg_local_dims(p, self.dp)
        k = nu + ntr
        dev = prob.vertices.device
        G = torch.empty((count, nt, nt), dtype=torch.complex128, device=dev)
        Bf = torch.empty((count, k, nt), dtype=torch.complex128, device=dev)
        lv = torch.empty((count, nt), dtype=torch.complex128, device=dev)
        rv = torch.empty((count, nt), dtype=torch.complex128, device=dev)
        d = torch.empty((count, nt), dtype=torch.float64, device=dev)
        info = torch.zeros(count, dtype=torch.int32, device=dev)
        s = prob.cstruct()
        _check(lib().dpg_form_augmented(self._h, C.byref(s), int(first), int(count), _ptr(x), _ptr(G), _ptr(Bf),
                                        _ptr(lv), _ptr(rv), _ptr(d), _ptr(info), _stream(stream)),
               "dpg_form_augmented")
        return G.transpose(1, 2), Bf.transpose(1, 2), lv, rv, d, info


def trace_numbering(cells, face_kind, degree):
    """dpg_trace_numbering (host): (glob, n_dofs), glob laid out cell by cell."""
    cells = np.ascontiguousarray(np.asarray(cells, np.int64))
    fk = np.ascontiguousarray(np.asarray(face_kind, np.int8))
    deg = np.ascontiguousarray(np.asarray(degree, np.int8))
    total = int(np.sum(24 * (deg.astype(np.int64) + 1) ** 2))
    glob = np.zeros(max(total, 1), np.int64)
    n = C.c_int64()
    _check(lib().dpg_trace_numbering(cells.ctypes.data, fk.ctypes.data, deg.ctypes.data, int(deg.shape[0]),
                                     glob.ctypes.data, C.byref(n)), "dpg_trace_numbering")
    return glob[:total], n.value


def sync(info=None, stream=None):
    """dpg_sync: waits for `stream`; returns (status, failed cells, first
    failed index) for the int32 device tensor `info` (or None).  Raises only
    for argument and HIP errors; DPG_ERR_CELL is returned, not raised."""
    n = 0 if info is None else int(info.numel())
    nf, ff = C.c_int64(), C.c_int64()
    rc = lib().dpg_sync(_stream(stream), _ptr(info) if n else None, n, C.byref(nf), C.byref(ff))
    if rc not in (DPG_OK, DPG_ERR_CELL):
        _check(rc, "dpg_sync")
    return rc, nf.value, ff.value


def cg_solve(n_rows: int, row_ptr, col, vals, b, x, tol: float, max_iter: int, stream=None):
    """dpg_cg_solve on a device CSR system (row_ptr, col: tensors or raw device
    addresses).  x: start in, last iterate out.  Returns (iterations, ||r|| / ||b||)."""
    it, rr = C.c_int64(), C.c_double()
    rp = row_ptr if isinstance(row_ptr, int) else _ptr(row_ptr)
    cl = col if isinstance(col, int) else _ptr(col)
    _check(lib().dpg_cg_solve(int(n_rows), rp, cl, _ptr(vals), _ptr(b), _ptr(x), float(tol), int(max_iter),
                              C.byref(it), C.byref(rr), _stream(stream)), "dpg_cg_solve")
    return it.value, rr.value


def dorfler_mark_workspace_size(n: int) -> int:
    """Bytes of the temporaries dorfler_mark needs for n values."""
    b = C.c_size_t()
    _check(lib().dpg_dorfler_mark_workspace_size(int(n), C.byref(b)), "dpg_dorfler_mark_workspace_size")
    return b.value


def dorfler_mark(values, refine_fraction: float = 0.30, coarsen_fraction: float = 0.05, flags=None, stream=None,
                 workspace=None):
    """dpg_dorfler_mark: int8 device flags (+1 refine, -1 coarsen, 0 keep) from
    the float64 device tensor `values` (one indicator per cell).  `workspace`
    (a device tensor of at least dorfler_mark_workspace_size(n) bytes): the
    library then allocates nothing and does not synchronise; without it the
    library allocates its temporaries and synchronises the stream."""
    import torch
    n = int(values.numel())
    if flags is None:
        flags = torch.empty(max(n, 1), dtype=torch.int8, device=values.device)
    wp, wb = None, 0
    if workspace is not None:
        wp, wb = _ptr(workspace), int(workspace.numel() * workspace.element_size())
    _check(lib().dpg_dorfler_mark(n, _ptr(values), float(refine_fraction), float(coarsen_fraction), _ptr(flags),
                                  wp, wb, _stream(stream)), "dpg_dorfler_mark")
    return flags


def dorfler_mark_noalloc(values, refine_fraction: float = 0.30, coarsen_fraction: float = 0.05, flags=None,
                        stream=None):
    """dpg_dorfler_mark_noalloc: the flags of dorfler_mark, with the library's
    static device scratch instead of an allocation (n <= 2^20); `flags`
    (int8, device, at least n entries) must be given to allocate nothing."""
    import torch
    n = int(values.numel())
    if flags is None:
        flags = torch.empty(max(n, 1), dtype=torch.int8, device=values.device)
    _check(lib().dpg_dorfler_mark_noalloc(n, _ptr(values), float(refine_fraction), float(coarsen_fraction),
                                          _ptr(flags), _stream(stream)), "dpg_dorfler_mark_noalloc")
    return flags


class TraceSystem:
    """dpg_trace_system_*: numbering, CSR structure and gather assembly of the condensed system."""

    def __init__(self, plan: "Plan", cells, face_kind):
        self._plan = plan
        cells = np.ascontiguousarray(np.asarray(cells, np.int64))
        fk = np.ascontiguousarray(np.asarray(face_kind, np.int8))
        h = C.c_void_p()
        _check(lib().dpg_trace_system_create(plan._h, cells.ctypes.data, fk.ctypes.data, C.byref(h)),
               "dpg_trace_system_create")
        self._h = h
        a, b = C.c_int64(), C.c_int64()
        _check(lib().dpg_trace_system_info(self._h, C.byref(a), C.byref(b)), "dpg_trace_system_info")
        self.n_dofs, self.nnz = a.value, b.value
        rp, cl = C.c_void_p(), C.c_void_p()
        _check(lib().dpg_trace_system_csr(self._h, C.byref(rp), C.byref(cl)), "dpg_trace_system_csr")
        self.row_ptr_ptr, self.col_ptr = rp.value, cl.value

    def numbering(self):
        total = int(self._plan.trace_offsets()[1][-1])
        glob = np.zeros(max(total, 1), np.int64)
        _check(lib().dpg_trace_system_numbering(self._h, glob.ctypes.data), "dpg_trace_system_numbering")
        return glob[:total]

    def assemble(self, A, b, stream=None):
        """(vals, rhs) device tensors of the assembled CSR matrix and right-hand side."""
        import torch
        vals = torch.empty(max(self.nnz, 1), dtype=torch.complex128, device=A.device)
        rhs = torch.empty(max(self.n_dofs, 1), dtype=torch.complex128, device=A.device)
        _check(lib().dpg_assemble(self._h, _ptr(A), _ptr(b), _ptr(vals), _ptr(rhs), _stream(stream)), "dpg_assemble")
        return vals, rhs

    def matvec(self, vals, x, y, stream=None):
        _check(lib().dpg_csr_matvec(self.n_dofs, self.row_ptr_ptr, self.col_ptr, _ptr(vals), _ptr(x), _ptr(y),
                                    _stream(stream)), "dpg_csr_matvec")

    def scatter(self, t, t_local=None, stream=None):
        """dpg_trace_system_scatter: the cells' local traces (b_off layout) from the global vector t."""
        import torch
        if t_local is None:
            total = int(self._plan.trace_offsets()[1][-1])
            t_local = torch.empty(max(total, 1), dtype=torch.complex128, device=t.device)
        _check(lib().dpg_trace_system_scatter(self._h, _ptr(t), _ptr(t_local), _stream(stream)),
               "dpg_trace_system_scatter")
        return t_local

    def solve(self, vals, rhs, x, tol: float, max_iter: int, stream=None):
        """CG on the assembled system (dpg_trace_system_cg, with the system's
        own CG vectors); x: start in, solution out.  Returns (iterations,
        relative residual)."""
        it, rr = C.c_int64(), C.c_double()
        _check(lib().dpg_trace_system_cg(self._h, _ptr(vals), _ptr(rhs), _ptr(x), float(tol), int(max_iter),
                                         C.byref(it), C.byref(rr), _stream(stream)), "dpg_trace_system_cg")
        return it.value, rr.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dpg_trace_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured solve (dpg_graph_create); keeps the plan and buffers it references alive."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def launch(self, stream=None):
        _check(lib().dpg_graph_launch(self._h, _stream(stream)), "dpg_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dpg_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cell_view(plan: Plan, K, l, c: int):
    """(K_e, l_e) of cell c as views into the packed outputs."""
    k = int(plan.v_off[c + 1] - plan.v_off[c])
    Kc = K[int(plan.K_off[c]):int(plan.K_off[c + 1])].view(k, k).transpose(0, 1)
    return Kc, l[int(plan.v_off[c]):int(plan.v_off[c + 1])]
