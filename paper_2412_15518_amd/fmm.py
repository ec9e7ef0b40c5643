"""Python binding of the C ABI in include/ot_fmm.h (argument marshalling only).

Every step of the solve runs in the HIP kernels of libotfmm.so; torch supplies
device memory and the current stream.  The library must be built
(python -m paper_2412_15518_amd.build); importing this module without it
raises, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotfmm.so")

# status codes and flags (include/ot_fmm.h)
OK = 0
INVALID_ARGUMENT = -1
INVALID_LAYOUT = -2
UNSUPPORTED_ORDER = -3
UNSUPPORTED_THETA = -4
UNSUPPORTED_LAYOUT = -5
OUT_OF_MEMORY = -6
DEVICE_ERROR = -7
NO_DEVICE_STATE = -8
FLAG_FP64 = 0
FLAG_HOST_ONLY = 1
FLAG_M2L_FP32 = 2
FLAG_AUTOTUNE = 4
FLAG_AM_CORRECTION = 8

NUM_PHASES = 8
PHASES = ["upward_leaf", "m2m", "m2l", "l2l", "leaf", "upward_leaf_adj", "leaf_adj", "total"]

EXPORTS = ["ot_fmm_plan_create", "ot_fmm_forward", "ot_fmm_adjoint", "ot_fmm_am_correction", "ot_fmm_plan_info",
           "ot_fmm_destroy", "ot_fmm_status_string", "ot_fmm_last_error", "ot_fmm_timing_begin",
           "ot_fmm_timing_end", "ot_fmm_phase_name", "ot_fmm_timing_phases", "ot_fmm_batch_create",
           "ot_fmm_batch_forward", "ot_fmm_batch_adjoint", "ot_fmm_batch_capture_forward",
           "ot_fmm_batch_capture_adjoint", "ot_fmm_graph_launch", "ot_fmm_graph_destroy", "ot_fmm_batch_destroy",
           "ot_fmm_plan_set_leaf_chunks"]


class OTFMMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class _Layout(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("level", C.POINTER(C.c_int32)), ("coord", C.POINTER(C.c_int32)),
                ("parent", C.POINTER(C.c_int32)), ("is_leaf", C.POINTER(C.c_uint8)),
                ("h_leaf_min", C.c_double), ("origin", C.c_double * 3), ("G", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("depth", C.c_int32), ("order", C.c_int32), ("theta", C.c_double),
                ("n_nodes", C.c_int64), ("n_leaf_nodes", C.c_int64), ("n_leaf_cells", C.c_int64),
                ("p2p_pairs", C.c_int64), ("m2l_pairs", C.c_int64), ("m2l_pairs_level", C.c_int64 * 16),
                ("flops_forward", C.c_double), ("flops_adjoint", C.c_double),
                ("bytes_forward", C.c_double), ("bytes_adjoint", C.c_double), ("device_bytes", C.c_size_t),
                ("leaf_chunks_forward", C.c_int32), ("leaf_chunks_adjoint", C.c_int32)]


class _Timing(C.Structure):
    _fields_ = [("calls", C.c_int32), ("launches", C.c_int64 * NUM_PHASES),
                ("events", C.c_int64 * NUM_PHASES), ("ms", C.c_double * NUM_PHASES)]


_lib = None


def load_library():
    """Load libotfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_15518_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.ot_fmm_plan_create.argtypes = [C.POINTER(_Layout), C.c_double, C.c_int, C.c_uint32, C.POINTER(vp)]
    lib.ot_fmm_plan_create.restype = C.c_int
    lib.ot_fmm_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.ot_fmm_forward.restype = C.c_int
    lib.ot_fmm_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.ot_fmm_adjoint.restype = C.c_int
    lib.ot_fmm_am_correction.argtypes = [vp, vp, vp, vp]
    lib.ot_fmm_am_correction.restype = C.c_int
    lib.ot_fmm_plan_info.argtypes = [vp, C.POINTER(_Info)]
    lib.ot_fmm_plan_info.restype = C.c_int
    lib.ot_fmm_destroy.argtypes = [vp]
    lib.ot_fmm_destroy.restype = None
    lib.ot_fmm_status_string.argtypes = [C.c_int]
    lib.ot_fmm_status_string.restype = C.c_char_p
    lib.ot_fmm_last_error.argtypes = []
    lib.ot_fmm_last_error.restype = C.c_char_p
    lib.ot_fmm_timing_begin.argtypes = [vp, C.c_int]
    lib.ot_fmm_timing_begin.restype = C.c_int
    lib.ot_fmm_timing_end.argtypes = [vp, C.POINTER(_Timing)]
    lib.ot_fmm_timing_end.restype = C.c_int
    lib.ot_fmm_phase_name.argtypes = [C.c_int]
    lib.ot_fmm_phase_name.restype = C.c_char_p
    lib.ot_fmm_timing_phases.argtypes = [vp, C.c_uint32]
    lib.ot_fmm_timing_phases.restype = C.c_int
    lib.ot_fmm_plan_set_leaf_chunks.argtypes = [vp, C.c_int, C.c_int]
    lib.ot_fmm_plan_set_leaf_chunks.restype = C.c_int
    pp = C.POINTER(vp)
    lib.ot_fmm_batch_create.argtypes = [pp, C.c_int, C.c_int, C.POINTER(vp)]
    lib.ot_fmm_batch_create.restype = C.c_int
    for name in ("ot_fmm_batch_forward", "ot_fmm_batch_adjoint"):
        getattr(lib, name).argtypes = [vp, pp, pp, pp, vp]
        getattr(lib, name).restype = C.c_int
    for name in ("ot_fmm_batch_capture_forward", "ot_fmm_batch_capture_adjoint"):
        getattr(lib, name).argtypes = [vp, pp, pp, pp, C.POINTER(vp)]
        getattr(lib, name).restype = C.c_int
    lib.ot_fmm_graph_launch.argtypes = [vp, vp]
    lib.ot_fmm_graph_launch.restype = C.c_int
    lib.ot_fmm_graph_destroy.argtypes = [vp]
    lib.ot_fmm_graph_destroy.restype = None
    lib.ot_fmm_batch_destroy.argtypes = [vp]
    lib.ot_fmm_batch_destroy.restype = None
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load_library()
        raise OTFMMError(rc, f"{lib.ot_fmm_status_string(rc).decode()}: {lib.ot_fmm_last_error().decode()}")


class Plan:
    """An FMM plan over one octree layout (see workloads.Layout).

    All device memory is allocated here, on the current device; forward and
    adjoint only enqueue kernels on the current torch stream.  m2l_fp32 runs
    the M2L in FP32 with FP64 accumulation (OT_FMM_M2L_FP32); autotune times
    the leaf passes' stencil chunk counts at creation (OT_FMM_AUTOTUNE);
    am_correction keeps what am_correction() needs (OT_FMM_AM_CORRECTION)."""

    def __init__(self, layout, theta: float = 0.4, order: int = 3, host_only: bool = False,
                 m2l_fp32: bool = False, autotune: bool = False, am_correction: bool = False):
        lib = load_library()
        self._keep = [np.ascontiguousarray(layout.level, dtype=np.int32),
                      np.ascontiguousarray(layout.coord, dtype=np.int32).reshape(-1),
                      np.ascontiguousarray(layout.parent, dtype=np.int32),
                      np.ascontiguousarray(layout.is_leaf, dtype=np.uint8)]
        lv, co, pa, il = self._keep
        L = _Layout()
        L.n_nodes = int(lv.shape[0])
        L.level = lv.ctypes.data_as(C.POINTER(C.c_int32))
        L.coord = co.ctypes.data_as(C.POINTER(C.c_int32))
        L.parent = pa.ctypes.data_as(C.POINTER(C.c_int32))
        L.is_leaf = il.ctypes.data_as(C.POINTER(C.c_uint8))
        L.h_leaf_min = float(layout.h_leaf_min)
        L.origin = (C.c_double * 3)(*[float(x) for x in layout.origin])
        L.G = float(layout.G)
        self._handle = C.c_void_p()
        flags = ((FLAG_HOST_ONLY if host_only else FLAG_FP64) | (FLAG_M2L_FP32 if m2l_fp32 else 0)
                 | (FLAG_AUTOTUNE if autotune else 0) | (FLAG_AM_CORRECTION if am_correction else 0))
        _check(lib.ot_fmm_plan_create(C.byref(L), float(theta), int(order), flags, C.byref(self._handle)))
        self._keep = None
        self.layout = layout
        inf = self.info()
        self.n_cells = inf["n_leaf_cells"]
        self.device = None
        if not host_only:
            import torch
            self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            load_library().ot_fmm_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = _Info()
        _check(load_library().ot_fmm_plan_info(self._handle, C.byref(inf)))
        d = {k: getattr(inf, k) for k, _ in _Info._fields_}
        d["m2l_pairs_level"] = list(inf.m2l_pairs_level)[: max(inf.depth, 0)]
        return d

    def set_leaf_chunks(self, forward: int, adjoint: int):
        """Stencil chunk counts (1..8) of the forward and adjoint leaf passes."""
        _check(load_library().ot_fmm_plan_set_leaf_chunks(self._handle, int(forward), int(adjoint)))

    # ------------------------------------------------------------------ calls
    def _stream(self):
        import torch
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check_field(self, t, ncomp: int, name: str):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA float64 tensor")
        if t.numel() != ncomp * self.n_cells or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {ncomp} x {self.n_cells} values")

    def forward_into(self, rho, phi, g):
        for t, k, n in ((rho, 1, "rho"), (phi, 1, "phi"), (g, 3, "g")):
            self._check_field(t, k, n)
        _check(load_library().ot_fmm_forward(self._handle, C.c_void_p(rho.data_ptr()), C.c_void_p(phi.data_ptr()),
                                             C.c_void_p(g.data_ptr()), self._stream()))

    def adjoint_into(self, dphi, dg, drho):
        for t, k, n in ((dphi, 1, "dphi"), (dg, 3, "dg"), (drho, 1, "drho")):
            self._check_field(t, k, n)
        _check(load_library().ot_fmm_adjoint(self._handle, C.c_void_p(dphi.data_ptr()), C.c_void_p(dg.data_ptr()),
                                             C.c_void_p(drho.data_ptr()), self._stream()))

    def am_correction(self, rho):
        """rho [N] -> t [3, N]: the spin torque per unit mass of the
        angular-momentum correction (ot_fmm_am_correction)."""
        import torch
        rho = rho.contiguous().reshape(-1)
        self._check_field(rho, 1, "rho")
        t = torch.empty((3, self.n_cells), dtype=torch.float64, device=rho.device)
        _check(load_library().ot_fmm_am_correction(self._handle, C.c_void_p(rho.data_ptr()),
                                                   C.c_void_p(t.data_ptr()), self._stream()))
        return t

    def forward(self, rho):
        """rho [N] -> (phi [N], g [3, N]) in layout order."""
        import torch
        rho = rho.contiguous()
        phi = torch.empty(self.n_cells, dtype=torch.float64, device=rho.device)
        g = torch.empty((3, self.n_cells), dtype=torch.float64, device=rho.device)
        self.forward_into(rho.reshape(-1), phi, g)
        return phi, g

    def adjoint(self, dphi, dg):
        """(dphi [N], dg [3, N]) -> drho [N]."""
        import torch
        dphi = dphi.contiguous()
        dg = dg.contiguous()
        drho = torch.empty(self.n_cells, dtype=torch.float64, device=dphi.device)
        self.adjoint_into(dphi.reshape(-1), dg.reshape(-1), drho)
        return drho

    # ----------------------------------------------------------------- timing
    def timing_begin(self, max_calls: int):
        _check(load_library().ot_fmm_timing_begin(self._handle, int(max_calls)))

    def timing_phases(self, phases):
        """Record events only around the named phases (after timing_begin)."""
        mask = 0
        for name in phases:
            mask |= 1 << PHASES.index(name)
        _check(load_library().ot_fmm_timing_phases(self._handle, C.c_uint32(mask)))

    def timing_end(self) -> dict:
        t = _Timing()
        _check(load_library().ot_fmm_timing_end(self._handle, C.byref(t)))
        return {"calls": t.calls,
                "phases": {PHASES[i]: {"launches": t.launches[i], "events": t.events[i], "ms": t.ms[i]}
                           for i in range(NUM_PHASES)}}


def _ptrs(tensors):
    return (C.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


class Graph:
    """A captured batch call (ot_fmm_batch_capture_*): launch() replays it on
    the current torch stream, on the buffers it was captured with."""

    def __init__(self, handle, keep):
        self._handle = handle
        self._keep = keep           # the captured buffers stay alive with the graph

    def launch(self):
        import torch
        _check(load_library().ot_fmm_graph_launch(self._handle, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            load_library().ot_fmm_graph_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Forward or adjoint of several independent plans in one call, spread
    over n_streams internal streams (ot_fmm_batch_*).  The plans must outlive
    the batch."""

    def __init__(self, plans, n_streams: int = 4):
        self.plans = list(plans)
        handles = (C.c_void_p * len(self.plans))(*[p._handle.value for p in self.plans])
        self._handle = C.c_void_p()
        _check(load_library().ot_fmm_batch_create(handles, len(self.plans), int(n_streams), C.byref(self._handle)))

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            load_library().ot_fmm_batch_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_lists(self, lists, specs):
        for lst, (ncomp, name) in zip(lists, specs):
            if len(lst) != len(self.plans):
                raise ValueError(f"{name} needs one tensor per plan")
            for p, t in zip(self.plans, lst):
                p._check_field(t, ncomp, name)

    def _stream(self):
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def forward_into(self, rhos, phis, gs):
        self._check_lists((rhos, phis, gs), ((1, "rho"), (1, "phi"), (3, "g")))
        _check(load_library().ot_fmm_batch_forward(self._handle, _ptrs(rhos), _ptrs(phis), _ptrs(gs), self._stream()))

    def adjoint_into(self, dphis, dgs, drhos):
        self._check_lists((dphis, dgs, drhos), ((1, "dphi"), (3, "dg"), (1, "drho")))
        _check(load_library().ot_fmm_batch_adjoint(self._handle, _ptrs(dphis), _ptrs(dgs), _ptrs(drhos),
                                                   self._stream()))

    def capture_forward(self, rhos, phis, gs) -> Graph:
        self._check_lists((rhos, phis, gs), ((1, "rho"), (1, "phi"), (3, "g")))
        h = C.c_void_p()
        _check(load_library().ot_fmm_batch_capture_forward(self._handle, _ptrs(rhos), _ptrs(phis), _ptrs(gs),
                                                           C.byref(h)))
        return Graph(h, (list(rhos), list(phis), list(gs)))

    def capture_adjoint(self, dphis, dgs, drhos) -> Graph:
        self._check_lists((dphis, dgs, drhos), ((1, "dphi"), (3, "dg"), (1, "drho")))
        h = C.c_void_p()
        _check(load_library().ot_fmm_batch_capture_adjoint(self._handle, _ptrs(dphis), _ptrs(dgs), _ptrs(drhos),
                                                           C.byref(h)))
        return Graph(h, (list(dphis), list(dgs), list(drhos)))


def _make_function():
    import torch

    class OTFMM(torch.autograd.Function):
        """phi, g = OTFMM.apply(rho, plan); backward runs the hand-written
        adjoint (the transposed FMM) of the same plan."""

        @staticmethod
        def forward(ctx, rho, plan):
            ctx.plan = plan
            return plan.forward(rho)

        @staticmethod
        def backward(ctx, dphi, dg):
            import torch as _t
            plan = ctx.plan
            if dphi is None:
                dphi = _t.zeros(plan.n_cells, dtype=_t.float64, device=dg.device)
            if dg is None:
                dg = _t.zeros((3, plan.n_cells), dtype=_t.float64, device=dphi.device)
            return plan.adjoint(dphi, dg), None

    return OTFMM


_OTFMM = None


def otfmm(rho, plan):
    """Differentiable (phi, g) = FMM(rho) on `plan`."""
    global _OTFMM
    if _OTFMM is None:
        _OTFMM = _make_function()
    return _OTFMM.apply(rho, plan)
