"""Python binding of the C ABI in include/brahms.h (argument marshalling only).

Every step of the propagation runs in the HIP library; this module only
translates arguments, owns nothing but torch tensors for device memory, and
raises if the library is missing.  Names follow the C calls.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbrahms.so")

BRAHMS_OK = 0
BRAHMS_E_INVALID_ARG = 1
BRAHMS_E_UNSUPPORTED = 2
BRAHMS_E_DEVICE = 3
BRAHMS_E_NONFINITE = 4
BRAHMS_E_STATE = 5
BRAHMS_CHECK_FINITE = 1

STATUS_NAMES = {0: "OK", 1: "E_INVALID_ARG", 2: "E_UNSUPPORTED", 3: "E_DEVICE",
                4: "E_NONFINITE", 5: "E_STATE"}

SUPPORTED_LENGTHS = (1, 2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256)
# lengths whose linear passes have no 512-thread form (schedule field wide
# is ignored on their axes)
NARROW_ONLY_LENGTHS = (72, 144)
# lengths with a second register/lane split (schedule field split)
ALT_SPLIT_LENGTHS = (8, 12, 16, 24, 32, 48, 64)
TIMING_KINDS = 4
TIMING_NAMES = ("x_pass", "y_pass", "t_pass", "tables")


class BrahmsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: BRAHMS_{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ScheduleC(ctypes.Structure):
    _fields_ = [("pass_order", ctypes.c_int), ("graph", ctypes.c_int),
                ("merge_halves", ctypes.c_int), ("fuse_steps", ctypes.c_int),
                ("split", ctypes.c_int), ("wide", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class FieldParamsC(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("diffraction", ctypes.c_double),
                ("tan_rho", ctypes.c_double), ("delay", ctypes.c_double),
                ("k2", ctypes.c_double), ("k3", ctypes.c_double), ("alpha", ctypes.c_double)]


class ParamsC(ctypes.Structure):
    _fields_ = [("dz", ctypes.c_double), ("dk_const", ctypes.c_double),
                ("dk", ctypes.POINTER(ctypes.c_double)), ("n_dk", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("field", FieldParamsC * 3), ("flags", ctypes.c_uint),
                ("dk_map", ctypes.POINTER(ctypes.c_double)),
                ("dk_map_scale", ctypes.POINTER(ctypes.c_double)), ("n_dk_map_scale", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbrahms.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP engine library not found at {path}; build it with "
                           "`python -m paper_2609_08384_amd.build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "brahms_plan_create": [i, i, i, i, ctypes.POINTER(ParamsC), vp, ctypes.POINTER(vp)],
        "brahms_plan_workspace_size": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "brahms_plan_bind": [vp, ctypes.POINTER(vp), vp],
        "brahms_step": [vp, i],
        "brahms_propagate": [vp, d],
        "brahms_propagate_noalloc": [vp, ctypes.POINTER(vp), d],
        "brahms_get_z": [vp, ctypes.POINTER(d)],
        "brahms_set_z": [vp, d],
        "brahms_plan_destroy": [vp],
        "brahms_plan_set_schedule": [vp, ctypes.POINTER(ScheduleC)],
        "brahms_plan_get_schedule": [vp, ctypes.POINTER(ScheduleC)],
        "brahms_adjoint_workspace_size": [vp, i, i, ctypes.POINTER(ctypes.c_size_t)],
        "brahms_adjoint_forward": [vp, i, i, vp],
        "brahms_adjoint_backward": [vp, ctypes.POINTER(vp), ctypes.POINTER(d)],
        "brahms_adjoint": [vp, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                           ctypes.POINTER(d), vp],
        "brahms_batch_create": [i, ctypes.POINTER(i), ctypes.POINTER(ParamsC), ctypes.POINTER(i), vp,
                                ctypes.POINTER(vp)],
        "brahms_batch_set_schedule": [vp, i, ctypes.POINTER(i)],
        "brahms_batch_set_group_limits": [vp, ctypes.POINTER(i)],
        "brahms_batch_set_streams": [vp, i, i],
        "brahms_batch_set_wide": [vp, ctypes.POINTER(i)],
        "brahms_batch_set_splits": [vp, ctypes.POINTER(i)],
        "brahms_batch_set_merge_halves": [vp, i],
        "brahms_batch_set_fuse_steps": [vp, i],
        "brahms_batch_workspace_size": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "brahms_batch_bind": [vp, ctypes.POINTER(vp), vp],
        "brahms_batch_run": [vp],
        "brahms_batch_run_steps": [vp, ctypes.POINTER(i)],
        "brahms_batch_groups": [vp, ctypes.POINTER(i), ctypes.POINTER(i)],
        "brahms_batch_destroy": [vp],
        "brahms_timing_enable": [vp, i],
        "brahms_timing_read": [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong)],
        "brahms_record_size": [vp, ctypes.POINTER(i)],
        "brahms_diagnose": [vp, vp],
        "brahms_set_monitor": [vp, i, vp, i],
        "brahms_get_monitor_count": [vp, ctypes.POINTER(i)],
        "brahms_set_snapshots": [vp, i, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(vp)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.brahms_last_error.argtypes = []
    lib.brahms_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _device_bytes(nbytes: int, device, stream=None) -> torch.Tensor:
    """A uint8 device tensor of nbytes for a workspace used by library work on
    `stream`: allocated while that stream is current, so that torch's caching
    allocator does not hand the memory to other work before the work queued
    on that stream is done."""
    if stream is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _check(status: int, where: str):
    if status != BRAHMS_OK:
        msg = _lib.brahms_last_error().decode() if _lib is not None else ""
        raise BrahmsError(status, where, msg)


@dataclass
class FieldParams:
    kappa: float = 0.0
    diffraction: float = 0.0
    tan_rho: float = 0.0
    delay: float = 0.0
    k2: float = 0.0
    k3: float = 0.0
    alpha: float = 0.0


@dataclass
class Params:
    dz: float
    fields: List[FieldParams]
    dk_const: float = 0.0
    dk: Optional[Sequence[float]] = None
    dx: float = 1.0
    dy: float = 1.0
    dt: float = 1.0
    check_finite: bool = False
    dk_map: Optional[object] = None                # [ny, nx] array: m(x, y)
    dk_map_scale: Optional[Sequence[float]] = None  # s_n per step (None: 1)


def params_from_workload(wl) -> Params:
    fs = [FieldParams(f.kappa, f.diffraction, f.tan_rho, f.delay, f.k2, f.k3, f.alpha)
          for f in wl.fields]
    dk = None if wl.dk is None else [float(v) for v in wl.dk]
    return Params(dz=wl.dz, fields=fs, dk_const=wl.dk_const, dk=dk,
                  dk_map=getattr(wl, "dk_map", None), dk_map_scale=getattr(wl, "dk_map_scale", None))


def _doubles(values):
    arr = (ctypes.c_double * len(values))(*[float(v) for v in values])
    return arr, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))


def _params_c(p: Params, nf: int):
    c = ParamsC()
    c.dz = p.dz
    c.dk_const = p.dk_const
    keep = []
    if p.dk is not None:
        arr, c.dk = _doubles(p.dk)
        keep.append(arr)
        c.n_dk = len(p.dk)
    else:
        c.dk = None
        c.n_dk = 0
    c.dk_map, c.dk_map_scale, c.n_dk_map_scale = None, None, 0
    if p.dk_map is not None:
        arr, c.dk_map = _doubles(np.asarray(p.dk_map, dtype=np.float64).reshape(-1))
        keep.append(arr)
        if p.dk_map_scale is not None:
            arr, c.dk_map_scale = _doubles(p.dk_map_scale)
            keep.append(arr)
            c.n_dk_map_scale = len(p.dk_map_scale)
    c.dx, c.dy, c.dt = p.dx, p.dy, p.dt
    for j, f in enumerate(p.fields[:3]):
        c.field[j] = FieldParamsC(f.kappa, f.diffraction, f.tan_rho, f.delay, f.k2, f.k3, f.alpha)
    c.flags = BRAHMS_CHECK_FINITE if p.check_finite else 0
    return c, keep


class Plan:
    """brahms_plan: an nx x ny x nt grid with nf fields, bound to torch tensors.

    Fields are complex64 CUDA tensors of shape [nt, ny, nx] (x fastest),
    updated in place.  The workspace is a torch uint8 tensor owned here.
    """

    def __init__(self, nx: int, ny: int, nt: int, nf: int, params: Params,
                 stream: Optional[torch.cuda.Stream] = None):
        self._lib = load_library()
        self.nx, self.ny, self.nt, self.nf = nx, ny, nt, nf
        self.params = params
        self.stream = stream
        handle = ctypes.c_void_p()
        pc, keep = _params_c(params, nf)
        sptr = ctypes.c_void_p(stream.cuda_stream if stream is not None else
                               (torch.cuda.current_stream().cuda_stream
                                if torch.cuda.is_available() else 0))
        _check(self._lib.brahms_plan_create(nx, ny, nt, nf, ctypes.byref(pc), sptr,
                                            ctypes.byref(handle)), "brahms_plan_create")
        del keep
        self._h = handle
        size = ctypes.c_size_t()
        _check(self._lib.brahms_plan_workspace_size(self._h, ctypes.byref(size)),
               "brahms_plan_workspace_size")
        self.workspace_bytes = int(size.value)
        self.workspace = None
        self.fields: List[torch.Tensor] = []
        self._monitor: Optional[torch.Tensor] = None
        self._snapshots: List[List[torch.Tensor]] = []

    def bind(self, fields: Sequence[torch.Tensor], workspace: Optional[torch.Tensor] = None):
        if len(fields) != self.nf:
            raise ValueError(f"need {self.nf} fields")
        for f in fields:
            if (f.dtype != torch.complex64 or not f.is_cuda or not f.is_contiguous()
                    or tuple(f.shape) != (self.nt, self.ny, self.nx)):
                raise ValueError("fields must be contiguous complex64 CUDA tensors of shape "
                                 f"[{self.nt}, {self.ny}, {self.nx}]")
        if workspace is None:
            workspace = _device_bytes(self.workspace_bytes + 256, fields[0].device, self.stream)
        ptr = workspace.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        arr = (ctypes.c_void_p * self.nf)(*[f.data_ptr() for f in fields])
        _check(self._lib.brahms_plan_bind(self._h, arr, ctypes.c_void_p(aligned)),
               "brahms_plan_bind")
        self.workspace = workspace
        self.fields = list(fields)
        return self

    def step(self, nsteps: int):
        _check(self._lib.brahms_step(self._h, int(nsteps)), "brahms_step")

    def propagate(self, z_end: float):
        _check(self._lib.brahms_propagate(self._h, float(z_end)), "brahms_propagate")

    def propagate_noalloc(self, fields: Sequence[torch.Tensor], z_end: float):
        """brahms_propagate_noalloc: bind `fields` with the library's static
        device scratch as workspace and propagate to z_end (no device
        allocation in the library or here)."""
        if len(fields) != self.nf:
            raise ValueError(f"need {self.nf} fields")
        for f in fields:
            if (f.dtype != torch.complex64 or not f.is_cuda or not f.is_contiguous()
                    or tuple(f.shape) != (self.nt, self.ny, self.nx)):
                raise ValueError("fields must be contiguous complex64 CUDA tensors of shape "
                                 f"[{self.nt}, {self.ny}, {self.nx}]")
        arr = (ctypes.c_void_p * self.nf)(*[f.data_ptr() for f in fields])
        _check(self._lib.brahms_propagate_noalloc(self._h, arr, float(z_end)),
               "brahms_propagate_noalloc")
        self.workspace = None
        self.fields = list(fields)

    @property
    def z(self) -> float:
        out = ctypes.c_double()
        _check(self._lib.brahms_get_z(self._h, ctypes.byref(out)), "brahms_get_z")
        return out.value

    def set_z(self, z: float):
        _check(self._lib.brahms_set_z(self._h, float(z)), "brahms_set_z")

    def set_schedule(self, pass_order: int, graph: int = 0, merge_halves: int = 0,
                     fuse_steps: int = 0, split: int = 0, wide: int = 0):
        """Pass order 0-3, graph replay of 64-step chunks, merged RK4
        half-steps within a call (constant dk, no transverse map), fused
        step pairs (with merged half-steps: two passes per step), the
        per-axis choice of register/lane split and the per-axis choice of
        512-thread blocks for linear passes (bits x = 1, y = 2, tau = 4)."""
        sc = ScheduleC()
        sc.pass_order = int(pass_order)
        sc.graph = int(graph)
        sc.merge_halves = int(merge_halves)
        sc.fuse_steps = int(fuse_steps)
        sc.split = int(split)
        sc.wide = int(wide)
        _check(self._lib.brahms_plan_set_schedule(self._h, ctypes.byref(sc)),
               "brahms_plan_set_schedule")

    def get_schedule(self) -> dict:
        sc = ScheduleC()
        _check(self._lib.brahms_plan_get_schedule(self._h, ctypes.byref(sc)),
               "brahms_plan_get_schedule")
        return {"pass_order": sc.pass_order, "graph": sc.graph, "merge_halves": sc.merge_halves,
                "fuse_steps": sc.fuse_steps, "split": sc.split, "wide": sc.wide}

    # --- adjoint (reverse-mode gradient of the z-loop) ---
    def adjoint_workspace_bytes(self, nsteps: int, checkpoint_every: int) -> int:
        out = ctypes.c_size_t()
        _check(self._lib.brahms_adjoint_workspace_size(self._h, int(nsteps), int(checkpoint_every),
                                                       ctypes.byref(out)),
               "brahms_adjoint_workspace_size")
        return int(out.value)

    def adjoint_forward(self, nsteps: int, checkpoint_every: int):
        """Advance nsteps like step(), keeping checkpoints for the backward."""
        nbytes = self.adjoint_workspace_bytes(nsteps, checkpoint_every)
        ws = _device_bytes(nbytes + 256, self.fields[0].device, self.stream)
        aligned = (ws.data_ptr() + 255) // 256 * 256
        _check(self._lib.brahms_adjoint_forward(self._h, int(nsteps), int(checkpoint_every),
                                                ctypes.c_void_p(aligned)),
               "brahms_adjoint_forward")
        self.adjoint_workspace = ws

    def adjoint_backward(self, grads: Sequence[torch.Tensor]):
        """grads: dJ/dA_out (complex64, field layout), overwritten with
        dJ/dA_in.  Returns dJ/ddk as a float64 numpy array (profile length,
        or one entry for a constant dk)."""
        import numpy as np
        for g in grads:
            if (g.dtype != torch.complex64 or not g.is_cuda or not g.is_contiguous()
                    or tuple(g.shape) != (self.nt, self.ny, self.nx)):
                raise ValueError("grads must be contiguous complex64 CUDA tensors in field layout")
        n_dk = len(self.params.dk) if self.params.dk is not None else 1
        out = np.zeros(n_dk, dtype=np.float64)
        arr = (ctypes.c_void_p * self.nf)(*[g.data_ptr() for g in grads])
        _check(self._lib.brahms_adjoint_backward(
            self._h, arr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
            "brahms_adjoint_backward")
        return out

    def adjoint(self, nsteps: int, checkpoint_every: int, fields_in: Sequence[torch.Tensor],
                grad_out: Sequence[torch.Tensor], grad_in: Sequence[torch.Tensor]):
        """brahms_adjoint: dJ/dA at the current z into grad_in (and returns
        dJ/ddk) for the cotangent grad_out at z + nsteps dz, with the
        forward from fields_in run in the bound fields."""
        import numpy as np
        for t in list(fields_in) + list(grad_out) + list(grad_in):
            if (t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous()
                    or tuple(t.shape) != (self.nt, self.ny, self.nx)):
                raise ValueError("buffers must be contiguous complex64 CUDA tensors in field layout")
        nbytes = self.adjoint_workspace_bytes(nsteps, checkpoint_every)
        ws = _device_bytes(nbytes + 256, self.fields[0].device, self.stream)
        aligned = (ws.data_ptr() + 255) // 256 * 256
        n_dk = len(self.params.dk) if self.params.dk is not None else 1
        out = np.zeros(n_dk, dtype=np.float64)
        arr = lambda ts: (ctypes.c_void_p * self.nf)(*[t.data_ptr() for t in ts])  # noqa: E731
        _check(self._lib.brahms_adjoint(self._h, int(nsteps), int(checkpoint_every), arr(fields_in),
                                        arr(grad_out), arr(grad_in),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        ctypes.c_void_p(aligned)), "brahms_adjoint")
        self.adjoint_workspace = ws
        return out

    def timing_enable(self, enable: bool = True):
        _check(self._lib.brahms_timing_enable(self._h, 1 if enable else 0), "brahms_timing_enable")

    def timing_read(self):
        """{kind: (summed ms, launches)} for kinds x, y, t, tables; clears."""
        ms = (ctypes.c_double * TIMING_KINDS)()
        cnt = (ctypes.c_longlong * TIMING_KINDS)()
        _check(self._lib.brahms_timing_read(self._h, ms, cnt), "brahms_timing_read")
        return {name: (ms[k], int(cnt[k])) for k, name in enumerate(TIMING_NAMES)}

    # -- diagnostics (Sec. 6 outputs) ------------------------------------
    def record_size(self) -> int:
        n = ctypes.c_int()
        _check(self._lib.brahms_record_size(self._h, ctypes.byref(n)), "brahms_record_size")
        return int(n.value)

    def split_records(self, rec: torch.Tensor) -> dict:
        """Split [k, record_size] float64 records into their parts (a view of
        the layout documented at brahms_record_size in include/brahms.h)."""
        rec = rec.reshape(-1, self.record_size()).cpu()
        nf, nt = self.nf, self.nt
        return {"step": rec[:, 0].to(torch.int64),
                "power": rec[:, 1:1 + nf * nt].reshape(-1, nf, nt),
                "energy": rec[:, 1 + nf * nt:1 + nf * (nt + 1)],
                "manley_rowe": rec[:, 1 + nf * (nt + 1):1 + nf * (nt + 1) + (3 if nf == 3 else 1)]}

    def diagnose_into(self, rec: torch.Tensor):
        """Write one record of the fields now into the float64 device tensor
        `rec` (record_size() entries), asynchronously."""
        if rec.dtype != torch.float64 or not rec.is_cuda or rec.numel() < self.record_size():
            raise ValueError("rec must be a float64 CUDA tensor of record_size() entries")
        _check(self._lib.brahms_diagnose(self._h, ctypes.c_void_p(rec.data_ptr())), "brahms_diagnose")

    def diagnose(self) -> dict:
        """Power traces, energies and Manley-Rowe values of the fields now."""
        rec = torch.empty(self.record_size(), dtype=torch.float64, device=self.fields[0].device)
        self.diagnose_into(rec)
        return {k: v[0] for k, v in self.split_records(rec).items()}

    def set_monitor(self, every: int, capacity: int = 0):
        """Record diagnostics whenever a completed step index is a multiple of
        `every` (at most `capacity` records); every = 0 switches it off."""
        if every > 0:
            self._monitor = torch.zeros(capacity, self.record_size(), dtype=torch.float64,
                                        device=self.fields[0].device)
            ptr = ctypes.c_void_p(self._monitor.data_ptr())
        else:
            self._monitor, ptr, capacity = None, ctypes.c_void_p(), 0
        _check(self._lib.brahms_set_monitor(self._h, every, ptr, capacity), "brahms_set_monitor")

    def monitor_records(self) -> dict:
        n = ctypes.c_int()
        _check(self._lib.brahms_get_monitor_count(self._h, ctypes.byref(n)), "brahms_get_monitor_count")
        if self._monitor is None or n.value == 0:
            return self.split_records(torch.zeros(0, self.record_size(), dtype=torch.float64))
        return self.split_records(self._monitor[:n.value])

    def set_snapshots(self, steps: Sequence[int]) -> List[List[torch.Tensor]]:
        """Copy the fields into new device tensors when each of `steps` (step
        indices >= 1) is completed; returns those tensors."""
        steps = [int(s) for s in steps]
        dev = self.fields[0].device
        self._snapshots = [[torch.zeros(self.nt, self.ny, self.nx, dtype=torch.complex64, device=dev)
                            for _ in range(self.nf)] for _ in steps]
        ptrs = (ctypes.c_void_p * max(1, len(steps) * self.nf))(
            *[t.data_ptr() for snap in self._snapshots for t in snap])
        arr = (ctypes.c_longlong * max(1, len(steps)))(*steps)
        _check(self._lib.brahms_set_snapshots(self._h, len(steps), arr, ptrs), "brahms_set_snapshots")
        return self._snapshots

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._lib.brahms_plan_destroy(self._h), "brahms_plan_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def run_workload(wl, nsteps: Optional[int] = None, device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None,
                 pass_order: Optional[int] = None,
                 merge_halves: int = 0, fuse_steps: int = 0, split: int = 0,
                 wide: int = 0) -> List[torch.Tensor]:
    """Upload a seeded workload's entrance fields, propagate nsteps (default:
    all of them) and return the device fields."""
    nsteps = wl.nz if nsteps is None else nsteps
    fields = [torch.from_numpy(a).to(device) for a in wl.init]
    plan = Plan(wl.nx, wl.ny, wl.nt, wl.nf, params_from_workload(wl), stream=stream)
    if pass_order is not None or merge_halves or split or wide:
        plan.set_schedule(pass_order or 0, 0, merge_halves, fuse_steps, split, wide)
    plan.bind(fields)
    plan.step(nsteps)
    torch.cuda.synchronize()
    plan.destroy()
    return fields


class Batch:
    """brahms_batch: many independent problems propagated together.

    problems: sequence of (nx, ny, nt, nf, Params, nsteps).  Every run
    propagates problem i nsteps[i] steps from z = 0.
    """

    def __init__(self, problems, stream: Optional[torch.cuda.Stream] = None):
        self._lib = load_library()
        self.stream = stream
        self.problems = list(problems)
        n = len(self.problems)
        shapes = (ctypes.c_int * (4 * n))()
        params = (ParamsC * n)()
        steps = (ctypes.c_int * n)()
        self._keep = []
        for k, (nx, ny, nt, nf, prm, ns) in enumerate(self.problems):
            shapes[4 * k: 4 * k + 4] = [nx, ny, nt, nf]
            c, keep = _params_c(prm, nf)
            params[k] = c
            self._keep.append(keep)
            steps[k] = int(ns)
        handle = ctypes.c_void_p()
        sptr = ctypes.c_void_p(stream.cuda_stream if stream is not None else
                               (torch.cuda.current_stream().cuda_stream
                                if torch.cuda.is_available() else 0))
        _check(self._lib.brahms_batch_create(n, shapes, params, steps, sptr, ctypes.byref(handle)),
               "brahms_batch_create")
        self._h = handle
        self.workspace = None
        self.fields = None

    def set_schedule(self, group_max: int = 0, pass_orders: Optional[Sequence[int]] = None):
        arr = None
        if pass_orders is not None:
            arr = (ctypes.c_int * len(self.problems))(*[int(v) for v in pass_orders])
        _check(self._lib.brahms_batch_set_schedule(self._h, int(group_max), arr),
               "brahms_batch_set_schedule")
        if self.fields is not None:
            self.bind(self.fields)

    def set_merge_halves(self, merge_halves: int):
        """1: merged RK4 half-steps for every problem (constant dk only)."""
        _check(self._lib.brahms_batch_set_merge_halves(self._h, int(merge_halves)),
               "brahms_batch_set_merge_halves")
        if self.fields is not None:
            self.bind(self.fields)

    def set_fuse_steps(self, fuse_steps: int):
        """1: fused step pairs for the launch groups of three-pass steps
        (needs merged half-steps)."""
        _check(self._lib.brahms_batch_set_fuse_steps(self._h, int(fuse_steps)),
               "brahms_batch_set_fuse_steps")
        if self.fields is not None:
            self.bind(self.fields)

    def set_group_limits(self, limits: Optional[Sequence[int]]):
        """Per-problem launch-group sizes (0: from the cache budget), or None."""
        arr = None
        if limits is not None:
            arr = (ctypes.c_int * len(self.problems))(*[int(v) for v in limits])
        _check(self._lib.brahms_batch_set_group_limits(self._h, arr), "brahms_batch_set_group_limits")
        if self.fields is not None:
            self.bind(self.fields)

    def set_splits(self, splits: Optional[Sequence[int]]):
        """Per-problem register/lane splits (bits x = 1, y = 2, tau = 4), or None."""
        arr = None
        if splits is not None:
            arr = (ctypes.c_int * len(self.problems))(*[int(v) for v in splits])
        _check(self._lib.brahms_batch_set_splits(self._h, arr), "brahms_batch_set_splits")
        if self.fields is not None:
            self.bind(self.fields)

    def set_wide(self, wide: Optional[Sequence[int]]):
        """Per-problem 512-thread blocks for the linear x and y passes (bits
        x = 1, y = 2), or None."""
        arr = None
        if wide is not None:
            arr = (ctypes.c_int * len(self.problems))(*[int(v) for v in wide])
        _check(self._lib.brahms_batch_set_wide(self._h, arr), "brahms_batch_set_wide")
        if self.fields is not None:
            self.bind(self.fields)

    def set_streams(self, streams: int, largest_alone: int = 0):
        """1: the run is one captured hipGraph (groups in sequence); 2-4:
        the run goes to that many streams, each replaying a linear graph of
        its own groups, so that launch groups of different shapes execute at
        the same time (with largest_alone, all but the largest group, which
        then runs alone)."""
        _check(self._lib.brahms_batch_set_streams(self._h, int(streams), int(largest_alone)),
               "brahms_batch_set_streams")

    def workspace_bytes(self) -> int:
        out = ctypes.c_size_t()
        _check(self._lib.brahms_batch_workspace_size(self._h, ctypes.byref(out)),
               "brahms_batch_workspace_size")
        return int(out.value)

    def bind(self, fields):
        """fields: one list of nf complex64 CUDA tensors [nt, ny, nx] per problem."""
        ptrs = []
        for (nx, ny, nt, nf, _, _), fs in zip(self.problems, fields):
            if len(fs) != nf:
                raise ValueError("wrong number of fields for a problem")
            for f in fs:
                if (f.dtype != torch.complex64 or not f.is_cuda or not f.is_contiguous()
                        or tuple(f.shape) != (nt, ny, nx)):
                    raise ValueError("fields must be contiguous complex64 CUDA tensors [nt, ny, nx]")
                ptrs.append(f.data_ptr())
        nbytes = self.workspace_bytes()
        if self.workspace is None or self.workspace.numel() < nbytes + 256:
            self.workspace = _device_bytes(nbytes + 256, fields[0][0].device, self.stream)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
        _check(self._lib.brahms_batch_bind(self._h, arr, ctypes.c_void_p(aligned)), "brahms_batch_bind")
        self.fields = [list(fs) for fs in fields]
        return self

    def run(self, nsteps: Optional[Sequence[int]] = None):
        """Propagate every problem from z = 0: nsteps[i] steps (each at most
        the count given at creation), or the counts given at creation."""
        if nsteps is None:
            _check(self._lib.brahms_batch_run(self._h), "brahms_batch_run")
        else:
            arr = (ctypes.c_int * len(self.problems))(*[int(v) for v in nsteps])
            _check(self._lib.brahms_batch_run_steps(self._h, arr), "brahms_batch_run_steps")

    def groups(self):
        n = ctypes.c_int()
        _check(self._lib.brahms_batch_groups(self._h, ctypes.byref(n), None), "brahms_batch_groups")
        arr = (ctypes.c_int * max(1, n.value))()
        _check(self._lib.brahms_batch_groups(self._h, ctypes.byref(n), arr), "brahms_batch_groups")
        return [arr[k] for k in range(n.value)]

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._lib.brahms_batch_destroy(self._h), "brahms_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
