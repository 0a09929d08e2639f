"""ctypes loader for libdcp.so (the C ABI declared in include/dcp.h).

The library is required: there is no CPU fallback.  If it is missing the
first call raises with instructions to build it.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcp.so")

# enums of include/dcp.h
DCP_OK = 0
F64, F32 = 0, 1
DIRICHLET0, PERIODIC = 0, 1
FUSED, UNFUSED = 0, 1
OP_STEP_FUSED, OP_STEP_UNFUSED, OP_RUN, OP_ADJOINT = 0, 1, 2, 3
E_SCRATCH = -8
NOALLOC_SCRATCH_BYTES = 1 << 20  # DCP_NOALLOC_SCRATCH_BYTES


class Coeffs(ctypes.Structure):
    """dcp_coeffs: the scalars of the program (h is the grid spacing)."""
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("h", ctypes.c_double),
                ("dt", ctypes.c_double)]

    @classmethod
    def make(cls, c) -> "Coeffs":
        if isinstance(c, Coeffs):
            return c
        return cls(float(c["alpha"]), float(c["beta"]), float(c["gamma"]),
                   float(c["h"]), float(c["dt"]))

    def as_dict(self) -> dict:
        return dict(alpha=self.alpha, beta=self.beta, gamma=self.gamma, h=self.h, dt=self.dt)


class RunInfo(ctypes.Structure):
    """dcp_run_info: the passes a dcp_run takes."""
    _fields_ = [("passes", ctypes.c_int32 * 3), ("steps_per_pass", ctypes.c_int32),
                ("segmented", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("lanes", ctypes.c_int32)]


class DcpError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: {msg} (status {status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_2107_00555_amd.build` "
            "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    dp = ctypes.c_void_p  # device double* passed as an address
    cp = ctypes.POINTER(Coeffs)
    sz = ctypes.c_size_t
    L.dcp_workspace_bytes.argtypes = [c_int, c_int, c_int, i64, i64, i64, i32, i32, i32, c_int,
                                      ctypes.POINTER(sz)]
    L.dcp_workspace_bytes.restype = c_int
    step_args = [c_int, vp, vp, vp, i64, i64, i64, cp, c_int, dp, vp, sz, vp]
    L.dcp_step_fused.argtypes = step_args
    L.dcp_step_fused.restype = c_int
    L.dcp_step_unfused.argtypes = step_args
    L.dcp_step_unfused.restype = c_int
    L.dcp_step_fused_noalloc.argtypes = [c_int, vp, vp, vp, i64, i64, i64, cp, c_int, dp, vp]
    L.dcp_step_fused_noalloc.restype = c_int
    L.dcp_run.argtypes = [c_int, c_int, vp, vp, i64, i64, i64, cp, c_int, i32, i32, dp, dp, vp, i32,
                          vp, sz, vp]
    L.dcp_run.restype = c_int
    L.dcp_run_plan.argtypes = [c_int, c_int, i64, i64, i64, i32, i32, c_int, ctypes.POINTER(RunInfo)]
    L.dcp_run_plan.restype = c_int
    L.dcp_adjoint_run.argtypes = [c_int, vp, i32, vp, vp, i64, i64, i64, cp, c_int, i32, i32, vp, dp,
                                  vp, dp, vp, sz, vp]
    L.dcp_adjoint_run.restype = c_int
    L.dcp_status_string.argtypes = [c_int]
    L.dcp_status_string.restype = ctypes.c_char_p
    L.dcp_max_tblock.argtypes = [c_int]
    L.dcp_max_tblock.restype = i32
    L.dcp_jacobi_workspace_bytes.argtypes = [c_int, i64, i64, i32, i32, ctypes.POINTER(sz)]
    L.dcp_jacobi_workspace_bytes.restype = c_int
    L.dcp_revolve_workspace_bytes.argtypes = [c_int, i64, i64, i64, i32, i32, c_int, ctypes.POINTER(sz)]
    L.dcp_revolve_workspace_bytes.restype = c_int
    L.dcp_revolve_forward.argtypes = [c_int, vp, vp, i64, i64, i64, cp, c_int, i32, i32, i32, vp, sz, vp]
    L.dcp_revolve_forward.restype = c_int
    L.dcp_revolve_adjoint.argtypes = [c_int, vp, vp, i64, i64, i64, cp, c_int, i32, i32, i32, vp, dp, vp, dp,
                                      vp, sz, vp]
    L.dcp_revolve_adjoint.restype = c_int
    i64p = ctypes.POINTER(i64)
    L.dcp_revolve_schedule.argtypes = [i64, i32, i64p, i64, i64p, i64p]
    L.dcp_revolve_schedule.restype = c_int
    L.dcp_jacobi_plan.argtypes = [c_int, i64, i64, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.dcp_jacobi_plan.restype = c_int
    L.dcp_jacobi_1d.argtypes = [i32, vp, vp, i64, i32, vp, sz, vp]
    L.dcp_jacobi_1d.restype = c_int
    L.dcp_jacobi_2d.argtypes = [i32, vp, vp, i64, i64, i32, vp, sz, vp]
    L.dcp_jacobi_2d.restype = c_int
    L.dcp_stream_probe.argtypes = [c_int, c_int, vp, vp, vp, sz, vp]
    L.dcp_stream_probe.restype = c_int
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != DCP_OK:
        raise DcpError(fn, status, lib().dcp_status_string(status).decode())


def workspace_bytes(op: int, dtype: int, nx: int, ny: int, nz: int, T: int = 0,
                    ckpt_every: int = 1, tblock: int = 1, norms: bool = False,
                    impl: int = FUSED) -> int:
    out = ctypes.c_size_t(0)
    check("dcp_workspace_bytes",
          lib().dcp_workspace_bytes(op, dtype, impl, nx, ny, nz, T, ckpt_every, tblock,
                                    int(bool(norms)), ctypes.byref(out)))
    return out.value


def run_plan(dtype: int, nx: int, ny: int, nz: int, T: int, tblock: int, norms: bool = True,
             impl: int = FUSED) -> dict:
    """The passes dcp_run takes for these arguments (16-byte aligned fields):
    {'passes': [one-step, two-step, three-step], 'steps_per_pass',
    'segmented', 'tile_rows', 'lanes'}."""
    info = RunInfo()
    check("dcp_run_plan", lib().dcp_run_plan(dtype, impl, nx, ny, nz, T, tblock, int(bool(norms)),
                                             ctypes.byref(info)))
    return {"passes": list(info.passes), "steps_per_pass": info.steps_per_pass, "segmented": info.segmented,
            "tile_rows": info.tile_rows, "lanes": info.lanes}


def jacobi_workspace_bytes(dims: int, n0: int, n1: int, tsteps: int, tblock: int = 0) -> int:
    out = ctypes.c_size_t(0)
    check("dcp_jacobi_workspace_bytes",
          lib().dcp_jacobi_workspace_bytes(dims, n0, n1, tsteps, tblock, ctypes.byref(out)))
    return out.value


def jacobi_plan(dims: int, n0: int, n1: int, tsteps: int, tblock: int = 0) -> tuple[int, int]:
    """(passes over memory, most half-steps in one pass) of a Jacobi call."""
    passes, halo = ctypes.c_int64(0), ctypes.c_int32(0)
    check("dcp_jacobi_plan",
          lib().dcp_jacobi_plan(dims, n0, n1, tsteps, tblock, ctypes.byref(passes), ctypes.byref(halo)))
    return passes.value, halo.value


def revolve_schedule(T: int, nslots: int):
    """(ops as a list of (kind, src, dst, t0, t1), forward steps) of the
    binomial checkpointing schedule (see dcp.h)."""
    n, fwd = ctypes.c_int64(0), ctypes.c_int64(0)
    check("dcp_revolve_schedule", lib().dcp_revolve_schedule(T, nslots, None, 0, ctypes.byref(n),
                                                              ctypes.byref(fwd)))
    buf = (ctypes.c_int64 * (5 * max(n.value, 1)))()
    check("dcp_revolve_schedule", lib().dcp_revolve_schedule(T, nslots, buf, n.value, ctypes.byref(n),
                                                              ctypes.byref(fwd)))
    ops = [tuple(buf[5 * i:5 * i + 5]) for i in range(n.value)]
    return ops, fwd.value


def revolve_workspace_bytes(dtype: int, nx: int, ny: int, nz: int, T: int, nslots: int,
                            lsum_field: bool = False) -> int:
    out = ctypes.c_size_t(0)
    check("dcp_revolve_workspace_bytes",
          lib().dcp_revolve_workspace_bytes(dtype, nx, ny, nz, T, nslots, int(bool(lsum_field)),
                                            ctypes.byref(out)))
    return out.value
