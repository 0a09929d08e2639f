"""torch-facing binding of libdcp: argument marshalling only.

Fields are CUDA (HIP) tensors of dtype float64 or float32, contiguous, shaped
(nz, ny, nx) -- x is the fastest axis, as in the C ABI.  Every call enqueues
its work on the current torch stream and returns without synchronising;
scratch memory comes from torch's allocator as a uint8 workspace tensor.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (DIRICHLET0, F32, F64, FUSED, OP_ADJOINT, OP_RUN, OP_STEP_FUSED,
                   OP_STEP_UNFUSED, PERIODIC, UNFUSED, Coeffs, DcpError)

__all__ = ["Coeffs", "DcpError", "DIRICHLET0", "PERIODIC", "FUSED", "UNFUSED",
           "step", "step_noalloc", "run", "adjoint_run", "workspace", "num_slots", "bc_code", "impl_code",
           "jacobi_1d", "jacobi_2d", "revolve_forward", "revolve_adjoint"]


def bc_code(bc) -> int:
    if isinstance(bc, str):
        return {"dirichlet0": DIRICHLET0, "dirichlet": DIRICHLET0, "periodic": PERIODIC}[bc.lower()]
    return int(bc)


def impl_code(impl) -> int:
    if isinstance(impl, str):
        return {"fused": FUSED, "unfused": UNFUSED}[impl.lower()]
    return int(impl)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"fields must be float64 or float32, got {t.dtype}")


def _field(name: str, t: torch.Tensor, like: torch.Tensor | None = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got device {t.device})")
    if t.dim() != 3:
        raise ValueError(f"{name} must be 3-D shaped (nz, ny, nx), got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if like is not None:
        if t.shape != like.shape or t.dtype != like.dtype or t.device != like.device:
            raise ValueError(f"{name} must match shape/dtype/device of the state field")
    return t


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _ws(ws, nbytes: int, device) -> torch.Tensor | None:
    """The caller's workspace if it is a contiguous tensor on the device with
    at least nbytes bytes, else a new one."""
    if (isinstance(ws, torch.Tensor) and ws.device == torch.device(device) and ws.is_contiguous()
            and ws.numel() * ws.element_size() >= nbytes):
        return ws
    return workspace(nbytes, device)


def num_slots(T: int, k: int) -> int:
    return 0 if T <= 0 else (T + k - 1) // k


def check_ckpt(ckpt, T: int, k: int, like: torch.Tensor) -> torch.Tensor:
    """The checkpoint store of a T-step run with a checkpoint every k steps:
    a contiguous tensor of num_slots(T, k) fields shaped like `like` (the
    state), with its dtype and on its device.  The library writes (dcp_run)
    or reads (dcp_adjoint_run) exactly that many fields through the pointer,
    so anything smaller, or of another element type, is refused here."""
    if not isinstance(ckpt, torch.Tensor):
        raise TypeError("ckpt must be a torch tensor")
    if k < 1:
        raise ValueError(f"ckpt_every must be >= 1 when a checkpoint store is used, got {k}")
    want = (num_slots(T, k),) + tuple(like.shape)
    if tuple(ckpt.shape) != want:
        raise ValueError(f"ckpt must be shaped {want} (ceil(T/k) fields), got {tuple(ckpt.shape)}")
    if ckpt.dtype != like.dtype:
        raise ValueError(f"ckpt must have the state's dtype {like.dtype}, got {ckpt.dtype}")
    if ckpt.device != like.device:
        raise ValueError(f"ckpt must be on the state's device {like.device}, got {ckpt.device}")
    if not ckpt.is_contiguous():
        raise ValueError("ckpt must be contiguous")
    return ckpt


def step(u: torch.Tensor, f: torch.Tensor, coeffs, bc, impl="fused", norms: bool = False,
         out: torch.Tensor | None = None):
    """One step u -> u_out.  Returns (u_out, norms2) where norms2 is a float64
    tensor {sum u_out^2, sum (u_out-u)^2} or None."""
    u = _field("u", u)
    f = _field("f", f, u)
    if out is None:
        out = torch.empty_like(u)
    else:
        _field("out", out, u)
    dt = _dtype_code(u)
    nz, ny, nx = u.shape
    c = Coeffs.make(coeffs)
    ic = impl_code(impl)
    op = OP_STEP_FUSED if ic == FUSED else OP_STEP_UNFUSED
    wsb = _lib.workspace_bytes(op, dt, nx, ny, nz, norms=norms)
    ws = workspace(wsb, u.device)
    n2 = torch.empty(2, dtype=torch.float64, device=u.device) if norms else None
    fn = _lib.lib().dcp_step_fused if ic == FUSED else _lib.lib().dcp_step_unfused
    with torch.cuda.device(u.device):
        _lib.check(fn.__name__, fn(dt, _ptr(u), _ptr(f), _ptr(out), nx, ny, nz, ctypes.byref(c),
                                   bc_code(bc), _ptr(n2), _ptr(ws), wsb, _stream(u.device)))
    return out, n2


def step_noalloc(u: torch.Tensor, f: torch.Tensor, coeffs, bc, out: torch.Tensor,
                 norms2: torch.Tensor | None = None) -> None:
    """One fused step u -> out through dcp_step_fused_noalloc: the caller
    passes every buffer (out, and norms2 as a float64 tensor of 2 elements
    when the norms are wanted) and neither this function nor the library
    allocates device memory; the norms' partial sums use the library's
    fixed per-GPU scratch (calls overlapping on one GPU race)."""
    u = _field("u", u)
    f = _field("f", f, u)
    _field("out", out, u)
    if norms2 is not None:
        if (not isinstance(norms2, torch.Tensor) or norms2.dtype != torch.float64 or norms2.numel() != 2
                or norms2.device != u.device or not norms2.is_contiguous()):
            raise ValueError("norms2 must be a contiguous float64 tensor of 2 elements on u's device")
    dt = _dtype_code(u)
    nz, ny, nx = u.shape
    c = Coeffs.make(coeffs)
    with torch.cuda.device(u.device):
        _lib.check("dcp_step_fused_noalloc", _lib.lib().dcp_step_fused_noalloc(
            dt, _ptr(u), _ptr(f), _ptr(out), nx, ny, nz, ctypes.byref(c), bc_code(bc), _ptr(norms2),
            _stream(u.device)))


def run(u: torch.Tensor, f: torch.Tensor, coeffs, T: int, bc, impl="fused", tblock: int | None = None,
        norms: bool = True, ckpt_every: int = 0, ws: torch.Tensor | None = None,
        ckpt: torch.Tensor | None = None):
    """T steps in place on u.  Returns a dict with 'energy' and 'resid'
    (float64 [T] tensors, or None) and 'ckpt' (tensor of ceil(T/k) fields
    shaped (slots, nz, ny, nx), or None when ckpt_every == 0).  tblock
    defaults to 3 (up to three steps per pass where the grid allows it) for
    the fused form and 1 for the unfused one."""
    u = _field("u", u)
    f = _field("f", f, u)
    dt = _dtype_code(u)
    nz, ny, nx = u.shape
    c = Coeffs.make(coeffs)
    ic = impl_code(impl)
    if tblock is None:
        tblock = 3 if ic == FUSED else 1
    wsb = _lib.workspace_bytes(OP_RUN, dt, nx, ny, nz, T=T, tblock=tblock, norms=norms, impl=ic)
    ws = _ws(ws, wsb, u.device)
    energy = torch.empty(max(T, 0), dtype=torch.float64, device=u.device) if norms else None
    resid = torch.empty(max(T, 0), dtype=torch.float64, device=u.device) if norms else None
    if ckpt is not None:
        check_ckpt(ckpt, T, ckpt_every, u)
    elif ckpt_every:
        ckpt = torch.empty((num_slots(T, ckpt_every), nz, ny, nx), dtype=u.dtype, device=u.device)
    with torch.cuda.device(u.device):
        _lib.check("dcp_run", _lib.lib().dcp_run(
            dt, ic, _ptr(u), _ptr(f), nx, ny, nz, ctypes.byref(c), bc_code(bc), int(T), int(tblock),
            _ptr(energy), _ptr(resid), _ptr(ckpt), int(ckpt_every), _ptr(ws), wsb, _stream(u.device)))
    return {"energy": energy, "resid": resid, "ckpt": ckpt}


def adjoint_run(ckpt: torch.Tensor | None, ckpt_every: int, f: torch.Tensor, lam_T: torch.Tensor,
                coeffs, T: int, bc, tblock: int = 3, ws: torch.Tensor | None = None,
                grad_u0: torch.Tensor | None = None, want_f: bool = False, want_gamma: bool = False):
    """Gradient through T fused steps from dcp_run's checkpoints.
    Returns (dL/du0, float64 tensor [dL/dalpha, dL/dbeta]), or with
    want_f / want_gamma a dict with keys 'u0', 'ab', and 'f' / 'gamma'."""
    lam_T = _field("lam_T", lam_T)
    f = _field("f", f, lam_T)
    dt = _dtype_code(lam_T)
    nz, ny, nx = lam_T.shape
    if T > 0 and lam_T.numel() > 0:
        if ckpt is None:
            raise ValueError("ckpt (the checkpoints dcp_run wrote) is required for T > 0")
        check_ckpt(ckpt, T, ckpt_every, lam_T)
    c = Coeffs.make(coeffs)
    wsb = _lib.workspace_bytes(OP_ADJOINT, dt, nx, ny, nz, T=T, ckpt_every=ckpt_every, tblock=tblock,
                               norms=want_gamma and not want_f)
    ws = _ws(ws, wsb, lam_T.device)
    if grad_u0 is None:
        grad_u0 = torch.empty_like(lam_T)
    else:
        _field("grad_u0", grad_u0, lam_T)
    gab = torch.empty(2, dtype=torch.float64, device=lam_T.device)
    gf = torch.empty_like(lam_T) if want_f else None
    gg = torch.empty(1, dtype=torch.float64, device=lam_T.device) if want_gamma else None
    with torch.cuda.device(lam_T.device):
        _lib.check("dcp_adjoint_run", _lib.lib().dcp_adjoint_run(
            dt, _ptr(ckpt), int(ckpt_every), _ptr(f), _ptr(lam_T), nx, ny, nz, ctypes.byref(c),
            bc_code(bc), int(T), int(tblock), _ptr(grad_u0), _ptr(gab), _ptr(gf), _ptr(gg), _ptr(ws), wsb,
            _stream(lam_T.device)))
    if not (want_f or want_gamma):
        return grad_u0, gab
    out = {"u0": grad_u0, "ab": gab}
    if want_f:
        out["f"] = gf
    if want_gamma:
        out["gamma"] = gg[0]
    return out

def revolve_forward(u: torch.Tensor, f: torch.Tensor, coeffs, T: int, bc, nslots: int, tblock: int = 3,
                    reserve_sum: bool = False) -> torch.Tensor:
    """T steps in place on u with binomial checkpointing snapshots; returns
    the workspace tensor the matching revolve_adjoint call needs (keep it
    untouched).  reserve_sum: room for dL/dgamma without dL/df."""
    u = _field("u", u)
    f = _field("f", f, u)
    dt = _dtype_code(u)
    nz, ny, nx = u.shape
    c = Coeffs.make(coeffs)
    wsb = _lib.revolve_workspace_bytes(dt, nx, ny, nz, T, nslots, reserve_sum)
    ws = workspace(wsb, u.device)
    with torch.cuda.device(u.device):
        _lib.check("dcp_revolve_forward", _lib.lib().dcp_revolve_forward(
            dt, _ptr(u), _ptr(f), nx, ny, nz, ctypes.byref(c), bc_code(bc), int(T), int(nslots), int(tblock),
            _ptr(ws), wsb, _stream(u.device)))
    return ws if ws is not None else torch.empty(0, dtype=torch.uint8, device=u.device)


def revolve_adjoint(ws: torch.Tensor, f: torch.Tensor, lam_T: torch.Tensor, coeffs, T: int, bc, nslots: int,
                    tblock: int = 3, want_f: bool = False, want_gamma: bool = False):
    """The gradient from revolve_forward's workspace; returns like adjoint_run."""
    lam_T = _field("lam_T", lam_T)
    f = _field("f", f, lam_T)
    dt = _dtype_code(lam_T)
    nz, ny, nx = lam_T.shape
    c = Coeffs.make(coeffs)
    wsb = _lib.revolve_workspace_bytes(dt, nx, ny, nz, T, nslots, want_gamma and not want_f)
    if (not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8 or ws.device != lam_T.device
            or not ws.is_contiguous()):
        raise ValueError("ws must be the byte workspace revolve_forward returned, on lam_T's device")
    if ws.numel() < wsb:
        raise ValueError("workspace smaller than this call needs (reserve_sum in revolve_forward?)")
    grad_u0 = torch.empty_like(lam_T)
    gab = torch.empty(2, dtype=torch.float64, device=lam_T.device)
    gf = torch.empty_like(lam_T) if want_f else None
    gg = torch.empty(1, dtype=torch.float64, device=lam_T.device) if want_gamma else None
    with torch.cuda.device(lam_T.device):
        _lib.check("dcp_revolve_adjoint", _lib.lib().dcp_revolve_adjoint(
            dt, _ptr(f), _ptr(lam_T), nx, ny, nz, ctypes.byref(c), bc_code(bc), int(T), int(nslots), int(tblock),
            _ptr(grad_u0), _ptr(gab), _ptr(gf), _ptr(gg), _ptr(ws) if ws.numel() else None, ws.numel(),
            _stream(lam_T.device)))
    if not (want_f or want_gamma):
        return grad_u0, gab
    out = {"u0": grad_u0, "ab": gab}
    if want_f:
        out["f"] = gf
    if want_gamma:
        out["gamma"] = gg[0]
    return out

def _jacobi_arrays(A: torch.Tensor, B: torch.Tensor, dims: int):
    for name, t in (("A", A), ("B", B)):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be a GPU tensor (got device {t.device})")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64, got {t.dtype}")
        if t.dim() != dims:
            raise ValueError(f"{name} must be {dims}-D, got shape {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if A.shape != B.shape or A.device != B.device:
        raise ValueError("A and B must have the same shape and device")


def jacobi_1d(A: torch.Tensor, B: torch.Tensor, tsteps: int, tblock: int = 0,
              ws: torch.Tensor | None = None):
    """The jacobi_1d listing, in place on float64 vectors A and B."""
    _jacobi_arrays(A, B, 1)
    n = A.shape[0]
    wsb = _lib.jacobi_workspace_bytes(1, n, 1, tsteps, tblock)
    ws = _ws(ws, wsb, A.device)
    with torch.cuda.device(A.device):
        _lib.check("dcp_jacobi_1d", _lib.lib().dcp_jacobi_1d(
            int(tsteps), _ptr(A), _ptr(B), n, int(tblock), _ptr(ws), wsb, _stream(A.device)))
    return A, B


def jacobi_2d(A: torch.Tensor, B: torch.Tensor, tsteps: int, tblock: int = 0,
              ws: torch.Tensor | None = None):
    """The jacobi_2d listing, in place on float64 (n0, n1) arrays A and B."""
    _jacobi_arrays(A, B, 2)
    n0, n1 = A.shape
    wsb = _lib.jacobi_workspace_bytes(2, n0, n1, tsteps, tblock)
    ws = _ws(ws, wsb, A.device)
    with torch.cuda.device(A.device):
        _lib.check("dcp_jacobi_2d", _lib.lib().dcp_jacobi_2d(
            int(tsteps), _ptr(A), _ptr(B), n0, n1, int(tblock), _ptr(ws), wsb, _stream(A.device)))
    return A, B
