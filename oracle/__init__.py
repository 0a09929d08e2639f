"""Plain serial FP64 CPU oracle for the reaction-diffusion array program and
for the two Jacobi stencil programs the paper lists.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
does, and this package imports nothing from it.  The arithmetic lives in
``rd3d_oracle.c`` and ``jacobi_oracle.c`` (built with gcc, no FMA
contraction); this module only marshals NumPy arrays into them.  Where each function comes from in the paper
is stated in the C source.

Reaction-diffusion arrays are float64, C-contiguous, shape ``(nz, ny, nx)``
(x fastest); boundary modes: 0 = ghost-zero Dirichlet, 1 = periodic.
Jacobi arrays are float64 vectors (1D) or C-order (n0, n1) matrices (2D).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "rd3d_oracle.c"), os.path.join(_HERE, "jacobi_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
# void cb(int t, const double *u_t, double e_t, double r_t, void *ctx)
_STEP_CB = ctypes.CFUNCTYPE(None, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                            ctypes.c_double, ctypes.c_void_p)

DIRICHLET0 = 0
PERIODIC = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (serial, -O3, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c11", "-O3", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, *_SRCS, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        i64p = ctypes.POINTER(ctypes.c_int64)
        d = ctypes.c_double
        lib.oracle_run.argtypes = [i64, i64, i64, dp, dp, d, d, d, d, d,
                                   ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_run_stream.argtypes = [i64, i64, i64, dp, dp, d, d, d, d, d,
                                          ctypes.c_int, ctypes.c_int, _STEP_CB, ctypes.c_void_p]
        lib.oracle_run_stream.restype = ctypes.c_int
        lib.oracle_run_box.argtypes = [i64, i64, i64, dp, dp, d, d, d, d, d,
                                       ctypes.c_int, ctypes.c_int, i64p, i64p, dp]
        lib.oracle_run_box.restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = [i64, i64, i64, dp, dp, dp, d, d, d, d, d,
                                       ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        lib.oracle_adjoint.restype = ctypes.c_int
        lib.oracle_half_sq_dist.argtypes = [i64, dp, dp]
        lib.oracle_half_sq_dist.restype = d
        i32 = ctypes.c_int32
        lib.oracle_jacobi_1d_box.argtypes = [i32, i64, i64, i64, dp, dp]
        lib.oracle_jacobi_1d_box.restype = ctypes.c_int
        lib.oracle_jacobi_2d_box.argtypes = [i32, i64, i64, i64, i64, i64, i64, dp, dp]
        lib.oracle_jacobi_2d_box.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("fields are 3-D arrays shaped (nz, ny, nx)")
    return a


def _coeffs(c):
    return (float(c["alpha"]), float(c["beta"]), float(c["gamma"]),
            float(c["h"]), float(c["dt"]))


def run(u0, f, coeffs: dict, T: int, bc: int, norms: bool = True):
    """T steps on the whole grid.

    Returns ``(u_T, energy[T], resid[T])`` where energy[t-1] = sum u_t^2 and
    resid[t-1] = ||u_t - u_{t-1}||_2 for t = 1..T.
    """
    u0 = _field(u0)
    f = _field(f)
    if f.shape != u0.shape:
        raise ValueError("u0 and f must have the same shape")
    nz, ny, nx = u0.shape
    uT = np.empty_like(u0)
    e = np.empty(max(T, 0), dtype=np.float64)
    r = np.empty(max(T, 0), dtype=np.float64)
    rc = _load().oracle_run(nx, ny, nz, _ptr(u0), _ptr(f), *_coeffs(coeffs),
                            int(bc), int(T), _ptr(uT),
                            _ptr(e) if norms else None, _ptr(r) if norms else None)
    if rc != 0:
        raise ValueError(f"oracle_run failed with code {rc}")
    return uT, e, r


def run_stream(u0, f, coeffs: dict, T: int, bc: int, observe) -> None:
    """The same T steps as run(), calling ``observe(t, u_t, E_t, R_t)`` after
    every step t = 1..T.  ``u_t`` is a read-only view of the oracle's own
    buffer, valid during the call only (copy it to keep it).  An exception
    raised by ``observe`` is re-raised once the run has finished."""
    u0 = _field(u0)
    f = _field(f)
    if f.shape != u0.shape:
        raise ValueError("u0 and f must have the same shape")
    shape = u0.shape
    errors = []

    def _cb(t, p, e, r, _ctx):
        if errors:
            return
        try:
            view = np.ctypeslib.as_array(p, shape=shape)
            view.flags.writeable = False
            observe(int(t), view, float(e), float(r))
        except BaseException as exc:  # noqa: BLE001 -- handed back to the caller
            errors.append(exc)

    cb = _STEP_CB(_cb)
    nz, ny, nx = shape
    rc = _load().oracle_run_stream(nx, ny, nz, _ptr(u0), _ptr(f), *_coeffs(coeffs),
                                   int(bc), int(T), cb, None)
    if errors:
        raise errors[0]
    if rc != 0:
        raise ValueError(f"oracle_run_stream failed with code {rc}")


def run_box(u0, f, coeffs: dict, T: int, bc: int, lo, hi) -> np.ndarray:
    """u_T on the box [lo, hi) given as (x, y, z) triples; returns (hz, hy, hx)."""
    u0 = _field(u0)
    f = _field(f)
    nz, ny, nx = u0.shape
    blo = (ctypes.c_int64 * 3)(*[int(v) for v in lo])
    bhi = (ctypes.c_int64 * 3)(*[int(v) for v in hi])
    shape = (int(hi[2]) - int(lo[2]), int(hi[1]) - int(lo[1]), int(hi[0]) - int(lo[0]))
    out = np.empty(shape, dtype=np.float64)
    rc = _load().oracle_run_box(nx, ny, nz, _ptr(u0), _ptr(f), *_coeffs(coeffs),
                                int(bc), int(T), blo, bhi, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_run_box failed with code {rc}")
    return out


def adjoint(u0, f, lam_T, coeffs: dict, T: int, bc: int):
    """Gradient through T steps given the seed lam_T = dL/du_T.

    Returns ``(dL/du0, dL/dalpha, dL/dbeta)``.
    """
    r = adjoint_full(u0, f, lam_T, coeffs, T, bc)
    return r["u0"], r["alpha"], r["beta"]


def adjoint_full(u0, f, lam_T, coeffs: dict, T: int, bc: int) -> dict:
    """Every gradient through T steps given lam_T = dL/du_T: a dict with
    'u0', 'f' (fields) and 'alpha', 'beta', 'gamma' (floats)."""
    u0 = _field(u0)
    f = _field(f)
    lam_T = _field(lam_T)
    nz, ny, nx = u0.shape
    g = np.empty_like(u0)
    gf = np.empty_like(u0)
    gab = np.empty(2, dtype=np.float64)
    gg = np.empty(1, dtype=np.float64)
    rc = _load().oracle_adjoint(nx, ny, nz, _ptr(u0), _ptr(f), _ptr(lam_T),
                                *_coeffs(coeffs), int(bc), int(T), _ptr(g), _ptr(gab),
                                _ptr(gf), _ptr(gg))
    if rc != 0:
        raise ValueError(f"oracle_adjoint failed with code {rc}")
    return {"u0": g, "f": gf, "alpha": float(gab[0]), "beta": float(gab[1]), "gamma": float(gg[0])}


def half_sq_dist(a, b) -> float:
    """0.5 * sum (a - b)^2 with a compensated sum (the config loss)."""
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    return float(_load().oracle_half_sq_dist(a.size, _ptr(a), _ptr(b)))


def grad_of_half_sq_dist(u0, f, u_tgt, coeffs: dict, T: int, bc: int):
    """Loss L = 0.5*||u_T - u_tgt||^2 and its gradient (dL/du0, dL/dalpha, dL/dbeta)."""
    uT, _, _ = run(u0, f, coeffs, T, bc, norms=False)
    loss = half_sq_dist(uT, u_tgt)
    lam_T = uT - _field(u_tgt)
    g, ga, gb = adjoint(u0, f, lam_T, coeffs, T, bc)
    return loss, g, ga, gb


def _vec(a, ndim: int) -> np.ndarray:
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    if a.ndim != ndim:
        raise ValueError(f"expected a {ndim}-D array, got shape {a.shape}")
    return a


def jacobi_1d(tsteps: int, A, B):
    """The jacobi_1d listing (Sec. 2.2) on copies of A and B; returns (A, B)."""
    A = _vec(A, 1)
    B = _vec(B, 1)
    if A.shape != B.shape:
        raise ValueError("A and B must have the same length")
    return jacobi_1d_box(tsteps, A.size, 0, A, B)


def jacobi_1d_box(tsteps: int, n: int, c0: int, A, B):
    """The window [c0, c0+len(A)) of a length-n jacobi_1d run (see the C
    source for which cells are exact); works on copies, returns (A, B)."""
    A = _vec(A, 1)
    B = _vec(B, 1)
    if A.shape != B.shape:
        raise ValueError("A and B must have the same length")
    rc = _load().oracle_jacobi_1d_box(int(tsteps), int(n), int(c0), A.size, _ptr(A), _ptr(B))
    if rc != 0:
        raise ValueError(f"oracle_jacobi_1d_box failed with code {rc}")
    return A, B


def jacobi_2d(tsteps: int, A, B):
    """The jacobi_2d listing (Sec. 4.3) on copies of A and B; returns (A, B)."""
    A = _vec(A, 2)
    B = _vec(B, 2)
    if A.shape != B.shape:
        raise ValueError("A and B must have the same shape")
    return jacobi_2d_box(tsteps, A.shape[0], A.shape[1], 0, 0, A, B)


def jacobi_2d_box(tsteps: int, n0: int, n1: int, r0: int, c0: int, A, B):
    """The window starting at (r0, c0) of an n0 x n1 jacobi_2d run; works on
    copies, returns (A, B)."""
    A = _vec(A, 2)
    B = _vec(B, 2)
    if A.shape != B.shape:
        raise ValueError("A and B must have the same shape")
    h0, h1 = A.shape
    rc = _load().oracle_jacobi_2d_box(int(tsteps), int(n0), int(n1), int(r0), int(c0), h0, h1,
                                      _ptr(A), _ptr(B))
    if rc != 0:
        raise ValueError(f"oracle_jacobi_2d_box failed with code {rc}")
    return A, B
