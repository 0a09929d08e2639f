"""Front end of the fusing compiler (dcp_fuse_* in include/dcp.h).

A Program records NumPy-style expressions over 3-D fields as single-operator
SSA statements, in Python's evaluation order (each operator one temporary,
the first translation pass of Sec. 2.3); the library partitions them into
fused kernels (Sec. 3.1), generates HIP for gfx950 and runs it.  This module
only builds the program text and marshals arguments.

    P = Program("f64")
    u, f = P.input("u", "f")
    a, = P.param("alpha")
    lap = lap7(u)                      # six shifted reads and a subtraction
    P.output("unew", u + a * lap + f)
    prog = P.compile()                 # fused; compile(fuse=False): one kernel per statement
    (unew,) = prog.run([u_t, f_t], {"alpha": 0.1}, bc="periodic")
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

__all__ = ["Program", "Fused", "lap7", "compile_text"]


class Expr:
    __slots__ = ("p", "name", "field")

    def __init__(self, p: "Program", name: str, field: bool):
        self.p, self.name, self.field = p, name, field

    def _bin(self, op, other, rev=False):
        a, b = (other, self) if rev else (self, other)
        return self.p._stmt(op, a, b)

    def __add__(self, o): return self._bin("add", o)
    def __radd__(self, o): return self._bin("add", o, True)
    def __sub__(self, o): return self._bin("sub", o)
    def __rsub__(self, o): return self._bin("sub", o, True)
    def __mul__(self, o): return self._bin("mul", o)
    def __rmul__(self, o): return self._bin("mul", o, True)
    def __truediv__(self, o): return self._bin("div", o)
    def __rtruediv__(self, o): return self._bin("div", o, True)
    def __neg__(self): return self.p._stmt("neg", self)

    def shift(self, dx: int = 0, dy: int = 0, dz: int = 0) -> "Expr":
        """This field read at (x+dx, y+dy, z+dz)."""
        if not self.field:
            raise TypeError("shift of a scalar")
        return self.p._stmt("shift", self, extra=f" {int(dx)} {int(dy)} {int(dz)}")


def lap7(u: Expr, h=None) -> Expr:
    """(u[x-1] + u[x+1] + u[y-1] + u[y+1] + u[z-1] + u[z+1] - 6u) / h^2,
    added left to right; without h, the sum times no factor.  h^2 is a
    statement of the program (a scalar product of two literals, rounded in
    the program's dtype like every other operation)."""
    s = u.shift(-1, 0, 0) + u.shift(1, 0, 0) + u.shift(0, -1, 0) + u.shift(0, 1, 0) \
        + u.shift(0, 0, -1) + u.shift(0, 0, 1)
    d = s - 6.0 * u
    if h is None:
        return d
    return d / u.p._stmt("mul", float(h), float(h))


class Program:
    def __init__(self, dtype: str = "f64"):
        if dtype not in ("f64", "f32"):
            raise ValueError("dtype is 'f64' or 'f32'")
        self.dtype = dtype
        self.lines = [f"dtype {dtype}"]
        self.inputs, self.params, self.outputs = [], [], []
        self._n = 0

    def _operand(self, x) -> str:
        if isinstance(x, Expr):
            if x.p is not self:
                raise ValueError("operand from another program")
            return x.name
        if isinstance(x, (int, float)):
            return repr(float(x))
        raise TypeError(f"unsupported operand {x!r}")

    def _stmt(self, op, a, b=None, extra="") -> Expr:
        name = f"t{self._n}"
        self._n += 1
        ops = " ".join(self._operand(x) for x in (a, b) if x is not None)
        field = any(isinstance(x, Expr) and x.field for x in (a, b))
        self.lines.append(f"{name} = {op} {ops}{extra}")
        return Expr(self, name, field or op == "shift")

    def input(self, *names) -> tuple:
        self.lines.append("input " + " ".join(names))
        self.inputs += names
        return tuple(Expr(self, n, True) for n in names)

    def param(self, *names) -> tuple:
        self.lines.append("param " + " ".join(names))
        self.params += names
        return tuple(Expr(self, n, False) for n in names)

    def output(self, name: str, e: Expr) -> None:
        if not isinstance(e, Expr) or not e.field:
            raise TypeError("outputs are field expressions")
        self.lines.append(f"{name} = copy {e.name}")
        self.lines.append(f"output {name}")
        self.outputs.append(name)

    def text(self) -> str:
        return "\n".join(self.lines) + "\n"

    def compile(self, fuse: bool = True, cache: bool = True) -> "Fused":
        return compile_text(self.text(), fuse, cache)


def _load():
    L = _lib.lib()
    if not getattr(L, "_fuse_ready", False):
        vp, c_int, i64, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        L.dcp_fuse_build.argtypes = [ctypes.c_char_p, c_int, ctypes.POINTER(vp), ctypes.c_char_p, sz]
        L.dcp_fuse_build.restype = c_int
        L.dcp_fuse_free.argtypes = [vp]
        L.dcp_fuse_free.restype = None
        L.dcp_fuse_info.argtypes = [vp, ctypes.POINTER(i32), i32]
        L.dcp_fuse_info.restype = c_int
        L.dcp_fuse_source.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
        L.dcp_fuse_source.restype = c_int
        L.dcp_fuse_workspace_bytes.argtypes = [vp, i64, i64, i64, ctypes.POINTER(sz)]
        L.dcp_fuse_workspace_bytes.restype = c_int
        L.dcp_fuse_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp),
                                   i64, i64, i64, c_int, vp, sz, vp]
        L.dcp_fuse_run.restype = c_int
        L._fuse_ready = True
    return L


class FuseError(ValueError):
    pass


_CACHE: dict = {}
_CACHE_MAX = 64


def compile_text(text: str, fuse: bool = True, cache: bool = True) -> "Fused":
    """Builds (parses, partitions, generates, compiles) a program.  The same
    text and mode compiled again in this process returns the same object
    (run-time compilation takes about a second); cache=False forces a build."""
    key = (text, bool(fuse))
    if cache and key in _CACHE:
        return _CACHE[key]
    L = _load()
    h = ctypes.c_void_p()
    err = ctypes.create_string_buffer(4096)
    rc = L.dcp_fuse_build(text.encode(), int(bool(fuse)), ctypes.byref(h), err, len(err))
    if rc != 0:
        raise FuseError(f"dcp_fuse_build: {err.value.decode()} (status {rc})")
    prog = Fused(h, text)
    if cache:
        if len(_CACHE) >= _CACHE_MAX:
            _CACHE.pop(next(iter(_CACHE)))        # the oldest entry
        _CACHE[key] = prog
    return prog


class Fused:
    """A compiled program: run() on torch tensors (current stream)."""

    def __init__(self, handle: ctypes.c_void_p, text: str):
        self._h = handle
        self.text = text
        info = (ctypes.c_int32 * 6)()
        _lib.check("dcp_fuse_info", _load().dcp_fuse_info(self._h, info, 6))
        self.dtype = torch.float64 if info[0] == 0 else torch.float32
        self.n_inputs, self.n_params, self.n_outputs, self.n_kernels, self.n_buffers = info[1:6]
        self.params = [ln.split()[1:] for ln in text.splitlines() if ln.split()[:1] == ["param"]]
        self.params = [p for group in self.params for p in group]

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h:
            try:
                _load().dcp_fuse_free(h)
            except Exception:        # interpreter shutdown: the library is gone
                pass

    @property
    def source(self) -> str:
        L = _load()
        need = ctypes.c_size_t(0)
        _lib.check("dcp_fuse_source", L.dcp_fuse_source(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _lib.check("dcp_fuse_source", L.dcp_fuse_source(self._h, buf, need.value, ctypes.byref(need)))
        return buf.value.decode()

    def workspace_bytes(self, shape) -> int:
        nz, ny, nx = shape
        out = ctypes.c_size_t(0)
        _lib.check("dcp_fuse_workspace_bytes",
                   _load().dcp_fuse_workspace_bytes(self._h, nx, ny, nz, ctypes.byref(out)))
        return out.value

    def run(self, inputs, params=None, bc="dirichlet0", outputs=None, ws=None):
        """inputs: tensors in declaration order (shape (nz, ny, nx), the
        program's dtype, contiguous, on one GPU); params: dict or sequence;
        outputs: tensors like the inputs (allocated when None); ws: a byte
        workspace (allocated when None or too small).  Runs on the inputs'
        device and its current stream.  Returns the list of output tensors."""
        from .api import bc_code
        if len(inputs) != self.n_inputs or self.n_inputs == 0:
            raise ValueError(f"expected {self.n_inputs} inputs")
        dev = inputs[0].device

        def check(t, what):
            if (not isinstance(t, torch.Tensor) or t.dtype != self.dtype or not t.is_contiguous()
                    or t.device != dev or t.dim() != 3 or t.shape != inputs[0].shape):
                raise ValueError(f"{what}: contiguous 3-D tensors of the program's dtype, of one shape, "
                                 "on one GPU")

        if dev.type != "cuda":
            raise ValueError("inputs must be on a GPU")
        for t in inputs:
            check(t, "inputs")
        shape = inputs[0].shape
        if isinstance(params, dict):
            params = [params[k] for k in self.params]
        params = list(params or [])
        if len(params) != self.n_params:
            raise ValueError(f"expected {self.n_params} params")
        if outputs is None:
            outputs = [torch.empty_like(inputs[0]) for _ in range(self.n_outputs)]
        if len(outputs) != self.n_outputs:
            raise ValueError(f"expected {self.n_outputs} outputs")
        for t in outputs:
            check(t, "outputs")
        wsb = self.workspace_bytes(shape)
        if wsb and (ws is None or ws.device != dev or not ws.is_contiguous()
                    or ws.numel() * ws.element_size() < wsb):
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        ip = (ctypes.c_void_p * len(inputs))(*[t.data_ptr() for t in inputs])
        op = (ctypes.c_void_p * len(outputs))(*[t.data_ptr() for t in outputs])
        pp = (ctypes.c_double * max(1, len(params)))(*[float(v) for v in params])
        nz, ny, nx = shape
        with torch.cuda.device(dev):
            stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
            _lib.check("dcp_fuse_run", _load().dcp_fuse_run(
                self._h, ip, pp, op, nx, ny, nz, bc_code(bc),
                ctypes.c_void_p(ws.data_ptr()) if wsb else None, wsb, stream))
        return outputs
