"""Statement-by-statement interpreter of single-operator array programs.

TEST INFRASTRUCTURE ONLY.  The reference for the fusing compiler: it
evaluates a program's statements in order, each over the whole grid with
NumPy, every value materialised (the unoptimised program of Sec. 2.3, before
any fusion), in the program's dtype, so each operation rounds once.  It
parses the program text itself and shares nothing with the library.

Program text (see the library header): `dtype f64|f32`, `input NAMES`,
`param NAMES`, `NAME = add|sub|mul|div A B`, `NAME = neg A`,
`NAME = copy A`, `NAME = shift A dx dy dz`, `output NAMES`; operands are
names or numeric literals; '#' starts a comment.  Fields are arrays shaped
(nz, ny, nx) (x fastest); a shift reads the field at (x+dx, y+dy, z+dz),
0 outside the grid (bc 0) or with indices mod n (bc 1).
"""
from __future__ import annotations

import numpy as np


def shift(a: np.ndarray, dx: int, dy: int, dz: int, bc: int) -> np.ndarray:
    """out[z, y, x] = a[z+dz, y+dy, x+dx] under the boundary rule."""
    if bc == 1:
        return np.roll(a, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
    nz, ny, nx = a.shape
    out = np.zeros_like(a)

    def rng(n, d):
        lo, hi = max(0, -d), min(n, n - d)
        return (slice(lo, hi), slice(lo + d, hi + d)) if hi > lo else None

    rx, ry, rz = rng(nx, dx), rng(ny, dy), rng(nz, dz)
    if rx and ry and rz:
        out[rz[0], ry[0], rx[0]] = a[rz[1], ry[1], rx[1]]
    return out


def run(text: str, inputs, params=None, bc: int = 0) -> list:
    """Evaluates the program; inputs in declaration order (arrays), params a
    dict or sequence in declaration order.  Returns the outputs in
    declaration order, as arrays of the program's dtype."""
    dt = None
    env = {}
    in_names, par_names, outs = [], [], []
    stmts = []
    for raw in text.splitlines():
        t = raw.split("#", 1)[0].split()
        if not t:
            continue
        if t[0] == "dtype":
            dt = {"f64": np.float64, "f32": np.float32}[t[1]]
        elif t[0] == "input":
            in_names += t[1:]
        elif t[0] == "param":
            par_names += t[1:]
        elif t[0] == "output":
            outs += t[1:]
        else:
            assert t[1] == "=", raw
            stmts.append(t)
    if dt is None:
        raise ValueError("missing dtype")
    inputs = list(inputs)
    if len(inputs) != len(in_names):
        raise ValueError("input count")
    for n, a in zip(in_names, inputs):
        env[n] = np.ascontiguousarray(a, dtype=dt)
    if isinstance(params, dict):
        params = [params[n] for n in par_names]
    params = list(params or [])
    for n, v in zip(par_names, params):
        env[n] = dt(v)               # rounded to the dtype once

    def val(tok):
        if tok in env:
            return env[tok]
        return dt(float(tok))        # a literal, rounded to the dtype once

    for t in stmts:
        name, op, args = t[0], t[2], t[3:]
        if op == "shift":
            a = val(args[0])
            env[name] = shift(a, int(args[1]), int(args[2]), int(args[3]), bc)
        elif op == "neg":
            env[name] = -val(args[0])
        elif op == "copy":
            env[name] = val(args[0]).copy()
        else:
            a, b = val(args[0]), val(args[1])
            with np.errstate(all="ignore"):
                if op == "add":
                    r = a + b
                elif op == "sub":
                    r = a - b
                elif op == "mul":
                    r = a * b
                elif op == "div":
                    r = a / b
                else:
                    raise ValueError(f"unknown op {op}")
            env[name] = r.astype(dt) if isinstance(r, np.ndarray) else dt(r)
    return [np.asarray(env[n], dtype=dt) for n in outs]


def run_points(text: str, inputs, params=None, bc: int = 0, points=()) -> "np.ndarray":
    """The outputs at the given points only, each point (z, y, x).

    Every statement is evaluated per point, as in run(): an operation rounds
    once in the program's dtype, and a shift evaluates its operand at the
    shifted point under the boundary rule (zero outside the grid, or indices
    mod n).  Inputs may be any objects indexed as a[z, y, x] whose elements
    convert with float() (so very large fields need not be copied whole).
    Returns an array [outputs, points] of the program's dtype."""
    dt = None
    in_names, par_names, outs = [], [], []
    defs = {}
    for raw in text.splitlines():
        t = raw.split("#", 1)[0].split()
        if not t:
            continue
        if t[0] == "dtype":
            dt = {"f64": np.float64, "f32": np.float32}[t[1]]
        elif t[0] == "input":
            in_names += t[1:]
        elif t[0] == "param":
            par_names += t[1:]
        elif t[0] == "output":
            outs += t[1:]
        else:
            assert t[1] == "=", raw
            defs[t[0]] = (t[2], t[3:])
    if dt is None:
        raise ValueError("missing dtype")
    inputs = list(inputs)
    if len(inputs) != len(in_names):
        raise ValueError("input count")
    arrs = dict(zip(in_names, inputs))
    if isinstance(params, dict):
        params = [params[n] for n in par_names]
    scal = {n: dt(v) for n, v in zip(par_names, list(params or []))}
    nz, ny, nx = inputs[0].shape
    memo = {}

    def is_field(name):
        if name in arrs:
            return True
        if name not in defs:
            return False
        op, args = defs[name]
        return op == "shift" or any(is_field(a) for a in (args[:1] if op == "shift" else args))

    def val(name, z, y, x):
        if name in scal:
            return scal[name]
        if name in arrs:
            return dt(float(arrs[name][z, y, x]))
        if name not in defs:
            return dt(float(name))                       # a literal
        key = (name, z, y, x) if is_field(name) else (name,)
        if key in memo:
            return memo[key]
        op, args = defs[name]
        with np.errstate(all="ignore"):
            if op == "shift":
                zz, yy, xx = z + int(args[3]), y + int(args[2]), x + int(args[1])
                if bc == 1:
                    r = val(args[0], zz % nz, yy % ny, xx % nx)
                elif 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                    r = val(args[0], zz, yy, xx)
                else:
                    r = dt(0)
            elif op == "neg":
                r = -val(args[0], z, y, x)
            elif op == "copy":
                r = val(args[0], z, y, x)
            else:
                a, b = val(args[0], z, y, x), val(args[1], z, y, x)
                if op == "add":
                    r = a + b
                elif op == "sub":
                    r = a - b
                elif op == "mul":
                    r = a * b
                elif op == "div":
                    r = a / b
                else:
                    raise ValueError(f"unknown op {op}")
        r = dt(r)
        memo[key] = r
        return r

    out = np.empty((len(outs), len(points)), dtype=dt)
    for j, (z, y, x) in enumerate(points):
        for i, name in enumerate(outs):
            out[i, j] = val(name, int(z), int(y), int(x))
    return out
