"""Pins of the program interpreter (oracle/fuse_interp.py), the reference of
the fusing compiler: the reaction-diffusion step written as single-operator
statements reproduces the C oracle (itself pinned) bit for bit; shifts
match their definition on brute force; the 7-point sum has the Fourier
eigenvalue; FP32 programs round every operation to float32."""
import numpy as np
import pytest

import oracle
from oracle import fuse_interp

STEP = """
dtype {dt}
input u f
param alpha beta gamma dt
# lap = (xm + xp + ym + yp + zm + zp - 6u) / (h*h), added left to right
xm = shift u -1 0 0
xp = shift u 1 0 0
ym = shift u 0 -1 0
yp = shift u 0 1 0
zm = shift u 0 0 -1
zp = shift u 0 0 1
s1 = add xm xp
s2 = add s1 ym
s3 = add s2 yp
s4 = add s3 zm
s5 = add s4 zp
six = mul 6.0 u
d = sub s5 six
hh = mul {h} {h}
lap = div d hh
uu = mul u u
u3 = mul uu u
t1 = mul alpha lap
t2 = mul beta u3
t3 = sub t1 t2
t4 = mul gamma f
t5 = add t3 t4
t6 = mul dt t5
unew = add u t6
output unew
"""

C = dict(alpha=1.0, beta=0.1, gamma=0.5, h=1.0, dt=0.1)


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(6, 5, 4), (1, 1, 1), (2, 3, 2), (7, 1, 3), (2, 2, 2)])
@pytest.mark.parametrize("h", [1.0, 0.7])
def test_step_program_equals_c_oracle_bitwise(shape, bc, h):
    nx, ny, nz = shape
    r = np.random.default_rng(sum(shape) + bc)
    u, f = r.uniform(-1, 1, (nz, ny, nx)), r.uniform(-1, 1, (nz, ny, nx))
    c = dict(C, h=h)
    want, _, _ = oracle.run(u, f, c, 1, bc, norms=False)
    (got,) = fuse_interp.run(STEP.format(dt="f64", h=repr(h)), [u, f], c, bc)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("d", [(1, 0, 0), (-2, 1, 0), (0, 0, 3), (5, -4, 1), (-7, 0, -9)])
def test_shift_brute_force(d, bc):
    dx, dy, dz = d
    nz, ny, nx = 3, 4, 5
    a = np.arange(nx * ny * nz, dtype=np.float64).reshape(nz, ny, nx) + 1.0
    want = np.zeros_like(a)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                xx, yy, zz = x + dx, y + dy, z + dz
                if bc == 1:
                    want[z, y, x] = a[zz % nz, yy % ny, xx % nx]
                elif 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                    want[z, y, x] = a[zz, yy, xx]
    assert np.array_equal(fuse_interp.shift(a, dx, dy, dz, bc), want)


def test_seven_point_sum_fourier_mode():
    nz, ny, nx, m = 4, 6, 10, (1, 2, 1)
    x, y, z = np.arange(nx), np.arange(ny)[:, None], np.arange(nz)[:, None, None]
    ph = 2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)
    u = np.cos(ph)
    text = "\n".join(["dtype f64", "input u"] + STEP.split("hh =")[0].split("param alpha beta gamma dt")[1]
                     .strip().splitlines() + ["output d"])
    (d,) = fuse_interp.run(text, [u], bc=1)
    mu = sum(2 * np.cos(2 * np.pi * mm / n) - 2 for mm, n in zip(m, (nx, ny, nz)))
    assert np.max(np.abs(d - mu * u)) < 1e-13


def test_f32_rounds_every_operation():
    # 1 + 2^-24 is a tie between 1 and the next float above it: float32
    # arithmetic gives exactly 1, float64 keeps the 2^-24
    text = "dtype {}\ninput u\ny = add u 5.9604644775390625e-08\nz = sub y u\noutput z\n"
    u = np.ones((1, 1, 4))
    (z32,) = fuse_interp.run(text.format("f32"), [u])
    (z64,) = fuse_interp.run(text.format("f64"), [u])
    assert z32.dtype == np.float32 and np.all(z32 == 0.0)
    assert np.all(z64 == 2.0 ** -24)


def test_scalar_statements_and_params():
    text = "dtype f64\ninput u\nparam p\ns = mul 3 p\nq = div s 4\ny = mul q u\nw = neg y\noutput y w\n"
    u = np.full((2, 2, 2), 2.0)
    y, w = fuse_interp.run(text, [u], {"p": 0.5})
    assert np.all(y == 0.75) and np.all(w == -0.75)


@pytest.mark.parametrize("seed", [0, 4, 9])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [0, 1])
def test_run_points_equals_whole_grid_run(seed, dtype, bc):
    # the per-point evaluation (used at grid sizes the whole-array run cannot
    # hold) gives every output at every point exactly as run() does
    from fuse_programs import random_program
    P = random_program(seed, dtype)
    dt = np.float64 if dtype == "f64" else np.float32
    r = np.random.default_rng(seed + 5)
    shape = (4, 5, 6)
    arrays = [r.uniform(-1, 1, shape).astype(dt) for _ in range(3)]
    params = {"p": float(r.uniform(-1, 1)), "q": float(r.uniform(-1, 1))}
    want = fuse_interp.run(P.text(), arrays, params, bc)
    pts = [(z, y, x) for z in range(4) for y in range(5) for x in range(6)]
    got = fuse_interp.run_points(P.text(), arrays, params, bc, pts)
    for i, w in enumerate(want):
        assert got.dtype == w.dtype and np.array_equal(got[i], w.reshape(-1))
