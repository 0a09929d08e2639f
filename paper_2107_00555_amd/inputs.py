"""Seeded synthetic inputs for the reaction-diffusion and Jacobi workloads.

This module holds the random input generators only: none of the program's
arithmetic.  Both the GPU path's tests/benchmark and the CPU oracle consume
the arrays it returns, so the two sides never have to agree on anything but
these arrays.

Every stream draws from ``np.random.default_rng(SeedSequence([seed, s]))``
with a fixed stream id ``s``:

    0  u0             initial state
    1  f              source field
    2  u_tgt          loss target
    3  FD directions  finite-difference probes
    4  A              Jacobi programs, first array
    5  B              Jacobi programs, second array

Arrays are float64, C order, shape ``(nz, ny, nx)`` (x is the fastest axis).
Float32 workloads cast these once (round to nearest even).
"""
from __future__ import annotations

import numpy as np

STREAM_U0 = 0
STREAM_F = 1
STREAM_TGT = 2
STREAM_FD = 3
STREAM_JA = 4
STREAM_JB = 5


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def uniform(nx: int, ny: int, nz: int, seed: int, stream: int) -> np.ndarray:
    """i.i.d. uniform[-1, 1] field of shape (nz, ny, nx)."""
    return rng(seed, stream).uniform(-1.0, 1.0, size=(nz, ny, nx))


def sinusoid_params(seed: int, stream: int = STREAM_F, count: int = 8):
    """Draw ``count`` low-frequency modes: integer wave numbers m in
    {-4..4}^3 (redrawn if all zero), amplitude a ~ U[-1,1], phase phi ~ U[0,2pi)."""
    r = rng(seed, stream)
    modes = []
    for _ in range(count):
        m = r.integers(-4, 5, size=3)
        while not m.any():
            m = r.integers(-4, 5, size=3)
        a = r.uniform(-1.0, 1.0)
        phi = r.uniform(0.0, 2.0 * np.pi)
        modes.append((int(m[0]), int(m[1]), int(m[2]), float(a), float(phi)))
    return modes


def sinusoids(nx: int, ny: int, nz: int, seed: int, stream: int = STREAM_F,
              count: int = 8, box=None) -> np.ndarray:
    """f = sum_j a_j sin(2 pi (mx x/nx + my y/ny + mz z/nz) + phi_j).

    Periodic on the grid and smooth.  ``box`` = ((x0, x1), (y0, y1), (z0, z1))
    evaluates the same field on a sub-box of the (nx, ny, nz) grid only.
    With sin(A + B) = sin A cos B + cos A sin B, A over (y, x) and B over z,
    the sum over modes is one product of a (z, 2*count) by a (2*count, y*x)
    matrix, which keeps the 512^3 and 1024x1024x512 grids cheap to build.
    """
    modes = sinusoid_params(seed, stream, count)
    (x0, x1), (y0, y1), (z0, z1) = box if box is not None else ((0, nx), (0, ny), (0, nz))
    x = np.arange(x0, x1, dtype=np.float64)
    y = np.arange(y0, y1, dtype=np.float64)
    z = np.arange(z0, z1, dtype=np.float64)
    k = len(modes)
    S = np.empty((2 * k, y.size * x.size))
    W = np.empty((z.size, 2 * k))
    for j, (mx, my, mz, a, phi) in enumerate(modes):
        A = (2.0 * np.pi * (my * y / ny))[:, None] + (2.0 * np.pi * (mx * x / nx))[None, :] + phi
        S[j] = (a * np.sin(A)).ravel()
        S[k + j] = (a * np.cos(A)).ravel()
        B = 2.0 * np.pi * (mz * z / nz)
        W[:, j] = np.cos(B)
        W[:, k + j] = np.sin(B)
    return (W @ S).reshape(z.size, y.size, x.size)


def uniform_zslab(nx: int, ny: int, nz_lo: int, seed: int, stream: int) -> np.ndarray:
    """The first nz_lo z-planes of uniform(nx, ny, nz, seed, stream) for any
    nz >= nz_lo (the generator fills the array in C order, so a shorter draw
    is a prefix of a longer one)."""
    return rng(seed, stream).uniform(-1.0, 1.0, size=(nz_lo, ny, nx))


def fd_directions(nx: int, ny: int, nz: int, seed: int, count: int):
    """Yield ``count`` probe directions (d_u ~ U[-1,1]^N, d_alpha ~ N(0,1),
    d_beta ~ N(0,1)), drawn in order from the FD stream."""
    r = rng(seed, STREAM_FD)
    for _ in range(count):
        du = r.uniform(-1.0, 1.0, size=(nz, ny, nx))
        da = float(r.standard_normal())
        db = float(r.standard_normal())
        yield du, da, db


# Named workloads: the grids, boundaries and coefficient sets the library is
# measured and checked on.
DIRICHLET0 = 0
PERIODIC = 1

BASE_COEFFS = dict(alpha=1.0, beta=0.1, gamma=0.5, h=1.0, dt=0.1)

WORKLOADS = {
    # 64^3 float64, ghost-zero boundary, u0 and f uniform, T=10, forward.
    "plain_64": dict(shape=(64, 64, 64), dtype="f64", bc=DIRICHLET0, T=10,
                     u0="uniform", f="uniform"),
    # 512^3 float64, periodic, u0 uniform, f = 8 sinusoids, T=100.
    "fwd_512_f64": dict(shape=(512, 512, 512), dtype="f64", bc=PERIODIC, T=100,
                        u0="uniform", f="sinusoids"),
    # Same generator, float32 storage and compute, FP64 norms.
    "fwd_512_f32": dict(shape=(512, 512, 512), dtype="f32", bc=PERIODIC, T=100,
                        u0="uniform", f="sinusoids"),
    # 256^3 float64, ghost-zero, T=50, checkpoint every 10, loss 0.5||u_T-u_tgt||^2.
    "grad_256_f64": dict(shape=(256, 256, 256), dtype="f64", bc=DIRICHLET0, T=50,
                         ckpt_every=10, u0="uniform", f="uniform"),
    # 1024x1024x512 float32, periodic, T=200, checkpoint every 20.
    "grad_large_f32": dict(shape=(1024, 1024, 512), dtype="f32", bc=PERIODIC, T=200,
                           ckpt_every=20, u0="uniform", f="sinusoids"),
}


def make_fields(workload: str | dict, seed: int = 0, shape=None):
    """(u0, f) for a workload, float64, shape (nz, ny, nx); ``shape`` = (nx, ny, nz)
    overrides the workload's grid."""
    w = WORKLOADS[workload] if isinstance(workload, str) else workload
    nx, ny, nz = shape if shape is not None else w["shape"]
    u0 = uniform(nx, ny, nz, seed, STREAM_U0)
    if w["f"] == "uniform":
        f = uniform(nx, ny, nz, seed, STREAM_F)
    else:
        f = sinusoids(nx, ny, nz, seed, STREAM_F)
    return u0, f


def target(nx: int, ny: int, nz: int, seed: int = 0) -> np.ndarray:
    """u_tgt ~ U[-1,1] for the gradient workloads."""
    return uniform(nx, ny, nz, seed, STREAM_TGT)


# The two Jacobi listings (jacobi_1d in Sec. 2.2, jacobi_2d in Sec. 4.3),
# float64 in and out.  "paper" sizes are the initial problem sizes of the
# distributed-benchmark table in Sec. 4.4 (one process: T=1000 with N=24000,
# and T=1000 with N=1300); "p1296" sizes are those problems weak-scaled, by
# the table's scaling factors (N*S in 1D, N*sqrt(S) in 2D), to the largest
# run of that section, S = 1296 processes, all on one GPU.  The paper gives
# no input values; A and B are i.i.d. U[-1, 1] here.
JACOBI_WORKLOADS = {
    "jacobi_1d_paper": dict(dims=1, n=24000, tsteps=1000),
    "jacobi_2d_paper": dict(dims=2, n=1300, tsteps=1000),
    "jacobi_1d_p1296": dict(dims=1, n=24000 * 1296, tsteps=1000),
    "jacobi_2d_p1296": dict(dims=2, n=1300 * 36, tsteps=1000),
}


def jacobi_shape(dims: int, n: int, n1: int | None = None) -> tuple:
    if dims == 1:
        return (int(n),)
    return (int(n), int(n if n1 is None else n1))


def jacobi_fields(dims: int, n: int, seed: int = 0, n1: int | None = None):
    """(A, B) ~ U[-1, 1], float64 NumPy arrays of shape (n,) or (n, n1)."""
    shape = jacobi_shape(dims, n, n1)
    return (rng(seed, STREAM_JA).uniform(-1.0, 1.0, size=shape),
            rng(seed, STREAM_JB).uniform(-1.0, 1.0, size=shape))


def jacobi_fields_device(dims: int, n: int, seed: int = 0, device="cuda", n1: int | None = None):
    """(A, B) ~ U[-1, 1] as float64 torch tensors drawn on the device (for
    sizes too large to draw on the host); a different sequence from
    jacobi_fields, reproducible for a given seed and device type."""
    import torch
    shape = jacobi_shape(dims, n, n1)
    out = []
    for stream in (STREAM_JA, STREAM_JB):
        g = torch.Generator(device=device)
        g.manual_seed(int(np.random.SeedSequence([int(seed), stream]).generate_state(1, np.uint64)[0]
                          & 0x7FFFFFFFFFFFFFFF))
        t = torch.empty(shape, dtype=torch.float64, device=device)
        t.uniform_(-1.0, 1.0, generator=g)
        out.append(t)
    return out[0], out[1]
