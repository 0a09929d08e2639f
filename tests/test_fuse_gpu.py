"""Generated kernels of the fusing compiler on the GPU, against the program
interpreter (oracle/fuse_interp.py): bit for bit, fused and unfused, FP64
and FP32, both boundary rules; the reaction-diffusion step also against the
C oracle and the hand-written unfused chain."""
import numpy as np
import pytest
import torch

import oracle
from fuse_programs import random_program
from gpu_util import BASE, DEV, rand_fields, say, to_dev, to_host
from oracle import fuse_interp

pytestmark = pytest.mark.gpu


def _fuse():
    from paper_2107_00555_amd import fuse
    return fuse


def step_program(dtype="f64", h=1.0):
    F = _fuse()
    P = F.Program(dtype)
    u, f = P.input("u", "f")
    alpha, beta, gamma, dt = P.param("alpha", "beta", "gamma", "dt")
    lap = F.lap7(u, h)
    u3 = (u * u) * u
    t1 = alpha * lap
    t2 = beta * u3
    t3 = t1 - t2
    t4 = gamma * f
    t5 = t3 + t4
    t6 = dt * t5
    P.output("unew", u + t6)
    return P


PARAMS = {k: BASE[k] for k in ("alpha", "beta", "gamma", "dt")}


def run_gpu(prog, arrays, params, bc):
    tdt = prog.dtype
    outs = prog.run([to_dev(a, tdt) for a in arrays], params, bc=bc)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(37, 19, 23), (1, 1, 1), (64, 3, 5), (2, 2, 9), (130, 66, 4),
                                   # (nx, ny, nz): three x tiles of 256 lanes (512 points in
                                   # float64, 1024 in float32) with interior tiles, a ragged last
                                   # tile, and a row length that is not a multiple of 4
                                   (2150, 4, 5), (3073, 3, 3),
                                   # more rows than the grid's y extent; more z chunks than its z extent
                                   (3, 70000, 2), (1, 1, 1100000)])
def test_step_program_matches_interpreter_bitwise(shape, bc, dtype, fuse):
    P = step_program(dtype)
    prog = P.compile(fuse)
    u0, f = rand_fields(shape, 1000 + sum(shape))
    dt = np.float64 if dtype == "f64" else np.float32
    u0, f = u0.astype(dt), f.astype(dt)
    say("fuse step", shape, bc, dtype, fuse)
    (got,) = run_gpu(prog, [u0, f], PARAMS, bc)
    (want,) = fuse_interp.run(P.text(), [u0, f], PARAMS, bc)
    assert got.dtype == want.dtype and np.array_equal(got, want)


@pytest.mark.parametrize("bc", [0, 1])
def test_ten_generated_steps_equal_c_oracle_and_unfused_chain(bc):
    from paper_2107_00555_amd import api
    shape, T = (40, 24, 20), 10
    prog = step_program("f64").compile()
    u0, f = rand_fields(shape, 1001)
    want, _, _ = oracle.run(u0, f, BASE, T, bc, norms=False)
    u, fd = to_dev(u0), to_dev(f)
    v = torch.empty_like(u)
    say("fuse 10 steps", bc)
    for _ in range(T):
        prog.run([u, fd], PARAMS, bc=bc, outputs=[v])
        u, v = v, u
    torch.cuda.synchronize()
    assert np.array_equal(to_host(u), want)
    w = to_dev(u0)
    api.run(w, fd, BASE, T, bc, impl="unfused", norms=False)
    torch.cuda.synchronize()
    assert torch.equal(w, u)


@pytest.mark.parametrize("seed", list(range(12)))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_programs_match_interpreter_bitwise(seed, dtype):
    P = random_program(seed, dtype)
    dt = np.float64 if dtype == "f64" else np.float32
    r = np.random.default_rng(seed + 77)
    shape = (int(r.integers(1, 50)), int(r.integers(1, 20)), int(r.integers(1, 12)))
    arrays = [r.uniform(-1, 1, shape).astype(dt) for _ in range(3)]
    params = {"p": float(r.uniform(-1, 1)), "q": float(r.uniform(-1, 1))}
    for bc in (0, 1):
        want = fuse_interp.run(P.text(), arrays, params, bc)
        for fuse in (True, False):
            prog = P.compile(fuse)
            say("fuse random", seed, dtype, shape, bc, fuse, prog.n_kernels)
            got = run_gpu(prog, arrays, params, bc)
            for g, w in zip(got, want):
                assert np.array_equal(g, w), (seed, bc, fuse)


@pytest.mark.parametrize("seed", [3, 5, 8, 11])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_programs_wide_grid_bitwise(seed, dtype):
    # rows of several tiles: interior workgroups take the vector reads at
    # fixed offsets, edge and ragged workgroups the boundary rule
    P = random_program(seed, dtype)
    r = np.random.default_rng(seed + 99)
    shape = (5, 4, 2301)
    dt = np.float64 if dtype == "f64" else np.float32
    arrays = [r.uniform(-1, 1, shape).astype(dt) for _ in range(3)]
    params = {"p": float(r.uniform(-1, 1)), "q": float(r.uniform(-1, 1))}
    for bc in (0, 1):
        want = fuse_interp.run(P.text(), arrays, params, bc)
        for fuse in (True, False):
            prog = P.compile(fuse)
            say("fuse random wide", seed, dtype, shape, bc, fuse, prog.n_kernels)
            got = run_gpu(prog, arrays, params, bc)
            for g, w in zip(got, want):
                assert np.array_equal(g, w), (seed, bc, fuse)


def test_run_argument_errors():
    F = _fuse()
    from paper_2107_00555_amd import _lib
    prog = step_program("f64").compile()
    u = torch.zeros((4, 4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        prog.run([u], PARAMS)                           # one input short
    with pytest.raises(ValueError):
        prog.run([u, u.float()], PARAMS)                # wrong dtype
    with pytest.raises(_lib.DcpError):
        prog.run([u, u.clone()], PARAMS, outputs=[u])   # output aliases an input
    with pytest.raises(_lib.DcpError):
        prog.run([u, u.clone()], dict(PARAMS, alpha=float("nan")))
    # outputs are checked before anything is launched
    with pytest.raises(ValueError):
        prog.run([u, u.clone()], PARAMS, outputs=[torch.zeros((4, 4, 3), dtype=torch.float64, device=DEV)])
    with pytest.raises(ValueError):
        prog.run([u, u.clone()], PARAMS, outputs=[torch.zeros((4, 4, 4), dtype=torch.float32, device=DEV)])
    with pytest.raises(ValueError):
        prog.run([u, u.clone()], PARAMS, outputs=[])
    with pytest.raises(ValueError):
        prog.run([u, u.clone()], PARAMS, outputs=[torch.zeros((4, 4, 8), dtype=torch.float64, device=DEV)[:, :, ::2]])


def test_two_threads_share_one_program():
    # the first run on the device loads the code under a lock; both threads'
    # results equal the interpreter's
    import threading
    P = step_program("f64")
    prog = P.compile()
    shape = (40, 12, 9)
    u0, f = rand_fields(shape, 1200)
    (want,) = fuse_interp.run(P.text(), [u0, f], PARAMS, 1)
    u, fd = to_dev(u0), to_dev(f)
    outs = [torch.empty_like(u) for _ in range(2)]
    errs = []

    def work(o):
        try:
            for _ in range(5):
                prog.run([u, fd], PARAMS, bc=1, outputs=[o])
            torch.cuda.synchronize()
        except Exception as e:          # reported below
            errs.append(e)

    say("fuse two threads")
    ts = [threading.Thread(target=work, args=(o,)) for o in outs]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs, errs
    for o in outs:
        assert np.array_equal(to_host(o), want)


def test_free_right_after_a_run():
    # freeing the program waits for the device before unloading the code
    P = step_program("f32")
    shape = (300, 20, 16)
    u0, f = rand_fields(shape, 1201)
    u0, f = u0.astype(np.float32), f.astype(np.float32)
    (want,) = fuse_interp.run(P.text(), [u0, f], PARAMS, 0)
    u, fd = to_dev(u0, torch.float32), to_dev(f, torch.float32)
    out = torch.empty_like(u)
    say("fuse free after run")
    prog = P.compile(cache=False)                       # the only reference
    prog.run([u, fd], PARAMS, bc=0, outputs=[out])
    del prog
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), want)


def shifts_program(dtype):
    # shifts beyond the lane width (|dx| > V), exactly +-V, a z-queue of five
    # planes, several rows of one field, and a chained shift of a temporary
    F = _fuse()
    P = F.Program(dtype)
    a, b = P.input("a", "b")
    (p,) = P.param("p")
    s = (a.shift(5, 0, 0) + a.shift(-7, 2, -1)) + (a.shift(0, -3, 3) + a.shift(9, 0, 0))
    s = s + (a.shift(2, 0, 0) - a.shift(-2, 0, 0)) + (a.shift(4, 1, 0) - a.shift(-4, -1, 0))
    q = (b.shift(0, 0, -2) + b.shift(0, 0, -1)) + (b.shift(0, 0, 1) + b.shift(0, 0, 2)) + p * b
    P.output("o", s * 0.25 + q)
    P.output("r", (s - q).shift(1, -1, 1))
    return P


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [
    (300, 7, 6),     # (nx, ny, nz): every fast-path condition holds (nx >= V + 9, ny >= 3, nz > 3)
    (13, 3, 4),      # the shortest rows on the fast path in float32 (nx = V + 9 with V = 4)
    (12, 3, 4),      # one point shorter: per-point path in float32, fast path in float64 (V = 2)
    (64, 2, 3),      # ny < 3, nz = 3: every point through the rule
    (517, 5, 9),     # ragged row end in both dtypes
])
def test_large_and_long_shifts_bitwise(shape, bc, dtype):
    P = shifts_program(dtype)
    dt = np.float64 if dtype == "f64" else np.float32
    r = np.random.default_rng(sum(shape) + bc)
    nx, ny, nz = shape
    arrays = [r.uniform(-1, 1, (nz, ny, nx)).astype(dt) for _ in range(2)]
    want = fuse_interp.run(P.text(), arrays, {"p": 0.375}, bc)
    for fuse in (True, False):
        prog = P.compile(fuse)
        say("fuse shifts", shape, bc, dtype, fuse, prog.n_kernels)
        got = run_gpu(prog, arrays, {"p": 0.375}, bc)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), (shape, bc, dtype, fuse)


def test_grid_beyond_32_bit_indices_sampled():
    # 2048 x 1024 x 1030 float32 points (8.6 GB a field): point indices pass
    # 2^31, so the 64-bit index variant runs; outputs are checked at the
    # corners, along the last planes (indices above 2^31) and at random
    # points against the per-point interpreter (inputs read from the device
    # one point at a time)
    P = step_program("f32")
    prog = P.compile()
    nx, ny, nz = 2048, 1024, 1030
    assert nx * ny * nz > 2 ** 31
    g = torch.Generator(device=DEV).manual_seed(77)
    u = torch.rand((nz, ny, nx), generator=g, device=DEV, dtype=torch.float32) * 2 - 1
    f = torch.rand((nz, ny, nx), generator=g, device=DEV, dtype=torch.float32) * 2 - 1
    r = np.random.default_rng(78)
    pts = [(z, y, x) for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, 1, nx - 2, nx - 1)]
    pts += [(nz - 1, int(y), int(x)) for y, x in zip(r.integers(0, ny, 40), r.integers(0, nx, 40))]
    pts += [(int(z), int(y), int(x)) for z, y, x in zip(r.integers(0, nz, 60), r.integers(0, ny, 60),
                                                         r.integers(0, nx, 60))]
    for bc in (0, 1):
        say("fuse beyond 32-bit indices", (nx, ny, nz), bc)
        (out,) = prog.run([u, f], PARAMS, bc=bc)
        torch.cuda.synchronize()
        want = fuse_interp.run_points(P.text(), [u, f], PARAMS, bc, pts)[0]
        got = np.array([out[z, y, x].item() for z, y, x in pts], dtype=np.float32)
        assert np.array_equal(got, want), bc
        del out
    del u, f
    torch.cuda.empty_cache()


def adjoint_step_program(dtype="f64", h=1.0):
    # the transposed step Jacobian applied to lambda: the Laplacian is
    # symmetric, so lambda + dt*(alpha*Lap7(lambda) - 3*beta*u^2*lambda)
    F = _fuse()
    P = F.Program(dtype)
    lam, u = P.input("lam", "u")
    alpha, beta, dt = P.param("alpha", "beta", "dt")
    P.output("lam_prev", lam + dt * (alpha * F.lap7(lam, h) - (3.0 * beta) * ((u * u) * lam)))
    return P


@pytest.mark.parametrize("bc", [0, 1])
def test_generated_adjoint_step(bc):
    # a second program of the method: bit for bit the interpreter, and one
    # step of the C oracle's adjoint (T = 1: dL/du0 = J^T lambda_1) within
    # the FP64 tolerance (the oracle scatters L^T, a different rounding order)
    P = adjoint_step_program()
    prog = P.compile()
    assert prog.n_kernels == 1
    shape = (37, 23, 19)
    u0, f = rand_fields(shape, 1300 + bc)
    seed, _ = rand_fields(shape, 1302 + bc)
    prm = {k: BASE[k] for k in ("alpha", "beta", "dt")}
    say("fuse adjoint step", bc)
    (got,) = run_gpu(prog, [seed, u0], prm, bc)
    (want,) = fuse_interp.run(P.text(), [seed, u0], prm, bc)
    assert np.array_equal(got, want)
    g_u0, _, _ = oracle.adjoint(u0, f, seed, BASE, 1, bc)
    assert np.max(np.abs(got - g_u0)) / np.max(np.abs(g_u0)) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_step_sampled(dtype):
    # the benchmark's configuration: the step program on the 512^3 periodic
    # workload (seeded fields), one generated kernel; 300 sampled points
    # (faces, edges, corners, the interior) against the per-point interpreter
    from paper_2107_00555_amd import inputs
    u0, f = inputs.make_fields("fwd_512_f64", seed=0)
    dt = np.float64 if dtype == "f64" else np.float32
    u0, f = u0.astype(dt), f.astype(dt)
    P = step_program(dtype)
    prog = P.compile()
    say("fuse full size", dtype)
    (out,) = prog.run([to_dev(u0, prog.dtype), to_dev(f, prog.dtype)], PARAMS, bc=1)
    torch.cuda.synchronize()
    n = 512
    r = np.random.default_rng(5)
    edge = [0, 1, n - 2, n - 1]
    pts = [(z, y, x) for z in edge for y in edge for x in edge]
    pts += [tuple(int(v) for v in r.integers(0, n, 3)) for _ in range(300 - len(pts))]
    want = fuse_interp.run_points(P.text(), [u0, f], PARAMS, 1, pts)[0]
    got = np.array([out[z, y, x].item() for z, y, x in pts], dtype=dt)
    assert np.array_equal(got, want)
