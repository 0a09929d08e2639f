"""Forward parity: the HIP path against the CPU oracle, element by element,
on seeded inputs.  Shapes span several tiles along every axis and end in
ragged tails (tiles are 128 or 256 points along x, 8-16 rows along y and
8-64 planes along z), plus the degenerate grids.

Tolerances: float64 1e-12 normwise, float32 1e-5 normwise against the FP64
oracle run on the float32-rounded inputs; the unfused float64 chain rounds
every statement exactly as the oracle does and must match it bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (BASE, DEV, assert_normwise, assert_rel, f32_round, misaligned_like, rand_fields,
                      say, to_dev, to_host)

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64, 64), (67, 33, 17), (200, 40, 33), (130, 5, 3), (1, 1, 9), (1, 1, 1),
          (2, 3, 4), (3, 70, 2), (256, 17, 70), (513, 9, 5)]
BCS = [0, 1]


def _api():
    from paper_2107_00555_amd import api
    return api


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_fused_f64_matches_oracle(shape, bc):
    api = _api()
    u0, f = rand_fields(shape, 100 + sum(shape))
    T = 6
    want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
    say("fused f64", shape, bc)
    u = to_dev(u0)
    out = api.run(u, to_dev(f), BASE, T, bc, impl="fused", norms=True)
    torch.cuda.synchronize()
    assert_normwise("u_T", to_host(u), want, 1e-12)
    assert_rel("E_t", to_host(out["energy"]), e_want, 1e-12)
    assert_rel("R_t", to_host(out["resid"]), r_want, 1e-12)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_unfused_f64_is_bitwise_oracle(shape, bc):
    api = _api()
    u0, f = rand_fields(shape, 200 + sum(shape))
    T = 4
    want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
    say("unfused f64", shape, bc)
    u = to_dev(u0)
    out = api.run(u, to_dev(f), BASE, T, bc, impl="unfused", norms=True)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(u), want)
    assert_rel("E_t", to_host(out["energy"]), e_want, 1e-12)
    assert_rel("R_t", to_host(out["resid"]), r_want, 1e-12)


@pytest.mark.parametrize("impl", ["fused", "unfused"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(64, 64, 64), (67, 33, 17), (256, 17, 70), (1, 1, 9), (5, 3, 2)])
def test_f32_matches_oracle(shape, bc, impl):
    api = _api()
    u0, f = rand_fields(shape, 300 + sum(shape))
    u0, f = f32_round(u0), f32_round(f)
    T = 10
    want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
    say("f32", impl, shape, bc)
    u = to_dev(u0, torch.float32)
    out = api.run(u, to_dev(f, torch.float32), BASE, T, bc, impl=impl, norms=True)
    torch.cuda.synchronize()
    assert_normwise("u_T", to_host(u), want, 1e-5)
    assert_rel("E_t", to_host(out["energy"]), e_want, 1e-5)
    assert_rel("R_t", to_host(out["resid"]), r_want, 1e-5)


@pytest.mark.parametrize("impl", ["fused", "unfused"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_single_step_and_norms(impl, dtype):
    api = _api()
    shape, bc = (70, 20, 12), 1
    u0, f = rand_fields(shape, 7)
    if dtype == torch.float32:
        u0, f = f32_round(u0), f32_round(f)
    want, e_want, r_want = oracle.run(u0, f, BASE, 1, bc)
    say("single step", impl, dtype)
    out, n2 = api.step(to_dev(u0, dtype), to_dev(f, dtype), BASE, bc, impl=impl, norms=True)
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert_normwise("u_1", to_host(out), want, 0 if (impl == "unfused" and dtype == torch.float64) else tol)
    n2 = to_host(n2)
    assert_rel("E_1", n2[0], e_want[0], tol)
    assert_rel("R_1", np.sqrt(n2[1]), r_want[0], tol)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", BCS)
def test_run_equals_repeated_steps_and_checkpoints(dtype, bc):
    api = _api()
    shape, T, k = (130, 36, 20), 7, 3
    u0, f = rand_fields(shape, 11)
    fd = to_dev(f, dtype)
    say("run vs steps", dtype, bc)
    states = [to_dev(u0, dtype)]
    for _ in range(T):
        nxt, _ = api.step(states[-1], fd, BASE, bc, impl="fused")
        states.append(nxt)
    u_plain = to_dev(u0, dtype)
    api.run(u_plain, fd, BASE, T, bc, norms=False)
    u_ck = to_dev(u0, dtype)
    out = api.run(u_ck, fd, BASE, T, bc, norms=True, ckpt_every=k)
    torch.cuda.synchronize()
    assert torch.equal(u_plain, states[-1])
    assert torch.equal(u_ck, states[-1])
    ck = out["ckpt"]
    assert ck.shape[0] == 3
    for c in range(ck.shape[0]):
        assert torch.equal(ck[c], states[c * k])


# whole-row tiles and x-segments, both boundary rules: repeated runs of the
# multi-step passes (whose LDS buffers are reused plane after plane) must
# give the same states and norms bit for bit
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(96, 48, 40), (600, 37, 40)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_run_is_bitwise_reproducible(dtype, shape, bc):
    api = _api()
    T = 8
    u0, f = rand_fields(shape, 12)
    say("reproducible", dtype, shape, bc)
    res = []
    fd = to_dev(f, dtype)
    for _ in range(10):
        u = to_dev(u0, dtype)
        out = api.run(u, fd, BASE, T, bc, norms=True)
        res.append((u, out["energy"], out["resid"]))
    torch.cuda.synchronize()
    for u, e, r in res[1:]:
        assert torch.equal(u, res[0][0]) and torch.equal(e, res[0][1]) and torch.equal(r, res[0][2])


@pytest.mark.parametrize("impl", ["fused", "unfused"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_unaligned_pointers_take_the_scalar_path_with_same_result(impl, dtype):
    api = _api()
    shape, bc = (64, 24, 20), 0
    u0, f = rand_fields(shape, 13)
    say("unaligned", impl, dtype)
    ua, fa = to_dev(u0, dtype), to_dev(f, dtype)
    oa, na = api.step(ua, fa, BASE, bc, impl=impl, norms=True)
    um, fm = misaligned_like(ua), misaligned_like(fa)
    om, nm = api.step(um, fm, BASE, bc, impl=impl, norms=True)
    torch.cuda.synchronize()
    assert torch.equal(oa, om)
    assert torch.allclose(na, nm, rtol=1e-13, atol=0)


def test_zero_steps_and_empty_grids():
    api = _api()
    u0, f = rand_fields((9, 8, 7), 14)
    u = to_dev(u0)
    out = api.run(u, to_dev(f), BASE, 0, 1, norms=True)
    assert out["energy"].numel() == 0
    assert np.array_equal(to_host(u), u0)
    say("empty grid")
    e = torch.empty((0, 4, 4), dtype=torch.float64, device=DEV)
    out = api.run(e, torch.empty_like(e), BASE, 3, 0, norms=True)
    _, n2 = api.step(e, torch.empty_like(e), BASE, 0, norms=True)
    torch.cuda.synchronize()
    assert torch.equal(out["energy"], torch.zeros(3, dtype=torch.float64, device=DEV))
    assert torch.equal(out["resid"], torch.zeros(3, dtype=torch.float64, device=DEV))
    assert torch.equal(n2, torch.zeros(2, dtype=torch.float64, device=DEV))


def test_nan_propagates_to_norms():
    api = _api()
    u0, f = rand_fields((40, 30, 20), 15)
    u0[3, 4, 5] = np.nan
    out = api.run(to_dev(u0), to_dev(f), BASE, 3, 1, norms=True)
    torch.cuda.synchronize()
    assert torch.isnan(out["energy"]).all() and torch.isnan(out["resid"]).all()


def test_python_binding_rejects_bad_tensors():
    api = _api()
    u = torch.zeros((4, 4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(TypeError):
        api.step(u.to(torch.int32), u.to(torch.int32), BASE, 0)
    with pytest.raises(ValueError):
        api.step(u, torch.zeros((4, 4, 5), dtype=torch.float64, device=DEV), BASE, 0)
    with pytest.raises(ValueError):
        api.step(u.transpose(0, 2), u, BASE, 0)
    with pytest.raises(ValueError):
        api.step(u.cpu(), u.cpu(), BASE, 0)
    with pytest.raises(api.DcpError):
        api.run(u, u.clone(), BASE, 3, 0, tblock=1000)


# ------------------------------------------------------------ two-step passes
TB_SHAPES = [(64, 64, 64), (512, 24, 10), (256, 17, 70), (128, 5, 3), (8, 3, 2), (4, 1, 1),
             (67, 33, 17), (1024, 9, 6)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", TB_SHAPES)
def test_two_step_passes_equal_single_steps_bitwise(shape, bc, dtype):
    # a two-step pass computes every point with the same operations as the
    # one-step kernel, so the state must match bit for bit (odd T exercises
    # the single-step tail; shapes the pass does not support fall back)
    api = _api()
    u0, f = rand_fields(shape, 500 + sum(shape))
    T = 7
    say("tblock", shape, bc, dtype)
    fd = to_dev(f, dtype)
    u1, u2 = to_dev(u0, dtype), to_dev(u0, dtype)
    o1 = api.run(u1, fd, BASE, T, bc, tblock=1, norms=True)
    o2 = api.run(u2, fd, BASE, T, bc, tblock=2, norms=True)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    rt = 1e-12 if dtype == torch.float64 else 1e-6
    assert torch.allclose(o1["energy"], o2["energy"], rtol=rt, atol=0)
    assert torch.allclose(o1["resid"], o2["resid"], rtol=10 * rt, atol=0)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(64, 64, 64), (256, 17, 70), (512, 24, 10)])
def test_two_step_passes_match_oracle(shape, bc):
    api = _api()
    u0, f = rand_fields(shape, 600 + sum(shape))
    T = 8
    want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
    say("tblock vs oracle", shape, bc)
    u = to_dev(u0)
    out = api.run(u, to_dev(f), BASE, T, bc, tblock=2, norms=True)
    torch.cuda.synchronize()
    assert_normwise("u_T", to_host(u), want, 1e-12)
    assert_rel("E_t", to_host(out["energy"]), e_want, 1e-12)
    assert_rel("R_t", to_host(out["resid"]), r_want, 1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_two_step_passes_with_checkpoints(k):
    api = _api()
    shape, T, bc = (128, 20, 18), 9, 1
    u0, f = rand_fields(shape, 700 + k)
    fd = to_dev(f)
    say("tblock ckpt", k)
    u1, u2 = to_dev(u0), to_dev(u0)
    o1 = api.run(u1, fd, BASE, T, bc, tblock=1, norms=False, ckpt_every=k)
    o2 = api.run(u2, fd, BASE, T, bc, tblock=2, norms=False, ckpt_every=k)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    assert torch.equal(o1["ckpt"], o2["ckpt"])


@pytest.mark.parametrize("impl,tblock", [("fused", 2), ("fused", 1), ("unfused", 1)])
def test_plain_workload_64_dirichlet(impl, tblock):
    # the plain workload as stated: 64^3 float64, ghost-zero boundary, u0 and
    # f uniform from the seeded streams, T = 10, forward only
    from paper_2107_00555_amd import inputs
    api = _api()
    w = inputs.WORKLOADS["plain_64"]
    u0, f = inputs.make_fields("plain_64", seed=0)
    T, bc = w["T"], w["bc"]
    want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
    say("plain workload", impl, tblock)
    u = to_dev(u0)
    out = api.run(u, to_dev(f), BASE, T, bc, impl=impl, tblock=tblock, norms=True)
    torch.cuda.synchronize()
    if impl == "unfused":
        assert np.array_equal(to_host(u), want)
    else:
        assert_normwise("u_10", to_host(u), want, 1e-12)
    assert_rel("E_t", to_host(out["energy"]), e_want, 1e-12)
    assert_rel("R_t", to_host(out["resid"]), r_want, 1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("k", [1, 2, 3])
def test_norms_do_not_depend_on_checkpoints(k, bc, dtype):
    # a two-step pass that also stores its middle state as a checkpoint must
    # still reduce the norms of both of its steps
    api = _api()
    shape, T = (96, 20, 14), 9
    u0, f = rand_fields(shape, 720 + k)
    fd = to_dev(f, dtype)
    say("norms with checkpoints", k, bc, dtype)
    u1, u2 = to_dev(u0, dtype), to_dev(u0, dtype)
    o1 = api.run(u1, fd, BASE, T, bc, tblock=2, norms=True)
    o2 = api.run(u2, fd, BASE, T, bc, tblock=2, norms=True, ckpt_every=k)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    assert torch.equal(o1["energy"], o2["energy"])
    assert torch.equal(o1["resid"], o2["resid"])


# rows that are not a power of two of 16-byte chunks (irregular row ends
# inside a wave), and a grid whose z-runs are long (many rotations of the
# register queues and of the level-1 plane buffers)
TB_ODD_SHAPES = [((70, 33, 21), torch.float64), ((100, 29, 19), torch.float32), ((64, 256, 64), torch.float64),
                 ((64, 256, 64), torch.float32), ((40, 128, 256), torch.float64)]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape,dtype", TB_ODD_SHAPES)
def test_two_step_passes_irregular_rows_and_long_runs(shape, dtype, bc):
    api = _api()
    u0, f = rand_fields(shape, 800 + sum(shape))
    T = 9
    say("tblock irregular", shape, dtype, bc)
    fd = to_dev(f, dtype)
    u1, u2 = to_dev(u0, dtype), to_dev(u0, dtype)
    o1 = api.run(u1, fd, BASE, T, bc, tblock=1, norms=True)
    o2 = api.run(u2, fd, BASE, T, bc, tblock=2, norms=True)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    rt = 1e-12 if dtype == torch.float64 else 1e-6
    assert torch.allclose(o1["energy"], o2["energy"], rtol=rt, atol=0)
    assert torch.allclose(o1["resid"], o2["resid"], rtol=rt, atol=0)
    if dtype == torch.float64:
        want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
        assert_normwise("u_T", to_host(u2), want, 1e-12)
        assert_rel("E_t", to_host(o2["energy"]), e_want, 1e-12)
        assert_rel("R_t", to_host(o2["resid"]), r_want, 1e-12)
