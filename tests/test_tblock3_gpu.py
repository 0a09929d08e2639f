"""Passes of several fused steps through the B-step kernel: three steps per
pass (tblock = 3) and two-step passes over x-segments for rows too long to
hold whole in LDS.  Every point of a pass is computed with the operations of
the one-step kernel, so the states must equal one-step runs bit for bit
(odd remainders of T run as shorter passes); the norms are summed in
another order (per tile) and agree to rounding.  A few cases also go
against the oracle at the stated tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import BASE, assert_normwise, assert_rel, rand_fields, say, to_dev, to_host

pytestmark = pytest.mark.gpu

BCS = [0, 1]


def _api():
    from paper_2107_00555_amd import api
    return api


def _same_as_single_steps(shape, dtype, bc, T, tblock, seed, ckpt_every=0):
    api = _api()
    u0, f = rand_fields(shape, seed)
    fd = to_dev(f, dtype)
    u1, u2 = to_dev(u0, dtype), to_dev(u0, dtype)
    o1 = api.run(u1, fd, BASE, T, bc, tblock=1, norms=True, ckpt_every=ckpt_every)
    o2 = api.run(u2, fd, BASE, T, bc, tblock=tblock, norms=True, ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    if ckpt_every:
        assert torch.equal(o1["ckpt"], o2["ckpt"])
    rt = 1e-12 if dtype == torch.float64 else 1e-6
    assert torch.allclose(o1["energy"], o2["energy"], rtol=rt, atol=0)
    assert torch.allclose(o1["resid"], o2["resid"], rtol=rt, atol=0)
    return u0, f, u2, o2


SHAPES3 = [(64, 64, 64), (512, 24, 10), (256, 17, 70), (128, 5, 3), (8, 3, 2), (4, 1, 1), (67, 33, 17),
           (70, 33, 21), (100, 29, 19), (40, 128, 64), (1024, 9, 6)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES3)
def test_three_step_passes_equal_single_steps_bitwise(shape, bc, dtype):
    say("tblock 3", shape, bc, dtype)
    for T in (3, 7, 8):  # whole passes, and remainders of one and two steps
        _same_as_single_steps(shape, dtype, bc, T, 3, 1000 + sum(shape) + T)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(64, 64, 64), (256, 17, 70), (512, 24, 10), (70, 33, 21)])
def test_three_step_passes_match_oracle(shape, bc):
    T = 9
    say("tblock 3 vs oracle", shape, bc)
    u0, f, u, out = _same_as_single_steps(shape, torch.float64, bc, T, 3, 1100 + sum(shape))
    want, e_want, r_want = oracle.run(u0, f, BASE, T, bc)
    assert_normwise("u_T", to_host(u), want, 1e-12)
    assert_rel("E_t", to_host(out["energy"]), e_want, 1e-12)
    assert_rel("R_t", to_host(out["resid"]), r_want, 1e-12)


@pytest.mark.parametrize("shape", [(128, 20, 18), (600, 37, 11)])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("bc", BCS)
def test_three_step_passes_store_checkpoints_inside_a_pass(k, bc, shape):
    # checkpoints at the first, second or last step of a pass, norms on;
    # whole-row tiles and x-segments
    say("tblock 3 checkpoints", k, bc, shape)
    for dtype in (torch.float64, torch.float32):
        _same_as_single_steps(shape, dtype, bc, 11, 3, 1200 + k, ckpt_every=k)


# rows longer than a whole-row tile can hold: two-step passes over x-segments
WIDE = [((1024, 20, 12), torch.float64), ((1030, 17, 9), torch.float64), ((2048, 12, 8), torch.float32),
        ((2052, 9, 7), torch.float32), ((4096, 5, 6), torch.float64)]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape,dtype", WIDE)
@pytest.mark.parametrize("tblock", [2, 3])
def test_wide_rows_keep_multi_step_passes(shape, dtype, bc, tblock):
    from paper_2107_00555_amd import _lib
    say("wide rows", shape, dtype, bc, tblock)
    nx, ny, nz = shape
    code = _lib.F64 if dtype == torch.float64 else _lib.F32
    plan = _lib.run_plan(code, nx, ny, nz, 9, tblock)
    assert plan["steps_per_pass"] == tblock and plan["segmented"] == 1, plan
    u0, f, u, out = _same_as_single_steps(shape, dtype, bc, 9, tblock, 1300 + sum(shape))
    if dtype == torch.float64:
        want, e_want, r_want = oracle.run(u0, f, BASE, 9, bc)
        assert_normwise("u_T", to_host(u), want, 1e-12)
        assert_rel("E_t", to_host(out["energy"]), e_want, 1e-12)
        assert_rel("R_t", to_host(out["resid"]), r_want, 1e-12)


# every tiling the B-step kernel compiles: whole rows (a width covering the
# row) or segments of 32 .. 256 chunks, slabs of 4 / 8 / 16 rows, the ring
# form (768 lanes) or the plain form (1024 or 512 lanes), forced through the
# planner's tuning override; each must give the same states (a tiling that
# does not fit the grid leaves one-step passes)
FORCED = [(wc, ty, lanes) for wc in (1 << 20, 32, 64, 128, 256) for ty in (4, 8, 16) for lanes in (768, 1024, 512)]


@pytest.mark.parametrize("wc,ty,lanes", FORCED)
def test_every_tiling_gives_the_same_states(monkeypatch, wc, ty, lanes):
    from paper_2107_00555_amd import _lib
    say("forced tiling", wc, ty, lanes)
    monkeypatch.setenv("DCP_TUNING", "1")
    monkeypatch.setenv("DCP_TBK_CFG", f"{wc},{ty},{lanes}")
    used = 0
    for shape in ((600, 37, 11), (96, 37, 11)):
        for dtype in (torch.float64, torch.float32):
            code = _lib.F64 if dtype == torch.float64 else _lib.F32
            plan = _lib.run_plan(code, *shape, 8, 3)
            if plan["steps_per_pass"] == 3:
                used += 1
                assert plan["tile_rows"] == ty and plan["lanes"] == lanes, plan
                chunks = shape[0] // (2 if dtype == torch.float64 else 4)  # 16-byte chunks per row
                assert plan["segmented"] == (0 if wc >= chunks else 1), plan
            for bc in BCS:
                _same_as_single_steps(shape, dtype, bc, 8, 3, 1400 + ty + shape[0])
    print(f"forced tiling {wc},{ty},{lanes}: three-step passes in {used} of 4 cases")



@pytest.mark.parametrize("sblk", [1, 3, 5, 7, 1000])
def test_tile_order_blocks_cover_every_tile(monkeypatch, sblk):
    # the tile order takes blocks of sblk slabs across all segments (the last
    # block shorter when sblk does not divide the slab count); every order
    # must visit each tile once: states equal one-step runs bit for bit
    say("tile order", sblk)
    monkeypatch.setenv("DCP_TUNING", "1")
    monkeypatch.setenv("DCP_TBK_SBLK", str(sblk))
    for shape, dtype in (((1030, 37, 11), torch.float64), ((600, 29, 9), torch.float32), ((96, 37, 11), torch.float64)):
        for bc in BCS:
            _same_as_single_steps(shape, dtype, bc, 8, 3, 1500 + sblk + shape[1])


@pytest.mark.parametrize("cfg", [0, 1])
def test_every_two_step_configuration(monkeypatch, cfg):
    # the two-step kernel's compiled slab heights (8 and 4 rows, 1024 lanes),
    # forced: forward states and dL/du0 equal one-step passes bit for bit
    api = _api()
    say("two-step configuration", cfg)
    monkeypatch.setenv("DCP_TUNING", "1")
    monkeypatch.setenv("DCP_TB_CFG", str(cfg))
    for dtype in (torch.float64, torch.float32):
        for bc in BCS:
            shape = (96, 37, 11)
            _same_as_single_steps(shape, dtype, bc, 8, 2, 1600 + cfg)
            u0, f = rand_fields(shape, 1700 + cfg)
            lam = np.random.default_rng(17).uniform(-1, 1, u0.shape)
            fd = to_dev(f, dtype)
            res = {}
            for tb in (1, 2):
                u = to_dev(u0, dtype)
                out = api.run(u, fd, BASE, 7, bc, tblock=tb, norms=False, ckpt_every=3)
                res[tb] = api.adjoint_run(out["ckpt"], 3, fd, to_dev(lam, dtype), BASE, 7, bc, tblock=tb)
            torch.cuda.synchronize()
            assert torch.equal(res[1][0], res[2][0])
            rt = 1e-12 if dtype == torch.float64 else 1e-6
            assert torch.allclose(res[1][1], res[2][1], rtol=rt, atol=0)
