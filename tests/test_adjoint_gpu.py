"""Adjoint parity: dcp_adjoint_run against the oracle's scatter-transpose
adjoint, checkpoint independence, central differences through the GPU
forward, and torch.autograd.gradcheck through RD3D."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import BASE, DEV, assert_normwise, assert_rel, f32_round, normwise, rand_fields, say, to_dev, to_host
from paper_2107_00555_amd import inputs

pytestmark = pytest.mark.gpu


def _api():
    from paper_2107_00555_amd import api
    return api


def gpu_grad(u0, f, lam, T, bc, k, dtype=torch.float64, coeffs=BASE):
    api = _api()
    u = to_dev(u0, dtype)
    fd = to_dev(f, dtype)
    out = api.run(u, fd, coeffs, T, bc, norms=False, ckpt_every=k)
    g, gab = api.adjoint_run(out["ckpt"], k, fd, to_dev(lam, dtype), coeffs, T, bc)
    return g, gab


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape,T,k", [((24, 20, 16), 7, 3), ((67, 33, 17), 5, 2),
                                       ((130, 18, 9), 4, 4), ((1, 1, 5), 3, 1),
                                       ((3, 2, 70), 6, 10)])
def test_adjoint_f64_matches_oracle(shape, T, k, bc):
    u0, f = rand_fields(shape, 400 + sum(shape))
    lam = np.random.default_rng(1).uniform(-1, 1, u0.shape)
    want, wa, wb = oracle.adjoint(u0, f, lam, BASE, T, bc)
    say("adjoint f64", shape, T, k, bc)
    g, gab = gpu_grad(u0, f, lam, T, bc, k)
    torch.cuda.synchronize()
    assert_normwise("dL/du0", to_host(g), want, 1e-12)
    gab = to_host(gab)
    assert_rel("dL/dalpha", gab[0], wa, 1e-12)
    assert_rel("dL/dbeta", gab[1], wb, 1e-12)


@pytest.mark.parametrize("bc", [0, 1])
def test_adjoint_f32_matches_oracle(bc):
    shape, T, k = (64, 40, 24), 8, 3
    u0, f = rand_fields(shape, 17)
    lam = np.random.default_rng(2).uniform(-1, 1, u0.shape)
    u0, f, lam = f32_round(u0), f32_round(f), f32_round(lam)
    want, wa, wb = oracle.adjoint(u0, f, lam, BASE, T, bc)
    say("adjoint f32", bc)
    g, gab = gpu_grad(u0, f, lam, T, bc, k, torch.float32)
    torch.cuda.synchronize()
    assert normwise(to_host(g), want) <= 1e-5
    gab = to_host(gab)
    assert gab[0] == pytest.approx(wa, rel=1e-5)
    assert gab[1] == pytest.approx(wb, rel=1e-5)


@pytest.mark.parametrize("tblock", [1, 2, 3])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gradient_is_bitwise_independent_of_checkpoint_interval(dtype, tblock):
    api = _api()
    shape, T, bc = (128, 30, 20), 11, 1
    u0, f = rand_fields(shape, 18)
    lam = np.random.default_rng(3).uniform(-1, 1, u0.shape)
    say("k independence", dtype, tblock)
    ref = None
    for k in (1, 2, 3, 4, 10, 25):
        u = to_dev(u0, dtype)
        fd = to_dev(f, dtype)
        out = api.run(u, fd, BASE, T, bc, tblock=tblock, norms=False, ckpt_every=k)
        g, gab = api.adjoint_run(out["ckpt"], k, fd, to_dev(lam, dtype), BASE, T, bc, tblock=tblock)
        if ref is None:
            ref = (g, gab)
        else:
            assert torch.equal(g, ref[0]), k
            assert torch.equal(gab, ref[1]), k


def test_adjoint_zero_steps_copies_seed():
    api = _api()
    lam = to_dev(np.random.default_rng(4).uniform(-1, 1, (5, 6, 7)))
    f = torch.zeros_like(lam)
    g, gab = api.adjoint_run(None, 3, f, lam, BASE, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(g, lam) and torch.equal(gab, torch.zeros_like(gab))


@pytest.mark.parametrize("bc", [0, 1])
def test_gradient_matches_central_differences_on_gpu_forward(bc):
    # loss L = 0.5*||u_T - u_tgt||^2, 8 seeded directions over (u0, alpha, beta)
    api = _api()
    shape, T, k, eps = (40, 32, 24), 12, 5, 1e-6
    nx, ny, nz = shape
    u0, f = inputs.make_fields(dict(f="uniform"), seed=5, shape=shape)
    tgt = inputs.target(nx, ny, nz, seed=5)
    fd, td = to_dev(f), to_dev(tgt)

    def loss(du=None, da=0.0, db=0.0):
        c = dict(BASE, alpha=BASE["alpha"] + da, beta=BASE["beta"] + db)
        u = to_dev(u0) if du is None else to_dev(u0 + du)
        api.run(u, fd, c, T, bc, norms=False)
        return oracle.half_sq_dist(to_host(u), tgt)  # compensated FP64 sum on the host

    say("fd", bc)
    u = to_dev(u0)
    out = api.run(u, fd, BASE, T, bc, norms=False, ckpt_every=k)
    g, gab = api.adjoint_run(out["ckpt"], k, fd, (u - td).contiguous(), BASE, T, bc)
    g, gab = to_host(g), to_host(gab)
    for du, da, db in inputs.fd_directions(nx, ny, nz, seed=5, count=8):
        fdv = (loss(eps * du, eps * da, eps * db) - loss(-eps * du, -eps * da, -eps * db)) / (2 * eps)
        an = float(np.sum(g * du)) + gab[0] * da + gab[1] * db
        assert abs(fdv - an) <= 1e-6 * abs(an)


def test_gradcheck_through_rd3d():
    from paper_2107_00555_amd.autograd import rd3d
    say("gradcheck")
    r = np.random.default_rng(6)
    u0 = torch.tensor(r.uniform(-1, 1, (3, 4, 5)), device=DEV, requires_grad=True)
    f = torch.tensor(r.uniform(-1, 1, (3, 4, 5)), device=DEV)
    alpha = torch.tensor(1.0, dtype=torch.float64, device=DEV, requires_grad=True)
    beta = torch.tensor(0.1, dtype=torch.float64, device=DEV, requires_grad=True)
    for bc in (0, 1):
        fn = lambda u, a, b: rd3d(u, f, a, b, 0.5, 0.1, 1.0, 5, bc, 2)
        assert torch.autograd.gradcheck(fn, (u0, alpha, beta), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_rd3d_backward_matches_oracle():
    from paper_2107_00555_amd.autograd import rd3d
    shape, T, k, bc = (20, 18, 16), 6, 4, 1
    u0, f = rand_fields(shape, 19)
    tgt = np.random.default_rng(7).uniform(-1, 1, u0.shape)
    loss_w, gw, gaw, gbw = oracle.grad_of_half_sq_dist(u0, f, tgt, BASE, T, bc)
    say("rd3d backward")
    u = to_dev(u0).requires_grad_(True)
    alpha = torch.tensor(BASE["alpha"], dtype=torch.float64, device=DEV, requires_grad=True)
    beta = torch.tensor(BASE["beta"], dtype=torch.float64, device=DEV, requires_grad=True)
    uT = rd3d(u, to_dev(f), alpha, beta, BASE["gamma"], BASE["dt"], BASE["h"], T, bc, k)
    loss = 0.5 * torch.sum((uT - to_dev(tgt)) ** 2)
    loss.backward()
    assert float(loss.detach()) == pytest.approx(loss_w, rel=1e-12)
    assert normwise(to_host(u.grad), gw) <= 1e-12
    assert_rel("dL/dalpha", float(alpha.grad), gaw, 1e-12)
    assert_rel("dL/dbeta", float(beta.grad), gbw, 1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape,T,k", [((64, 24, 20), 9, 4), ((128, 20, 18), 8, 3), ((256, 9, 11), 7, 1),
                                       ((512, 12, 6), 6, 6), ((67, 20, 9), 5, 2)])
def test_two_step_adjoint_equals_single_steps(shape, T, k, bc, dtype):
    # paired adjoint passes apply exactly the one-step operations: dL/du0 is
    # bitwise the same; the parameter sums differ only by summation order
    api = _api()
    u0, f = rand_fields(shape, 800 + sum(shape))
    lam = np.random.default_rng(8).uniform(-1, 1, u0.shape)
    fd = to_dev(f, dtype)
    say("two-step adjoint", shape, T, k, bc, dtype)
    res = {}
    for tb in (1, 2, 3):
        u = to_dev(u0, dtype)
        out = api.run(u, fd, BASE, T, bc, tblock=tb, norms=False, ckpt_every=k)
        res[tb] = api.adjoint_run(out["ckpt"], k, fd, to_dev(lam, dtype), BASE, T, bc, tblock=tb)
    torch.cuda.synchronize()
    assert torch.equal(res[1][0], res[2][0])
    assert torch.allclose(res[1][1], res[2][1], rtol=1e-12, atol=0)
    # three-step recomputation passes store the same states: the gradient
    # equals the two-step one bit for bit (the adjoint passes are the same)
    assert torch.equal(res[3][0], res[2][0]) and torch.equal(res[3][1], res[2][1])


@pytest.mark.parametrize("bc", [0, 1])
def test_two_step_adjoint_matches_oracle(bc):
    shape, T, k = (128, 24, 20), 9, 4
    u0, f = rand_fields(shape, 900 + bc)
    lam = np.random.default_rng(9).uniform(-1, 1, u0.shape)
    want, wa, wb = oracle.adjoint(u0, f, lam, BASE, T, bc)
    say("two-step adjoint vs oracle", bc)
    g, gab = gpu_grad(u0, f, lam, T, bc, k)
    torch.cuda.synchronize()
    assert_normwise("dL/du0", to_host(g), want, 1e-12)
    gab = to_host(gab)
    assert_rel("dL/dalpha", gab[0], wa, 1e-12)
    assert_rel("dL/dbeta", gab[1], wb, 1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", [0, 1])
def test_wide_rows_recompute_with_multi_step_passes(bc, dtype):
    # rows too long for whole-row tiles: the recomputation takes multi-step
    # passes over x-segments and the adjoint steps run one per pass, so the
    # whole gradient equals the one-step form bit for bit
    api = _api()
    shape, T, k = (1030 if dtype == torch.float64 else 2052, 11, 9), 10, 5
    u0, f = rand_fields(shape, 950 + bc)
    lam = np.random.default_rng(95).uniform(-1, 1, u0.shape)
    fd = to_dev(f, dtype)
    say("wide-row recomputation", shape, bc, dtype)
    res = {}
    for tb in (1, 3):
        u = to_dev(u0, dtype)
        out = api.run(u, fd, BASE, T, bc, tblock=tb, norms=False, ckpt_every=k)
        res[tb] = api.adjoint_run(out["ckpt"], k, fd, to_dev(lam, dtype), BASE, T, bc, tblock=tb)
    torch.cuda.synchronize()
    assert torch.equal(res[1][0], res[3][0]) and torch.equal(res[1][1], res[3][1])
    if dtype == torch.float64:
        want, wa, wb = oracle.adjoint(u0, f, lam, BASE, T, bc)
        assert_normwise("dL/du0", to_host(res[3][0]), want, 1e-12)
        gab = to_host(res[3][1])
        assert_rel("dL/dalpha", gab[0], wa, 1e-12)
        assert_rel("dL/dbeta", gab[1], wb, 1e-12)
