"""The binding's buffer checks on the device: api.run and api.adjoint_run
refuse a checkpoint store or a dL/du0 buffer that does not match what the
library writes or reads, before the library is called (the outputs are
untouched)."""
import pytest
import torch

from gpu_util import BASE, DEV, rand_fields, say, to_dev

pytestmark = pytest.mark.gpu

SHAPE, T, K = (24, 10, 8), 7, 3     # ceil(7/3) = 3 checkpoint slots


def _api():
    from paper_2107_00555_amd import api
    return api


def _ckpt(slots=3, dtype=torch.float64, device=DEV):
    nx, ny, nz = SHAPE
    return torch.full((slots, nz, ny, nx), -7.0, dtype=dtype, device=device)


@pytest.mark.parametrize("bad", ["few", "many", "dtype", "host", "strided"])
def test_run_refuses_a_mismatched_checkpoint_store(bad):
    api = _api()
    u0, f = rand_fields(SHAPE, 31)
    u, fd = to_dev(u0), to_dev(f)
    ck = {"few": lambda: _ckpt(2), "many": lambda: _ckpt(4), "dtype": lambda: _ckpt(dtype=torch.float32),
          "host": lambda: _ckpt(device="cpu"),
          "strided": lambda: _ckpt(6)[::2]}[bad]()
    say("run with bad ckpt", bad)
    with pytest.raises(ValueError):
        api.run(u, fd, BASE, T, 0, norms=False, ckpt_every=K, ckpt=ck)
    torch.cuda.synchronize()
    assert torch.equal(u, to_dev(u0))           # nothing ran
    assert bool((ck == -7.0).all())


@pytest.mark.parametrize("bad", ["few", "dtype", "host", "grad_shape", "grad_dtype", "grad_host"])
def test_adjoint_refuses_mismatched_buffers(bad):
    api = _api()
    u0, f = rand_fields(SHAPE, 32)
    u, fd = to_dev(u0), to_dev(f)
    out = api.run(u, fd, BASE, T, 0, norms=False, ckpt_every=K)
    ck, g = out["ckpt"], None
    lam = u.clone()
    if bad == "few":
        ck = ck[:2]
    elif bad == "dtype":
        ck = ck.float()
    elif bad == "host":
        ck = ck.cpu()
    elif bad == "grad_shape":
        g = torch.empty((SHAPE[2], SHAPE[1], SHAPE[0] + 2), dtype=torch.float64, device=DEV)
    elif bad == "grad_dtype":
        g = torch.empty_like(lam, dtype=torch.float32)
    else:
        g = torch.empty_like(lam, device="cpu")
    say("adjoint with bad buffer", bad)
    with pytest.raises(ValueError):
        api.adjoint_run(ck, K, fd, lam, BASE, T, 0, grad_u0=g)
    with pytest.raises(ValueError):
        api.adjoint_run(None if bad in ("few", "dtype", "host") else ck, K, fd, lam, BASE, T, 0, grad_u0=g)
