"""dcp_step_fused_noalloc: the fused step with the norms' partial sums in the
library's fixed per-GPU scratch instead of a caller workspace.  It runs the
kernels of dcp_step_fused with the same tiles, so its field and norms must
equal dcp_step_fused's bit for bit; two calls in a row (the second on a
smaller grid, with the first call's partial sums still in the scratch) check
that nothing carries over."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import BASE, rand_fields, say, to_dev

ROWS = [
    # (first grid, second grid), both boundaries, both dtypes
    ((96, 70, 33), (40, 24, 20)),
    ((512, 64, 48), (33, 17, 9)),
]


def _lib():
    from paper_2107_00555_amd import _lib
    return _lib


def _via_workspace(u, f, bc):
    from paper_2107_00555_amd import api
    out, n2 = api.step(u, f, BASE, bc, impl="fused", norms=True)
    return out, n2


def _via_noalloc(u, f, bc, norms=True):
    """Through the C ABI with caller-made buffers only."""
    L = _lib()
    out = torch.empty_like(u)
    n2 = torch.full((2,), float("nan"), dtype=torch.float64, device=u.device) if norms else None
    nz, ny, nx = u.shape
    dt = L.F64 if u.dtype == torch.float64 else L.F32
    c = L.Coeffs.make(BASE)
    stream = ctypes.c_void_p(torch.cuda.current_stream(u.device).cuda_stream)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(u.device)
    rc = L.lib().dcp_step_fused_noalloc(dt, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), nx, ny, nz, ctypes.byref(c), bc,
                                        ctypes.c_void_p(n2.data_ptr()) if norms else None, stream)
    torch.cuda.synchronize()
    assert rc == 0, L.lib().dcp_status_string(rc)
    assert torch.cuda.memory_allocated(u.device) == before
    return out, n2


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shapes", ROWS)
def test_noalloc_step_equals_workspace_step(shapes, bc, dtype):
    for i, shape in enumerate(shapes):   # the second call is on a smaller grid
        say("noalloc step", shape, bc, dtype, "call", i + 1)
        u0, f0 = rand_fields(shape, 4000 + 7 * i + sum(shape))
        u, f = to_dev(u0, dtype), to_dev(f0, dtype)
        want, n_want = _via_workspace(u, f, bc)
        got, n_got = _via_noalloc(u, f, bc)
        assert torch.equal(got, want)
        assert torch.equal(n_got, n_want), (n_got, n_want)
        assert np.all(np.isfinite(n_got.cpu().numpy()))


@pytest.mark.gpu
def test_noalloc_step_without_norms_and_through_the_binding():
    from paper_2107_00555_amd import api
    shape = (64, 40, 30)
    u0, f0 = rand_fields(shape, 4100)
    u, f = to_dev(u0), to_dev(f0)
    want, n_want = _via_workspace(u, f, 1)
    got, _ = _via_noalloc(u, f, 1, norms=False)
    assert torch.equal(got, want)
    out = torch.empty_like(u)
    n2 = torch.empty(2, dtype=torch.float64, device=u.device)
    api.step_noalloc(u, f, BASE, 1, out, n2)
    torch.cuda.synchronize()
    assert torch.equal(out, want) and torch.equal(n2, n_want)


def test_noalloc_rejects_grids_beyond_the_scratch():
    # argument checks run before anything touches the device (placeholder
    # addresses, never dereferenced): a grid whose norms need more than the
    # fixed scratch is refused, and other argument errors keep their codes
    L = _lib()
    lib = L.lib()
    c = L.Coeffs.make(BASE)
    P = ctypes.c_void_p
    u, f, o, n2 = P(0x10000000), P(0x20000000), P(0x30000000), P(0x40000000)
    # nx = 1 (one element per lane), 2^24 planes: more than 65536 workgroups of partial sums
    rc = lib.dcp_step_fused_noalloc(L.F64, u, f, o, 1, 16, 1 << 24, ctypes.byref(c), 1, n2, None)
    assert rc == L.E_SCRATCH == -8
    assert b"scratch" in lib.dcp_status_string(rc)
    assert lib.dcp_step_fused_noalloc(7, u, f, o, 8, 8, 8, ctypes.byref(c), 1, n2, None) == -3
    assert lib.dcp_step_fused_noalloc(L.F64, u, f, o, 8, 8, 8, ctypes.byref(c), 5, n2, None) == -4
    assert lib.dcp_step_fused_noalloc(L.F64, None, f, o, 8, 8, 8, ctypes.byref(c), 1, n2, None) == -1
    assert lib.dcp_step_fused_noalloc(L.F64, u, f, o, -1, 8, 8, ctypes.byref(c), 1, n2, None) == -2
    assert lib.dcp_step_fused_noalloc(L.F64, u, f, u, 8, 8, 8, ctypes.byref(c), 1, n2, None) == -7
    ws = L.workspace_bytes(L.OP_STEP_FUSED, L.F64, 1, 16, 1 << 24, norms=True)
    assert ws > L.NOALLOC_SCRATCH_BYTES
    assert L.workspace_bytes(L.OP_STEP_FUSED, L.F32, 1024, 1024, 512, norms=True) <= L.NOALLOC_SCRATCH_BYTES
