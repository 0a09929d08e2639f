"""The streaming probe moves what it claims: a copy reproduces its input,
two reads and a write give the sum, a fill writes the constant pattern."""
import ctypes

import pytest
import torch

from gpu_util import DEV, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nt", [0, 1])
def test_stream_probe_results(nt):
    from paper_2107_00555_amd import _lib
    L = _lib.lib()
    n = (1 << 20) + 4096          # elements (doubles): 8 MiB + 32 KiB, a ragged last grid stride
    nbytes = n * 8
    say("stream probe", nt)
    a = torch.rand(n, dtype=torch.float64, device=DEV)
    b = torch.rand(n, dtype=torch.float64, device=DEV)
    o = torch.zeros(n, dtype=torch.float64, device=DEV)
    st = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert L.dcp_stream_probe(0, nt, P(a), None, P(o), nbytes, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(o, a)
    assert L.dcp_stream_probe(1, nt, P(a), P(b), P(o), nbytes, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(o, a + b)
    assert L.dcp_stream_probe(3, nt, None, None, P(o), nbytes, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(o, torch.tensor([1.0, 2.0], dtype=torch.float64, device=DEV).repeat(n // 2))
    o.zero_()
    assert L.dcp_stream_probe(2, nt, P(a), None, P(o), nbytes, st) == 0   # finite data: nothing written
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(o)) == 0
