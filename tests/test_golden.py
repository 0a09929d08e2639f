"""The oracle reproduces its recorded fixtures bit for bit (CPU), and the
fused GPU path matches them within the FP64 tolerance (GPU)."""
import glob
import json
import os

import numpy as np
import pytest

import oracle
from paper_2107_00555_amd import inputs

FIXTURES = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "oracle_*.json")))


def _load(path):
    g = json.load(open(path))
    u0, f = inputs.make_fields(dict(f=g["f"]), seed=g["seed"], shape=tuple(g["shape_xyz"]))
    return g, u0, f


@pytest.mark.parametrize("path", FIXTURES, ids=os.path.basename)
def test_oracle_reproduces_golden(path):
    g, u0, f = _load(path)
    uT, e, r = oracle.run(u0, f, g["coeffs"], g["T"], g["bc"])
    assert [float(v) for v in g["energy"]] == list(e)
    assert [float(v) for v in g["resid"]] == list(r)
    for x, y, z, v in g["samples"]:
        assert uT[z, y, x] == float(v)
    assert float(np.sum(uT)) == float(g["checksum_sum"])


@pytest.mark.gpu
@pytest.mark.parametrize("tblock", [1, 2])
@pytest.mark.parametrize("path", FIXTURES, ids=os.path.basename)
def test_gpu_matches_golden(path, tblock):
    import torch
    from paper_2107_00555_amd import api
    g, u0, f = _load(path)
    dev = torch.device("cuda:0")
    u = torch.from_numpy(u0).to(dev)
    out = api.run(u, torch.from_numpy(f).to(dev), g["coeffs"], g["T"], g["bc"], tblock=tblock, norms=True)
    torch.cuda.synchronize()
    uh = u.cpu().numpy()
    scale = np.max(np.abs(uh))
    for x, y, z, v in g["samples"]:
        assert abs(uh[z, y, x] - float(v)) <= 1e-12 * scale
    np.testing.assert_allclose(out["energy"].cpu().numpy(), [float(v) for v in g["energy"]], rtol=1e-12)
    np.testing.assert_allclose(out["resid"].cpu().numpy(), [float(v) for v in g["resid"]], rtol=1e-12)
