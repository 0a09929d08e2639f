"""Shared helpers for the GPU tests (test-side only)."""
from __future__ import annotations

import sys

import numpy as np
import torch

DEV = torch.device("cuda:0")
BASE = dict(alpha=1.0, beta=0.1, gamma=0.5, h=1.0, dt=0.1)


def say(*a):
    """Name the case before a GPU step, flushed, so a crash still shows it."""
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray, dtype=torch.float64) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).numpy()


def f32_round(a: np.ndarray) -> np.ndarray:
    """Round to float32 (nearest even) and widen back exactly."""
    return a.astype(np.float32).astype(np.float64)


def normwise(a: np.ndarray, b: np.ndarray) -> float:
    """max|a-b| / max|b|: the error measure used for fields (pointwise
    relative error is unbounded where the field crosses zero)."""
    den = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b))) / den if den > 0 else float(np.max(np.abs(a - b), initial=0.0))


def rand_fields(shape, seed):
    nx, ny, nz = shape
    r = np.random.default_rng(seed)
    return r.uniform(-1, 1, (nz, ny, nx)), r.uniform(-1, 1, (nz, ny, nx))


def misaligned_like(a: torch.Tensor) -> torch.Tensor:
    """A contiguous copy of a whose data pointer is NOT 16-byte aligned."""
    buf = torch.empty(a.numel() + 1, dtype=a.dtype, device=a.device)
    v = buf[1:].view(a.shape)
    v.copy_(a)
    assert v.data_ptr() % 16 != 0
    return v


def progress(config, *a):
    """Print past pytest's output capture (a long full-size case reports its
    progress while it runs instead of staying silent for minutes)."""
    cap = config.pluginmanager.getplugin("capturemanager")
    if cap is None:
        say(*a)
        return
    with cap.global_and_fixture_disabled():
        say(*a)


def rel_err(a, b) -> float:
    """Largest |a_i - b_i| / |b_i| over a sequence of scalars."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / np.abs(b)))


def assert_rel(name: str, got, want, tol: float) -> float:
    """Assert max_i |got_i - want_i| / |want_i| <= tol, printing the achieved
    error (scalars or sequences of scalars)."""
    err = rel_err(np.atleast_1d(np.asarray(got, dtype=np.float64)),
                  np.atleast_1d(np.asarray(want, dtype=np.float64)))
    print(f"{name}: relative error {err:.3e} (bound {tol:.0e})")
    assert err <= tol, (name, err, tol)
    return err


def assert_normwise(name: str, got: np.ndarray, want: np.ndarray, tol: float) -> float:
    """Assert the normwise field error max|a-b|/max|b| <= tol, printing it."""
    err = normwise(got, want)
    print(f"{name}: normwise error {err:.3e} (bound {tol:.0e})")
    assert err <= tol, (name, err, tol)
    return err
