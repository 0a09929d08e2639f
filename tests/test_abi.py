"""libdcp C ABI, host side: the library loads, exports every function that
include/dcp.h declares, sizes workspaces, and rejects bad arguments before
enqueuing anything.  No GPU needed: every call below fails validation, so
no HIP call is made (the device pointers are never dereferenced)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2107_00555_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2107_00555_amd import build
        build.build(verbose=False)
    return _lib


def header_functions():
    text = open(os.path.join(ROOT, "include", "dcp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dcp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_four_entry_points():
    names = header_functions()
    for n in ("dcp_step_fused", "dcp_step_unfused", "dcp_run", "dcp_adjoint_run",
              "dcp_workspace_bytes", "dcp_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    for n in header_functions():
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value


def test_status_strings(L):
    lib = L.lib()
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -100):
        assert lib.dcp_status_string(s)
    assert lib.dcp_status_string(12345) == b"unknown status"


def test_workspace_sizes(L):
    GiB = 1 << 30
    w = L.workspace_bytes(L.OP_RUN, L.F64, 512, 512, 512, T=100, norms=True)
    assert GiB <= w < GiB + (64 << 20)            # one field plus small partials
    w = L.workspace_bytes(L.OP_RUN, L.F64, 512, 512, 512, T=100, norms=False, impl=L.UNFUSED)
    assert w == 4 * GiB                            # ping-pong field + 3 temporaries
    w = L.workspace_bytes(L.OP_RUN, L.F32, 512, 512, 512, T=100, norms=False)
    assert w == GiB // 2
    assert L.workspace_bytes(L.OP_STEP_FUSED, L.F64, 64, 64, 64) == 0
    w = L.workspace_bytes(L.OP_ADJOINT, L.F64, 256, 256, 256, T=50, ckpt_every=10)
    assert 11 * 128 * (1 << 20) <= w < 11 * 128 * (1 << 20) + (16 << 20)  # 2 lambdas + 9 states
    assert L.workspace_bytes(L.OP_RUN, L.F64, 0, 5, 5, T=3, norms=True) == 0
    assert L.workspace_bytes(L.OP_RUN, L.F64, 4, 4, 4, T=0, norms=True) == 0


@pytest.mark.parametrize("args,code", [
    (dict(op=9), -5), (dict(dtype=7), -3), (dict(nx=-1), -2), (dict(T=-1), -5),
    (dict(op=3, ckpt_every=0), -5), (dict(tblock=0), -5), (dict(impl=5), -5),
    (dict(nx=1 << 40), -2),
])
def test_workspace_bytes_errors(L, args, code):
    a = dict(op=L.OP_RUN, dtype=L.F64, impl=L.FUSED, nx=8, ny=8, nz=8, T=4, ckpt_every=2,
             tblock=1, norms=1)
    a.update(args)
    out = ctypes.c_size_t(0)
    rc = L.lib().dcp_workspace_bytes(a["op"], a["dtype"], a["impl"], a["nx"], a["ny"], a["nz"],
                                     a["T"], a["ckpt_every"], a["tblock"], a["norms"],
                                     ctypes.byref(out))
    assert rc == code
    assert L.lib().dcp_workspace_bytes(0, 0, 0, 4, 4, 4, 1, 1, 1, 0, None) == -1


# Fake, never-dereferenced device addresses, far apart (no overlap).
U, F, O, WS = 0x10000000, 0x20000000, 0x30000000, 0x40000000
C = None


@pytest.fixture
def host_only():
    """Calls with the placeholder addresses are all rejected (or are no-ops)
    before any device work; run them only where no GPU is visible, so a
    regression in a check could never reach a launch."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("placeholder device addresses: host-only check")


def coeffs(L, **kw):
    d = dict(alpha=1.0, beta=0.1, gamma=0.5, h=1.0, dt=0.1)
    d.update(kw)
    return L.Coeffs.make(d)


def step_call(L, fn="dcp_step_fused", dtype=0, u=U, f=F, o=O, n=(8, 8, 8), c=None, bc=0,
              norms=None, ws=WS, wsb=1 << 26):
    c = coeffs(L) if c is None else c
    return getattr(L.lib(), fn)(dtype, u, f, o, n[0], n[1], n[2], ctypes.byref(c), bc, norms, ws,
                                wsb, None)


@pytest.mark.parametrize("fn", ["dcp_step_fused", "dcp_step_unfused"])
def test_step_argument_errors(L, fn, host_only):
    assert step_call(L, fn, dtype=2) == -3
    assert step_call(L, fn, n=(-1, 8, 8)) == -2
    assert step_call(L, fn, bc=3) == -4
    assert step_call(L, fn, u=None) == -1
    assert step_call(L, fn, o=None) == -1
    assert step_call(L, fn, c=coeffs(L, h=0.0)) == -5
    assert step_call(L, fn, c=coeffs(L, alpha=float("nan"))) == -5
    assert step_call(L, fn, c=coeffs(L, dt=float("inf"))) == -5
    assert step_call(L, fn, o=U) == -7                       # u_out aliases u
    assert step_call(L, fn, o=F + 8) == -7                   # u_out overlaps f
    lib = L.lib()
    assert getattr(lib, fn)(0, U, F, O, 8, 8, 8, None, 0, None, None, 0, None) == -1  # no coeffs
    # norms requested without a workspace
    assert step_call(L, fn, norms=0x50000000, ws=None, wsb=0) == -6
    assert step_call(L, fn, norms=0x50000000, ws=None, wsb=1 << 30) == -1
    # workspace overlapping an input
    if fn == "dcp_step_unfused":
        assert step_call(L, fn, ws=None, wsb=0) == -6        # unfused always needs temporaries
        assert step_call(L, fn, ws=U, wsb=1 << 20) == -7


def run_call(L, dtype=0, impl=0, u=U, f=F, n=(8, 8, 8), c=None, bc=1, T=4, tblock=1, energy=None,
             resid=None, ckpt=None, k=0, ws=WS, wsb=1 << 24):
    c = coeffs(L) if c is None else c
    return L.lib().dcp_run(dtype, impl, u, f, n[0], n[1], n[2], ctypes.byref(c), bc, T, tblock,
                           energy, resid, ckpt, k, ws, wsb, None)


def test_run_argument_errors(L, host_only):
    assert run_call(L, T=-1) == -5
    assert run_call(L, impl=2) == -5
    assert run_call(L, tblock=0) == -5
    assert run_call(L, tblock=L.lib().dcp_max_tblock(0) + 1) == -5
    assert run_call(L, ckpt=0x50000000, k=0) == -5
    assert run_call(L, f=U) == -7                                 # f aliases u
    assert run_call(L, ckpt=U + 64, k=2) == -7                    # checkpoints overlap u
    assert run_call(L, ws=F) == -7                                # workspace overlaps f
    assert run_call(L, wsb=16) == -6
    assert run_call(L, u=None) == -1
    assert run_call(L, energy=0x50000000, resid=0x50000008) == -7  # norm outputs overlap
    assert run_call(L, bc=-1) == -4
    assert run_call(L, dtype=-1) == -3


def adj_call(L, dtype=0, ckpt=0x50000000, k=2, f=F, lam=U, n=(8, 8, 8), c=None, bc=0, T=4, tb=1,
             g=O, gab=0x60000000, gf=None, gg=None, ws=WS, wsb=1 << 26):
    c = coeffs(L) if c is None else c
    return L.lib().dcp_adjoint_run(dtype, ckpt, k, f, lam, n[0], n[1], n[2], ctypes.byref(c), bc,
                                   T, tb, g, gab, gf, gg, ws, wsb, None)


def test_adjoint_argument_errors(L, host_only):
    assert adj_call(L, k=0) == -5
    assert adj_call(L, T=-2) == -5
    assert adj_call(L, gab=None) == -1
    assert adj_call(L, ckpt=None) == -1
    assert adj_call(L, g=U) == -7          # grad_u0 aliases lam_T
    assert adj_call(L, g=0x50000000) == -7  # grad_u0 overlaps the checkpoints
    assert adj_call(L, wsb=8) == -6
    assert adj_call(L, ws=F) == -7
    assert adj_call(L, c=coeffs(L, beta=float("-inf"))) == -5
    assert adj_call(L, tb=0) == -5
    assert adj_call(L, tb=4) == -5
    assert adj_call(L, gf=F) == -7              # grad_f aliases f
    assert adj_call(L, gf=O + 8) == -7          # grad_f overlaps grad_u0
    assert adj_call(L, gf=WS + 64) == -7        # grad_f inside the workspace
    assert adj_call(L, gf=0x68000000, gg=0x60000008) == -7   # grad_gamma overlaps grad_ab
    assert adj_call(L, gf=0x68000000, gg=0x68000000) == -7   # grad_gamma inside grad_f


def test_adjoint_workspace_for_gamma_without_f(L, host_only):
    base = L.workspace_bytes(L.OP_ADJOINT, L.F64, 64, 64, 64, T=10, ckpt_every=5)
    extra = L.workspace_bytes(L.OP_ADJOINT, L.F64, 64, 64, 64, T=10, ckpt_every=5, norms=True)
    assert extra - base == 64 * 64 * 64 * 8      # one more field for the running sum
    # a call asking for grad_gamma without grad_f needs the larger workspace
    assert adj_call(L, n=(64, 64, 64), T=10, k=5, gg=0x60000010, wsb=base) == -6


# ------------------------------------------------------------------ Jacobi
JA, JB = 0x70000000, 0x78000000


def test_jacobi_workspace_sizes(L):
    assert L.jacobi_workspace_bytes(1, 24000, 1, 1000) == 2 * 24000 * 8   # two array copies
    assert L.jacobi_workspace_bytes(2, 1300, 1300, 1000) == 2 * 1300 * 1300 * 8 + 2 * 128
    assert L.jacobi_workspace_bytes(2, 1300, 7, 1000, 16) == 2 * 72960   # 72800 B rounded up to 256
    for args in ((1, 24000, 1, 1), (1, 24000, 1, 0), (1, 24000, 1, -3), (1, 2, 1, 50),
                 (2, 2, 900, 50), (2, 900, 2, 50), (2, 0, 0, 50)):
        assert L.jacobi_workspace_bytes(*args) == 0   # no pass runs


@pytest.mark.parametrize("args,code", [
    ((3, 10, 10, 5, 0), -5), ((0, 10, 10, 5, 0), -5),   # dims
    ((1, -1, 1, 5, 0), -2), ((2, 10, -1, 5, 0), -2),     # extents
    ((2, 1 << 40, 1 << 40, 5, 0), -2),                   # size overflow
    ((1, 10, 1, 5, -1), -5), ((1, 10, 1, 5, 257), -5), ((2, 10, 10, 5, 17), -5),  # tblock
])
def test_jacobi_workspace_errors(L, args, code):
    out = ctypes.c_size_t(0)
    assert L.lib().dcp_jacobi_workspace_bytes(*args, ctypes.byref(out)) == code


def j1(L, T=5, A=JA, B=JB, n=100, tb=0, ws=WS, wsb=1 << 26):
    return L.lib().dcp_jacobi_1d(T, A, B, n, tb, ws, wsb, None)


def j2(L, T=5, A=JA, B=JB, n0=40, n1=50, tb=0, ws=WS, wsb=1 << 26):
    return L.lib().dcp_jacobi_2d(T, A, B, n0, n1, tb, ws, wsb, None)


def test_jacobi_argument_errors(L, host_only):
    for call in (j1, j2):
        assert call(L, A=None) == -1
        assert call(L, B=None) == -1
        assert call(L, B=JA + 8) == -7          # B overlaps A
        assert call(L, ws=JB + 64) == -7        # workspace overlaps B
        assert call(L, wsb=64) == -6
        assert call(L, ws=None) == -1
        assert call(L, tb=-1) == -5
    assert j1(L, tb=257) == -5
    assert j2(L, tb=17) == -5
    assert j1(L, n=-4) == -2
    assert j2(L, n1=-4) == -2


def test_jacobi_noop_calls_enqueue_nothing(L, host_only):
    # no pass runs: OK without a workspace and without touching the arrays
    # (the addresses are not device memory, so any access would fail)
    assert j1(L, T=1, ws=None, wsb=0) == 0
    assert j1(L, T=-7, ws=None, wsb=0) == 0
    assert j1(L, n=2, ws=None, wsb=0) == 0
    assert j1(L, n=0, A=None, B=None, ws=None, wsb=0) == 0
    assert j2(L, T=0, ws=None, wsb=0) == 0
    assert j2(L, n0=2, ws=None, wsb=0) == 0
    assert j2(L, n1=1, ws=None, wsb=0) == 0


def test_jacobi_plan(L):
    assert L.jacobi_plan(1, 24000, 1, 1000) == (32, 64)      # 999 iterations, 32 passes of 31-32
    assert L.jacobi_plan(1, 24000 * 1296, 1, 1000) == (16, 126)
    assert L.jacobi_plan(2, 1300, 1300, 1000) == (168, 12)
    assert L.jacobi_plan(2, 1300, 1300, 1000, 1) == (1998, 1)
    assert L.jacobi_plan(2, 1300, 1300, 2, 8) == (2, 1)      # one iteration: split at the half-step
    assert L.jacobi_plan(1, 2, 1, 50) == (0, 0)
    assert L.jacobi_plan(2, 50, 50, 1) == (0, 0)
    for dims, n0, n1, T, tb in ((1, 5000, 1, 77, 5), (2, 300, 200, 33, 7), (1, 10, 1, 3, 256)):
        P, hh = L.jacobi_plan(dims, n0, n1, T, tb)
        assert P % 2 == 0 and 1 <= hh <= tb
        assert P * hh >= 2 * (T - 1)
    n = ctypes.c_int64(0)
    h = ctypes.c_int32(0)
    assert L.lib().dcp_jacobi_plan(2, 10, 1 << 30, 5, 0, ctypes.byref(n), ctypes.byref(h)) == -2
    assert L.lib().dcp_jacobi_plan(2, 10, 10, 5, 0, None, ctypes.byref(h)) == -1


# ------------------------------------------------ binomial checkpointing
def test_revolve_workspace_sizes(L):
    MiB = 1 << 20
    fb = 64 * 64 * 64 * 8                       # 2 MiB per field
    w = L.revolve_workspace_bytes(L.F64, 64, 64, 64, 10, 3)
    assert 8 * fb <= w < 8 * fb + 4 * MiB       # u0, 3 slots, work, scratch, 2 adjoint fields
    w2 = L.revolve_workspace_bytes(L.F64, 64, 64, 64, 10, 3, lsum_field=True)
    assert w2 - w == fb
    assert L.revolve_workspace_bytes(L.F64, 64, 64, 64, 0, 3) == 0
    assert L.revolve_workspace_bytes(L.F32, 0, 64, 64, 10, 3) == 0


def rev_fwd(L, dtype=0, u=U, f=F, n=(8, 8, 8), bc=0, T=5, s=2, tb=1, ws=WS, wsb=1 << 26):
    return L.lib().dcp_revolve_forward(dtype, u, f, n[0], n[1], n[2], ctypes.byref(coeffs(L)), bc, T, s, tb,
                                       ws, wsb, None)


def rev_adj(L, dtype=0, f=F, lam=U, n=(8, 8, 8), bc=0, T=5, s=2, tb=1, g=O, gab=0x60000000, gf=None, gg=None,
            ws=WS, wsb=1 << 26):
    return L.lib().dcp_revolve_adjoint(dtype, f, lam, n[0], n[1], n[2], ctypes.byref(coeffs(L)), bc, T, s, tb,
                                       g, gab, gf, gg, ws, wsb, None)


def test_revolve_argument_errors(L, host_only):
    assert rev_fwd(L, T=-1) == -5
    assert rev_fwd(L, s=-1) == -5
    assert rev_fwd(L, tb=4) == -5
    assert rev_fwd(L, u=None) == -1
    assert rev_fwd(L, f=U) == -7
    assert rev_fwd(L, ws=U + 64) == -7
    assert rev_fwd(L, wsb=64) == -6
    assert rev_fwd(L, bc=7) == -4
    assert rev_fwd(L, dtype=9) == -3
    assert rev_adj(L, T=-1) == -5
    assert rev_adj(L, gab=None) == -1
    assert rev_adj(L, g=None) == -1
    assert rev_adj(L, g=F) == -7
    assert rev_adj(L, ws=O + 8) == -7
    assert rev_adj(L, gf=O) == -7
    assert rev_adj(L, gf=0x68000000, gg=0x60000008) == -7
    assert rev_adj(L, wsb=64) == -6


def test_run_plan_reports_the_passes(L, monkeypatch):
    # which passes dcp_run takes (host-side plan; 160 KiB of LDS without a GPU)
    monkeypatch.delenv("DCP_TBK_CFG", raising=False)
    # three steps per pass; the last four steps as two passes of two
    p = L.run_plan(L.F64, 512, 512, 512, 100, 3)
    assert p["passes"] == [0, 2, 32] and p["steps_per_pass"] == 3
    p = L.run_plan(L.F64, 512, 512, 512, 100, 2)
    assert p["passes"] == [0, 50, 0] and p["steps_per_pass"] == 2 and p["segmented"] == 0
    p = L.run_plan(L.F32, 512, 512, 512, 100, 3)
    assert p["passes"] == [0, 2, 32]
    assert L.run_plan(L.F64, 512, 512, 512, 99, 3)["passes"] == [0, 0, 33]
    assert L.run_plan(L.F64, 512, 512, 512, 98, 3)["passes"] == [0, 1, 32]
    p = L.run_plan(L.F64, 512, 512, 512, 100, 1)
    assert p["passes"] == [100, 0, 0] and p["steps_per_pass"] == 1
    p = L.run_plan(L.F64, 512, 512, 512, 7, 1, impl=L.UNFUSED)
    assert p["passes"] == [7, 0, 0]
    # rows too long for a whole-row tile: two-step passes over x-segments
    for dtype, nx in ((L.F64, 1024), (L.F64, 1030), (L.F32, 2048)):
        p = L.run_plan(dtype, nx, 1024, 512, 200, 2)
        assert p["passes"] == [0, 100, 0] and p["segmented"] == 1, (dtype, nx, p)
    # rows that are not a whole number of 16-byte vectors: one step per pass
    p = L.run_plan(L.F64, 513, 16, 16, 10, 3)
    assert p["passes"] == [10, 0, 0]
    assert L.run_plan(L.F64, 0, 16, 16, 10, 3)["passes"] == [0, 0, 0]
    with pytest.raises(L.DcpError):
        L.run_plan(L.F64, 8, 8, 8, 10, 4)
    with pytest.raises(L.DcpError):
        L.run_plan(L.F64, 8, 8, 8, 10, 2, impl=L.UNFUSED)


def test_three_step_plan_prefers_the_ring_form(L, monkeypatch):
    # the ring form (768 lanes) is the planner's first choice for three-step
    # passes, the plain form (1024 lanes) for two-step passes over
    # x-segments; either stays reachable through the tuning override
    monkeypatch.delenv("DCP_TUNING", raising=False)
    for code, shape in ((L.F64, (512, 512, 512)), (L.F32, (1024, 1024, 512)), (L.F64, (64, 64, 64)),
                        (L.F64, (1030, 17, 9)), (L.F32, (8, 3, 2))):
        p = L.run_plan(code, *shape, 100, 3)
        assert p["steps_per_pass"] == 3 and p["lanes"] == 768, (shape, p)
    p = L.run_plan(L.F64, 1024, 1024, 512, 24, 2)
    assert p["steps_per_pass"] == 2 and p["segmented"] == 1 and p["lanes"] == 1024, p
    monkeypatch.setenv("DCP_TUNING", "1")
    monkeypatch.setenv("DCP_TBK_CFG", "0,0,1024")
    p = L.run_plan(L.F64, 512, 512, 512, 100, 3)
    assert p["steps_per_pass"] == 3 and p["lanes"] == 1024, p
    monkeypatch.setenv("DCP_TBK_CFG", "0,0,768")
    p = L.run_plan(L.F64, 1024, 1024, 512, 24, 2)
    assert p["steps_per_pass"] == 2 and p["lanes"] == 768, p


def test_tuning_overrides_need_the_master_switch(L, monkeypatch):
    # a tiling variable alone changes nothing; with DCP_TUNING=1 it is honoured
    monkeypatch.delenv("DCP_TUNING", raising=False)
    monkeypatch.delenv("DCP_TBK_CFG", raising=False)
    default = L.run_plan(L.F64, 512, 512, 512, 100, 3)
    monkeypatch.setenv("DCP_TBK_CFG", "32,4,512")
    assert L.run_plan(L.F64, 512, 512, 512, 100, 3) == default
    monkeypatch.setenv("DCP_TUNING", "1")
    forced = L.run_plan(L.F64, 512, 512, 512, 100, 3)
    assert forced["segmented"] == 1 and forced["tile_rows"] == 4 and forced["lanes"] == 512, forced
    monkeypatch.setenv("DCP_TUNING", "0")
    assert L.run_plan(L.F64, 512, 512, 512, 100, 3) == default


def test_stream_probe_argument_errors(L):
    lib = L.lib()
    P = ctypes.c_void_p
    a, b, o = P(0x10000000), P(0x50000000), P(0x90000000)
    MiB = 1 << 20
    assert lib.dcp_stream_probe(4, 0, a, b, o, MiB, None) == -5
    assert lib.dcp_stream_probe(-1, 0, a, b, o, MiB, None) == -5
    assert lib.dcp_stream_probe(0, 0, a, b, o, MiB + 8, None) == -5
    assert lib.dcp_stream_probe(0, 0, a, b, o, 0, None) == -5
    assert lib.dcp_stream_probe(2, 0, a, b, o, 4096, None) == -5        # read needs >= 1 MiB
    assert lib.dcp_stream_probe(1, 0, a, None, o, MiB, None) == -1
    assert lib.dcp_stream_probe(0, 0, None, b, o, MiB, None) == -1
    assert lib.dcp_stream_probe(3, 0, None, None, None, MiB, None) == -1
    assert lib.dcp_stream_probe(0, 0, P(0x10000008), b, o, MiB, None) == -5   # misaligned
    assert lib.dcp_stream_probe(0, 0, a, b, P(0x10000000 + MiB // 2), MiB, None) == -7
