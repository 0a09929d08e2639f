"""Binomial checkpointing schedule (dcp_revolve_schedule), host side: every
op reads the state it claims, the adjoint steps come in the order T-1 .. 0,
at most nslots slots are used, and the number of recomputed steps is the
least possible (an exhaustive dynamic program for small T, the binomial
closed form for large T)."""
from functools import lru_cache
from math import comb
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2107_00555_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2107_00555_amd import build
        build.build(verbose=False)
    return _lib


def simulate(ops, T, nslots):
    """Run the schedule on time labels; returns the forward steps taken."""
    buf = {-1: 0}
    expect = T - 1
    steps = 0
    for kind, src, dst, t0, t1 in ops:
        assert src in buf and buf[src] == t0, (kind, src, t0, buf.get(src))
        if kind == 0:
            assert t1 > t0 and dst != src and 0 <= dst <= nslots
            buf[dst] = t1
            steps += t1 - t0
        else:
            assert kind == 1 and t0 == expect
            expect -= 1
    assert expect == -1
    return steps


@lru_cache(None)
def best(l, s):
    """Least forward steps to reverse l steps from a held state with s free
    slots and a work buffer (exhaustive over the first split)."""
    if l == 1:
        return 0
    if s == 0:
        return l * (l - 1) // 2
    return min(m + best(l - m, s - 1) + best(m, s) for m in range(1, l))


def closed_form(T, s):
    if s == 0:
        return T * (T - 1) // 2
    c = s + 1
    r = 0
    while comb(c + r, c) < T:
        r += 1
    return r * T - (comb(c + r, c + 1) if r >= 1 else 0)


@pytest.mark.parametrize("s", [0, 1, 2, 3, 5])
def test_schedule_valid_and_optimal_small(L, s):
    for T in range(1, 70):
        ops, fwd = L.revolve_schedule(T, s)
        assert simulate(ops, T, s) == fwd
        assert fwd == best(T, s), (T, s)
        assert sum(1 for o in ops if o[0] == 1) == T


@pytest.mark.parametrize("T,s", [(1000, 4), (1000, 10), (5000, 3), (20000, 12), (777, 1)])
def test_schedule_valid_and_optimal_large(L, T, s):
    ops, fwd = L.revolve_schedule(T, s)
    assert simulate(ops, T, s) == fwd
    assert fwd == closed_form(T, s)


def test_closed_form_matches_exhaustive_search():
    for s in range(1, 6):
        for T in range(2, 120):
            assert closed_form(T, s) == best(T, s)


def test_first_ops_are_a_forward_chain(L):
    # the ops before the first adjoint step advance one state from u_0 to
    # u_{T-1}: the forward sweep stores exactly those snapshots
    for T, s in ((10, 2), (100, 3), (1, 4), (2, 0), (57, 1)):
        ops, _ = L.revolve_schedule(T, s)
        t = 0
        src = -1
        for kind, a, dst, t0, t1 in ops:
            if kind == 1:
                break
            assert a == src and t0 == t
            src, t = dst, t1
        assert t == T - 1


def test_schedule_arguments(L):
    import ctypes
    n = ctypes.c_int64(0)
    assert L.lib().dcp_revolve_schedule(-1, 2, None, 0, ctypes.byref(n), None) == -5
    assert L.lib().dcp_revolve_schedule(5, -1, None, 0, ctypes.byref(n), None) == -5
    assert L.lib().dcp_revolve_schedule(5, 1, None, 0, None, None) == -1
    buf = (ctypes.c_int64 * 5)()
    assert L.lib().dcp_revolve_schedule(5, 1, buf, 1, ctypes.byref(n), None) == -6
    assert L.lib().dcp_revolve_schedule(0, 3, None, 0, ctypes.byref(n), None) == 0 and n.value == 0
