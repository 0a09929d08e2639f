"""Pins of the Jacobi oracle (jacobi_1d, Sec. 2.2; jacobi_2d, Sec. 4.3)
against facts fixed by the listings and by linear algebra, not by the
oracle's own code: closed-form eigenmodes, dense brute force, the loop count
and the untouched boundary."""
import numpy as np
import pytest

import oracle
from paper_2107_00555_amd import inputs

W1 = 0.33333  # the listing's weight for jacobi_1d (not 1/3)
W2 = 0.2


def test_no_iteration_when_tsteps_at_most_one():
    # the loop is range(1, TSTEPS): empty for TSTEPS <= 1
    A, B = inputs.jacobi_fields(1, 37, seed=3)
    for t in (-5, 0, 1):
        a, b = oracle.jacobi_1d(t, A, B)
        assert np.array_equal(a, A) and np.array_equal(b, B)
    A, B = inputs.jacobi_fields(2, 9, seed=3, n1=11)
    for t in (-5, 0, 1):
        a, b = oracle.jacobi_2d(t, A, B)
        assert np.array_equal(a, A) and np.array_equal(b, B)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_1d_without_interior_is_unchanged(n):
    A, B = inputs.jacobi_fields(1, n, seed=1)
    a, b = oracle.jacobi_1d(7, A, B)
    assert np.array_equal(a, A) and np.array_equal(b, B)


@pytest.mark.parametrize("shape", [(0, 0), (1, 6), (2, 9), (9, 2), (5, 1)])
def test_2d_without_interior_is_unchanged(shape):
    A, B = inputs.jacobi_fields(2, shape[0], seed=1, n1=shape[1])
    a, b = oracle.jacobi_2d(7, A, B)
    assert np.array_equal(a, A) and np.array_equal(b, B)


def test_boundary_never_written():
    A, B = inputs.jacobi_fields(2, 12, seed=5, n1=15)
    a, b = oracle.jacobi_2d(9, A, B)
    for x, x0 in ((a, A), (b, B)):
        assert np.array_equal(x[0], x0[0]) and np.array_equal(x[-1], x0[-1])
        assert np.array_equal(x[:, 0], x0[:, 0]) and np.array_equal(x[:, -1], x0[:, -1])
    A, B = inputs.jacobi_fields(1, 20, seed=5)
    a, b = oracle.jacobi_1d(9, A, B)
    assert a[0] == A[0] and a[-1] == A[-1] and b[0] == B[0] and b[-1] == B[-1]


@pytest.mark.parametrize("n,k,tsteps", [(41, 3, 6), (64, 1, 20), (17, 5, 4)])
def test_1d_sine_mode_closed_form(n, k, tsteps):
    """With zero ends, sin(pi k i/(n-1)) is an eigenvector of the three-point
    average with eigenvalue mu = w (1 + 2 cos(pi k/(n-1))).  B is set from A
    first, so after TSTEPS-1 passes A = mu^(2m) A0 and B = mu^(2m-1) A0, with
    m = TSTEPS-1, whatever B's interior held at the start."""
    i = np.arange(n)
    mode = np.sin(np.pi * k * i / (n - 1))
    mode[0] = mode[-1] = 0.0
    junk = inputs.jacobi_fields(1, n, seed=9)[1]
    junk[0] = junk[-1] = 0.0
    mu = W1 * (1.0 + 2.0 * np.cos(np.pi * k / (n - 1)))
    m = tsteps - 1
    a, b = oracle.jacobi_1d(tsteps, mode, junk)
    tol = 8 * 2 * m * np.finfo(float).eps
    assert np.max(np.abs(a - mu ** (2 * m) * mode)) <= tol
    assert np.max(np.abs(b - mu ** (2 * m - 1) * mode)) <= tol
    # the weight is the listing's 0.33333: with 1/3 the decay would differ
    mu3 = (1.0 + 2.0 * np.cos(np.pi * k / (n - 1))) / 3.0
    assert np.max(np.abs(a - mu3 ** (2 * m) * mode)) > 100 * tol


@pytest.mark.parametrize("n0,n1,k,l,tsteps", [(13, 17, 2, 5, 5), (20, 9, 1, 3, 8), (16, 16, 3, 1, 3)])
def test_2d_sine_mode_closed_form(n0, n1, k, l, tsteps):
    """sin(pi k i/(n0-1)) sin(pi l j/(n1-1)) with zero edges has eigenvalue
    w (1 + 2 cos(pi k/(n0-1)) + 2 cos(pi l/(n1-1))) under the five-point
    average; on a non-square grid with k != l a swapped axis fails."""
    i = np.arange(n0)[:, None]
    j = np.arange(n1)[None, :]
    mode = np.sin(np.pi * k * i / (n0 - 1)) * np.sin(np.pi * l * j / (n1 - 1))
    mode[0, :] = mode[-1, :] = 0.0
    mode[:, 0] = mode[:, -1] = 0.0
    junk = inputs.jacobi_fields(2, n0, seed=4, n1=n1)[1]
    junk[0, :] = junk[-1, :] = 0.0
    junk[:, 0] = junk[:, -1] = 0.0
    mu = W2 * (1.0 + 2.0 * np.cos(np.pi * k / (n0 - 1)) + 2.0 * np.cos(np.pi * l / (n1 - 1)))
    m = tsteps - 1
    a, b = oracle.jacobi_2d(tsteps, mode, junk)
    tol = 16 * 2 * m * np.finfo(float).eps
    assert np.max(np.abs(a - mu ** (2 * m) * mode)) <= tol
    assert np.max(np.abs(b - mu ** (2 * m - 1) * mode)) <= tol


def test_1d_constant_decays_inside_light_cone():
    """A constant c is multiplied by 3w = 0.99999 per half-step wherever the
    fixed ends are not yet felt (distance to an end > number of half-steps)."""
    n, tsteps = 50, 5
    m = tsteps - 1
    a, b = oracle.jacobi_1d(tsteps, np.ones(n), np.ones(n))
    core = slice(2 * m + 1, n - 2 * m - 1)
    assert np.allclose(a[core], (3 * W1) ** (2 * m), rtol=0, atol=4e-16 * 2 * m)
    assert np.allclose(b[core], (3 * W1) ** (2 * m - 1), rtol=0, atol=4e-16 * 2 * m)


def _brute_1d(tsteps, A, B):
    n = A.size
    x = np.concatenate([A, B]).astype(np.float64)
    PB = np.eye(2 * n)  # B <- avg(A) on interior
    PA = np.eye(2 * n)  # A <- avg(B) on interior
    for i in range(1, n - 1):
        PB[n + i, :] = 0.0
        PA[i, :] = 0.0
        for d in (-1, 0, 1):
            PB[n + i, i + d] = W1
            PA[i, n + i + d] = W1
    for _ in range(1, tsteps):
        x = PA @ (PB @ x)
    return x[:n], x[n:]


def _brute_2d(tsteps, A, B):
    n0, n1 = A.shape
    N = n0 * n1
    x = np.concatenate([A.ravel(), B.ravel()]).astype(np.float64)
    PB = np.eye(2 * N)
    PA = np.eye(2 * N)
    for i in range(1, n0 - 1):
        for j in range(1, n1 - 1):
            p = i * n1 + j
            PB[N + p, :] = 0.0
            PA[p, :] = 0.0
            for q in (p, p - 1, p + 1, p + n1, p - n1):
                PB[N + p, q] = W2
                PA[p, N + q] = W2
    for _ in range(1, tsteps):
        x = PA @ (PB @ x)
    return x[:N].reshape(n0, n1), x[N:].reshape(n0, n1)


@pytest.mark.parametrize("n,tsteps", [(9, 4), (3, 6), (12, 2)])
def test_1d_brute_force(n, tsteps):
    """Dense matrices of the two half-steps on [A; B]; the ends of A and of B
    carry different values, so reading the wrong array's boundary fails."""
    A, B = inputs.jacobi_fields(1, n, seed=11)
    a, b = oracle.jacobi_1d(tsteps, A, B)
    ra, rb = _brute_1d(tsteps, A, B)
    assert np.max(np.abs(a - ra)) <= 1e-14
    assert np.max(np.abs(b - rb)) <= 1e-14


@pytest.mark.parametrize("n0,n1,tsteps", [(5, 6, 4), (7, 4, 3), (3, 3, 5), (6, 8, 2)])
def test_2d_brute_force(n0, n1, tsteps):
    A, B = inputs.jacobi_fields(2, n0, seed=12, n1=n1)
    a, b = oracle.jacobi_2d(tsteps, A, B)
    ra, rb = _brute_2d(tsteps, A, B)
    assert np.max(np.abs(a - ra)) <= 1e-14
    assert np.max(np.abs(b - rb)) <= 1e-14


@pytest.mark.parametrize("r0,c0,h0,h1", [(0, 0, 20, 24), (14, 30, 26, 18), (30, 5, 10, 40), (7, 9, 30, 30)])
def test_2d_window_matches_full_run_on_exact_region(r0, c0, h0, h1):
    """The window form, on the cells at distance > 2(TSTEPS-1) from every
    window edge that is not an array edge, equals the full run bit for bit."""
    n0, n1, tsteps = 40, 48, 4
    A, B = inputs.jacobi_fields(2, n0, seed=6, n1=n1)
    fa, fb = oracle.jacobi_2d(tsteps, A, B)
    wa, wb = oracle.jacobi_2d_box(tsteps, n0, n1, r0, c0, A[r0:r0 + h0, c0:c0 + h1],
                                  B[r0:r0 + h0, c0:c0 + h1])
    H = 2 * (tsteps - 1)
    lo0 = 0 if r0 == 0 else H
    hi0 = h0 if r0 + h0 == n0 else h0 - H
    lo1 = 0 if c0 == 0 else H
    hi1 = h1 if c0 + h1 == n1 else h1 - H
    assert hi0 > lo0 and hi1 > lo1
    sl = (slice(lo0, hi0), slice(lo1, hi1))
    gl = (slice(r0 + lo0, r0 + hi0), slice(c0 + lo1, c0 + hi1))
    assert np.array_equal(wa[sl], fa[gl]) and np.array_equal(wb[sl], fb[gl])


def test_1d_window_matches_full_run_on_exact_region():
    n, tsteps = 300, 6
    H = 2 * (tsteps - 1)
    A, B = inputs.jacobi_fields(1, n, seed=8)
    fa, fb = oracle.jacobi_1d(tsteps, A, B)
    for c0, h1 in ((0, 40), (120, 60), (250, 50)):
        wa, wb = oracle.jacobi_1d_box(tsteps, n, c0, A[c0:c0 + h1], B[c0:c0 + h1])
        lo = 0 if c0 == 0 else H
        hi = h1 if c0 + h1 == n else h1 - H
        assert np.array_equal(wa[lo:hi], fa[c0 + lo:c0 + hi])
        assert np.array_equal(wb[lo:hi], fb[c0 + lo:c0 + hi])
