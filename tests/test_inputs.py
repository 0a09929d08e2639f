"""Seeded input generators: determinism, stream separation and the sinusoid
field's definition."""
import numpy as np

from paper_2107_00555_amd import inputs


def test_uniform_is_deterministic_and_streams_differ():
    a = inputs.uniform(7, 5, 3, seed=0, stream=inputs.STREAM_U0)
    b = inputs.uniform(7, 5, 3, seed=0, stream=inputs.STREAM_U0)
    c = inputs.uniform(7, 5, 3, seed=0, stream=inputs.STREAM_F)
    d = inputs.uniform(7, 5, 3, seed=1, stream=inputs.STREAM_U0)
    assert a.shape == (3, 5, 7) and a.dtype == np.float64
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)
    assert a.min() >= -1 and a.max() <= 1


def test_sinusoids_match_direct_definition_and_are_periodic():
    nx, ny, nz = 16, 12, 10
    f = inputs.sinusoids(nx, ny, nz, seed=3)
    modes = inputs.sinusoid_params(seed=3)
    assert len(modes) == 8
    for mx, my, mz, a, phi in modes:
        assert (mx, my, mz) != (0, 0, 0)
        assert max(abs(mx), abs(my), abs(mz)) <= 4 and -1 <= a <= 1 and 0 <= phi < 2 * np.pi
    r = np.random.default_rng(0)
    for _ in range(20):
        x, y, z = r.integers(0, nx), r.integers(0, ny), r.integers(0, nz)
        want = sum(a * np.sin(2 * np.pi * (mx * x / nx + my * y / ny + mz * z / nz) + phi)
                   for mx, my, mz, a, phi in modes)
        assert abs(f[z, y, x] - want) < 1e-13
        # periodic extension: evaluating the definition one period away agrees
        want2 = sum(a * np.sin(2 * np.pi * (mx * (x + nx) / nx + my * y / ny + mz * (z - nz) / nz) + phi)
                    for mx, my, mz, a, phi in modes)
        assert abs(want2 - want) < 1e-12


def test_fd_directions_deterministic():
    d1 = list(inputs.fd_directions(4, 3, 2, seed=0, count=3))
    d2 = list(inputs.fd_directions(4, 3, 2, seed=0, count=3))
    for (a, b, c), (x, y, z) in zip(d1, d2):
        assert np.array_equal(a, x) and b == y and c == z
    assert not np.array_equal(d1[0][0], d1[1][0])


def test_sinusoid_box_and_zslab_are_crops_of_the_full_fields():
    nx, ny, nz = 12, 10, 8
    full = inputs.sinusoids(nx, ny, nz, seed=4)
    box = inputs.sinusoids(nx, ny, nz, seed=4, box=((2, 9), (0, 4), (3, 8)))
    assert np.max(np.abs(box - full[3:8, 0:4, 2:9])) < 1e-13
    u = inputs.uniform(nx, ny, nz, seed=4, stream=inputs.STREAM_U0)
    assert np.array_equal(inputs.uniform_zslab(nx, ny, 3, seed=4, stream=inputs.STREAM_U0), u[:3])
