"""Seeded random single-operator programs for the fusing compiler tests:
element-wise arithmetic, scalar parameters and literals, shifted reads in
all three axes (offsets up to 2 in x, 1 in y and z), chained shifts, and
one to three outputs."""
import numpy as np


def _fuse():
    from paper_2107_00555_amd import fuse
    return fuse


def random_program(seed, dtype):
    F = _fuse()
    rng = np.random.default_rng(seed)
    P = F.Program(dtype)
    ins = list(P.input("a", "b", "c"))
    ps = list(P.param("p", "q"))
    vals = list(ins)
    for _ in range(int(rng.integers(8, 30))):
        k = rng.integers(0, 10)
        x = vals[int(rng.integers(0, len(vals)))]
        y = vals[int(rng.integers(0, len(vals)))]
        s = ps[int(rng.integers(0, 2))] if rng.random() < 0.5 else float(rng.uniform(-2, 2))
        if k == 0:
            e = x + y
        elif k == 1:
            e = x - s
        elif k == 2:
            e = x * y
        elif k == 3:
            e = s * x
        elif k == 4:
            e = x / (y * y + 1.0)          # never divides by zero
        elif k == 5:
            e = -x
        elif k in (6, 7):
            e = x.shift(int(rng.integers(-2, 3)), int(rng.integers(-1, 2)), int(rng.integers(-1, 2)))
        else:
            e = (x + y) * 0.5
        vals.append(e)
    n_out = int(rng.integers(1, 4))
    for j in range(n_out):
        P.output(f"o{j}", vals[-1 - 3 * j] if len(vals) > 3 * j + 3 else vals[-1 - j])
    return P
