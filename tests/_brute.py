"""Brute-force helpers for pinning the oracle: an explicit dense Laplacian and
exact rational evaluation.  Test-only; they share nothing with the oracle's
C code and nothing with the GPU library.

Layout matches the library and the oracle: linear index p = x + nx*(y + ny*z),
fields shaped (nz, ny, nx).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

DIRS = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def _nbr(c, n, bc):
    if 0 <= c < n:
        return c
    if bc == 1:
        return c % n
    return None


def neighbours(x, y, z, nx, ny, nz, bc):
    """Face neighbours (with multiplicity) of (x, y, z); ghost cells omitted."""
    out = []
    for dx, dy, dz in DIRS:
        qx, qy, qz = _nbr(x + dx, nx, bc), _nbr(y + dy, ny, bc), _nbr(z + dz, nz, bc)
        if qx is None or qy is None or qz is None:
            continue
        out.append((qx, qy, qz))
    return out


def dense_laplacian(nx, ny, nz, bc, h=1.0):
    """L with (L u)[p] = (sum of the face neighbours of p - 6 u[p]) / h^2."""
    n = nx * ny * nz
    L = np.zeros((n, n))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                p = x + nx * (y + ny * z)
                L[p, p] -= 6.0 / h ** 2
                for qx, qy, qz in neighbours(x, y, z, nx, ny, nz, bc):
                    L[p, qx + nx * (qy + ny * qz)] += 1.0 / h ** 2
    return L


def laplacian_spectrum(nx, ny, nz, bc, h=1.0):
    """Closed-form eigenvalues of L: periodic Fourier modes, or the sine modes
    of the ghost-zero (Dirichlet) problem."""
    vals = []
    if bc == 1:
        ks = [range(n) for n in (nx, ny, nz)]
        lam1 = [lambda k, n=n: 2 * np.cos(2 * np.pi * k / n) - 2 for n in (nx, ny, nz)]
    else:
        ks = [range(1, n + 1) for n in (nx, ny, nz)]
        lam1 = [lambda k, n=n: 2 * np.cos(np.pi * k / (n + 1)) - 2 for n in (nx, ny, nz)]
    for kx in ks[0]:
        for ky in ks[1]:
            for kz in ks[2]:
                vals.append((lam1[0](kx) + lam1[1](ky) + lam1[2](kz)) / h ** 2)
    return np.sort(np.array(vals))


def step_dense(u, f, L, c):
    """One step by the matrix form u + dt*(alpha*L u - beta*u^3 + gamma*f)."""
    uf = u.ravel()
    out = uf + c["dt"] * (c["alpha"] * (L @ uf) - c["beta"] * uf ** 3 + c["gamma"] * f.ravel())
    return out.reshape(u.shape)


def jacobian_dense(u, L, c):
    """J = I + dt*alpha*L - diag(3*beta*dt*u^2)."""
    uf = u.ravel()
    return np.eye(uf.size) + c["dt"] * c["alpha"] * L - np.diag(3 * c["beta"] * c["dt"] * uf ** 2)


def step_exact(u, f, c, bc):
    """One step in exact rational arithmetic (inputs converted exactly from
    binary64); returns a float64 array of the exactly rounded result and the
    object array of Fractions."""
    nz, ny, nx = u.shape
    F = np.vectorize(Fraction, otypes=[object])
    uq, fq = F(u), F(f)
    a, b, g, h, dt = (Fraction(float(c[k])) for k in ("alpha", "beta", "gamma", "h", "dt"))
    out = np.empty(u.shape, dtype=object)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                s = sum((uq[qz, qy, qx] for qx, qy, qz in neighbours(x, y, z, nx, ny, nz, bc)),
                        Fraction(0))
                lap = (s - 6 * uq[z, y, x]) / (h * h)
                out[z, y, x] = uq[z, y, x] + dt * (a * lap - b * uq[z, y, x] ** 3 + g * fq[z, y, x])
    return np.vectorize(float, otypes=[np.float64])(out), out
