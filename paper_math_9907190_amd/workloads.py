"""Seeded synthetic right-hand sides for the Poisson problems this package
solves.  Shared by the tests (which feed the same arrays to the CPU oracle
and to the GPU library) and by the benchmark.  This module holds no part of
the multigrid method: only random numbers and sine modes.

All arrays are float64, shape (n+1,)*dim, indexed [.., y, x] (x fastest),
zero on the boundary.  Generators draw from numpy's PCG64 in lexicographic
interior order.
"""
import numpy as np


def _grid(n):
    return np.arange(n + 1, dtype=np.float64) / n


def _zero_boundary(f):
    for ax in range(f.ndim):
        idx = [slice(None)] * f.ndim
        idx[ax] = 0
        f[tuple(idx)] = 0
        idx[ax] = -1
        f[tuple(idx)] = 0
    return f


def uniform(dim, n, seed):
    """i.i.d. U(-1, 1) at interior nodes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros((n + 1,) * dim)
    f[(slice(1, -1),) * dim] = rng.uniform(-1.0, 1.0, (n - 1,) * dim)
    return f


def sine_mode(dim, n, ks, amp=1.0):
    """amp * prod_i sin(k_i pi x_i) on the grid (ks ordered x, y[, z])."""
    x = _grid(n)
    out = np.sin(ks[0] * np.pi * x)
    for k in ks[1:]:
        out = np.multiply.outer(np.sin(k * np.pi * x), out)
    return amp * out


def square_uniform_plus_mode(n=64, seed=1):
    """2D: U(-1,1) noise plus f = Lap(sin(pi x) sin(pi y)) = -2 pi^2 sin sin."""
    f = uniform(2, n, seed) + sine_mode(2, n, (1, 1), -2.0 * np.pi ** 2)
    return _zero_boundary(f)


def square_modes_noise(n=4096, seed=2, modes=16, kmax=64, noise=1e-3):
    """2D: sum of `modes` sine modes with N(0,1) amplitudes and wavenumbers
    U{1..kmax} per axis, plus `noise` times i.i.d. N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    amps = rng.standard_normal(modes)
    ks = rng.integers(1, kmax + 1, size=(modes, 2))
    x = _grid(n)
    f = np.zeros((n + 1, n + 1))
    for a, (k, l) in zip(amps, ks):
        f += a * np.outer(np.sin(l * np.pi * x), np.sin(k * np.pi * x))
    f[1:-1, 1:-1] += noise * rng.standard_normal((n - 1, n - 1))
    return _zero_boundary(f)


def cube_uniform(n=256, seed=3):
    """3D: i.i.d. U(-1,1) at interior nodes."""
    return uniform(3, n, seed)


BATCH_SIDES = (128, 256, 512, 1024)


def batch_sizes(count=512, seed=4, sides=BATCH_SIDES):
    """Interval counts n of `count` independent 2D problems, drawn uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(sides[i]) for i in rng.integers(0, len(sides), size=count)]


def batch_problem(n, b, base_seed=4, modes=4, kmax=8):
    """2D smooth-mode f of batch member b: sum of `modes` modes, N(0,1)
    amplitudes, wavenumbers U{1..kmax}; seed base_seed + b."""
    rng = np.random.Generator(np.random.PCG64(base_seed + b))
    amps = rng.standard_normal(modes)
    ks = rng.integers(1, kmax + 1, size=(modes, 2))
    x = _grid(n)
    f = np.zeros((n + 1, n + 1))
    for a, (k, l) in zip(amps, ks):
        f += a * np.outer(np.sin(l * np.pi * x), np.sin(k * np.pi * x))
    return _zero_boundary(f)


def training_rhs(dim, n, seed, smooth_modes=8, kmax=None):
    """Right-hand sides for the learned coarse correction: even seeds give a
    sum of smooth modes, odd seeds i.i.d. U(-1,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if seed % 2:
        f = np.zeros((n + 1,) * dim)
        f[(slice(1, -1),) * dim] = rng.uniform(-1.0, 1.0, (n - 1,) * dim)
        return f
    kmax = kmax or max(2, n // 8)
    f = np.zeros((n + 1,) * dim)
    for _ in range(smooth_modes):
        ks = rng.integers(1, kmax + 1, size=dim)
        f += rng.standard_normal() * sine_mode(dim, n, tuple(int(k) for k in ks))
    return _zero_boundary(f)
