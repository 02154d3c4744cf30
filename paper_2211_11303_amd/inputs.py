"""Seeded synthetic inputs shared by the library's tests, the benchmark and
the oracle checks.  This module draws random numbers only; it holds none of
the method's arithmetic (no assembly, no products, no solves).

* ``exact_solution`` -- x* with entries uniform in [-1, 1] (numpy PCG64,
  ``default_rng(seed)``), one column per right-hand side, in the natural
  (mesh) order of the unknowns.
* ``probe_block``    -- standard normal probe vectors for the factor error.
* ``batch_problems`` -- a list of (n, kappa) problems for the batched runs.
* ``serving_requests`` -- Poisson arrivals of solve requests.
"""

import numpy as np


def num_interior_edges(n):
    """Number of unknowns of the Kuhn cube mesh with n^3 cubes."""
    return 7 * n ** 3 - 9 * n ** 2 + 3 * n


def exact_solution(N, nrhs=1, seed=0):
    """x* of shape (N, nrhs), float64, column-major friendly (C-contiguous
    columns are produced by transposing a (nrhs, N) draw)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(nrhs, N)).T)


def exact_solution_cols(N, nrhs=1, seed=0):
    """The same draw as ``exact_solution`` laid out as nrhs contiguous
    columns: shape (nrhs, N)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(nrhs, N))


def probe_block(N, nprobe=8, seed=12345):
    """Standard normal (nprobe, N) block, one probe vector per row."""
    return np.random.default_rng(seed).standard_normal((N, nprobe)).T.copy()


def batch_problems(count=64, seed=7, sizes=(8, 12, 16, 20, 24), kappa_range=(1.0, 10.0)):
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    ks = rng.uniform(kappa_range[0], kappa_range[1], size=count)
    return [(int(n), float(k)) for n, k in zip(ns, ks)]


def serving_requests(count, rate, seed=11, sizes=(8, 12, 16, 20, 24, 32, 40),
                     kappas=tuple(range(1, 17)), max_rhs=32):
    """Poisson arrivals: list of dicts(t, n, kappa, nrhs, seed)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ns = rng.choice(np.asarray(sizes), size=count)
    ks = rng.choice(np.asarray(kappas), size=count)
    rh = rng.integers(1, max_rhs + 1, size=count)
    return [dict(t=float(t[i]), n=int(ns[i]), kappa=float(ks[i]), nrhs=int(rh[i]), seed=1000 + i)
            for i in range(count)]
