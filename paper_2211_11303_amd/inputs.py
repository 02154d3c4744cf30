"""Seeded synthetic inputs shared by the library's tests, the benchmark and
the oracle checks.  This module draws random numbers and lays out input
geometries only; it holds none of the method's arithmetic (no assembly, no
products, no solves).

* ``exact_solution`` -- x* with entries uniform in [-1, 1] (numpy PCG64,
  ``default_rng(seed)``), one column per right-hand side, in the natural
  (mesh) order of the unknowns.
* ``probe_block``    -- standard normal probe vectors for the factor error.
* ``batch_problems`` -- a list of (n, kappa) problems for the batched runs.
* ``serving_requests`` -- Poisson arrivals of solve requests.
* ``two_box_mask``   -- the cubes of the two-box domain (Example 2) on the
  lattice.
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


def two_box_mask(m):
    """The two-box domain of Example 2 on the Kuhn lattice, m cubes per unit
    length: (n, mask) with n = 4m and mask[i + n (j + n k)] set for the cubes
    of the union of
      [-2, 2] x [-1, 2] x [-1, 1]   (cubes i in [0, 4m), j in [0, 3m), k in [m, 3m))
      [-1, 1] x [-1, 1] x [-2, 2]   (cubes i in [m, 3m), j in [0, 2m), k in [0, 4m))
    after the shift (x, y, z) -> (x + 2, y + 1, z + 2) and the scaling by
    1/4 into the unit cube of the lattice.  This is a reading of the
    domain's printed union of five boxes, whose first box has an empty
    interval; their union is these two boxes crossing."""
    n = 4 * m
    mask = np.zeros(n ** 3, dtype=np.uint8)
    for k in range(n):
        for j in range(n):
            for i in range(n):
                a = i < 4 * m and j < 3 * m and m <= k < 3 * m
                b = m <= i < 3 * m and j < 2 * m
                if a or b:
                    mask[i + n * (j + n * k)] = 1
    return n, mask
