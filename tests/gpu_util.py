"""Helpers shared by the GPU tests (oracle side and library side kept apart)."""
import functools

import numpy as np

from oracle.assemble import Discretisation
from oracle.cluster import Structure
from oracle.hmatrix import HLU as OracleHLU
from oracle.krylov import gmres as oracle_gmres


@functools.lru_cache(maxsize=16)
def oracle_problem(n, kappa, leaf):
    d = Discretisation(n, kappa)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0)
    return d, s


@functools.lru_cache(maxsize=16)
def oracle_factor(n, kappa, leaf, eps, max_rank=0):
    d, s = oracle_problem(n, kappa, leaf)
    return OracleHLU(s, d.A, eps, max_rank).factor()


def oracle_solve(n, kappa, leaf, eps, b, restart, tol):
    d, s = oracle_problem(n, kappa, leaf)
    h = oracle_factor(n, kappa, leaf, eps)
    return oracle_gmres(d.A, b, h.solve, restart=restart, tol=tol, max_iters=2000)


def gpu_factor_error(H, A_csr, perm, nprobe=8, seed=12345):
    """Same probe as the oracle's factor_error, through hlu_apply_lu."""
    import torch
    N = A_csr.shape[0]
    Om = np.random.default_rng(seed).standard_normal((N, nprobe))   # cluster order
    v = np.empty_like(Om)
    v[perm] = Om                                                      # natural order
    vt = torch.tensor(v.T.copy(), dtype=torch.float64, device="cuda")
    y = H.hlu_apply_lu(vt).cpu().numpy().T
    ref = A_csr @ v
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def fp32_factor_bound(e_or, e_st, leaf):
    """Parity bound for the factor error of an FP32 H-LU (factors stored in
    FP32, dense task arithmetic in FP32 or FP64), derived from the FP32 unit
    roundoff through the oracle itself:

      e_round = sqrt(e_st^2 - e_or^2) is the error that rounding the oracle's
        own factors to FP32 adds (e_st: the oracle's factor error with its
        factors rounded to FP32; truncation and rounding errors are
        uncorrelated, so their squares add);
      FP32 arithmetic inside a task rounds inner products of length at most
        `leaf` (dense leaves; ranks stay below the 64-column block capacity),
        whose error grows like sqrt(leaf) u32 |terms| in the probabilistic
        rounding model, i.e. sqrt(leaf) times the storage rounding of the
        same entries;

    so e_fp32 <= 2 e_or + (1 + sqrt(leaf)) e_round, the FP64 bar (2x the
    oracle's truncation error) plus the rounding terms."""
    import math
    e_round = math.sqrt(max(e_st * e_st - e_or * e_or, 0.0))
    return 2.0 * e_or + (1.0 + math.sqrt(leaf)) * e_round
