"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the AM method: it only draws data
matrices, starting points and problem parameters.  Both the FP64 oracle and
the GPU path receive their inputs from here, so the two never depend on each
other.

Data model (the paper's experiments use real data sets that are not
available here; the stand-in is a spiked covariance model):
    A = G + sum_k theta_k u_k v_k^T
with G i.i.d. N(0, 1), u_k = g / ||g|| for g ~ N(0, I_n) and v_k a unit
vector with ``spike_nnz`` N(0, 1) nonzeros on a uniformly drawn support; the
supports of different v_k are disjoint.  Matrices are returned in FP32,
column-major (Fortran order): column a_i is contiguous, as the method reads
it column by column.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 0x5EED0000


@dataclasses.dataclass(frozen=True)
class Spiked:
    A: np.ndarray            # n x p float32, Fortran order
    supports: tuple          # planted supports, one sorted int array per spike
    thetas: tuple


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_matrix(seed: int, n: int, p: int) -> np.ndarray:
    """n x p, entries i.i.d. N(0, 1), FP32 column-major."""
    g = rng(seed).standard_normal((p, n), dtype=np.float32)
    return np.asfortranarray(g.T)


def spiked_matrix(seed: int, n: int, p: int, thetas=(60.0, 40.0, 25.0),
                  spike_nnz: int = 50) -> Spiked:
    """Spiked model A = G + sum_k theta_k u_k v_k^T (see module docstring)."""
    r = rng(seed)
    k = len(thetas)
    assert k * spike_nnz <= p
    G = r.standard_normal((p, n), dtype=np.float32)  # G^T, rows = columns of A
    perm = r.permutation(p)
    supports = []
    At = G.astype(np.float64)
    for t, theta in enumerate(thetas):
        sup = np.sort(perm[t * spike_nnz:(t + 1) * spike_nnz])
        supports.append(sup)
        u = r.standard_normal(n)
        u /= np.linalg.norm(u)
        vals = r.standard_normal(spike_nnz)
        vals /= np.linalg.norm(vals)
        At[sup, :] += theta * np.outer(vals, u)
    A = np.asfortranarray(At.T.astype(np.float32))
    return Spiked(A=A, supports=tuple(supports), thetas=tuple(thetas))


def random_unit_starts(seed: int, r: int, p: int) -> np.ndarray:
    """r x p FP32, each row an N(0, I_p) draw scaled to unit length."""
    X = rng(seed).standard_normal((r, p))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return np.ascontiguousarray(X.astype(np.float32))


def column_norm_max(A: np.ndarray, ord_: int = 2) -> float:
    """max_i ||a_i|| (FP64), used to set the penalty parameter gamma."""
    return float(np.max(np.linalg.norm(np.asarray(A, dtype=np.float64), ord=ord_,
                                       axis=0)))


def gamma_literal(A: np.ndarray) -> float:
    """gamma = 0.1 * max_i ||a_i||_2 for every penalised formulation."""
    return 0.1 * column_norm_max(A, 2)


def gamma_scaled(A: np.ndarray, fid: int) -> float:
    """A scale-consistent gamma: 0.1 of the zero-solution threshold's root.

    gamma is compared with v_i^2 (L0 penalty) or |v_i| (L1 penalty), and
    |v_i| is at most ||a_i||_2 (L2 variance) or ||a_i||_1 (L1 variance).
    """
    base = 0.1 * column_norm_max(A, 2 if fid % 2 == 1 else 1)
    return base * base if fid in (5, 6) else base


def s_or_gamma_for(fid: int, A: np.ndarray, s: float, gamma_mode: str = "literal"):
    """The parameter of formulation ``fid``: s for constraints, gamma else."""
    if fid <= 4:
        return float(s)
    if gamma_mode == "literal":
        return gamma_literal(A)
    return gamma_scaled(A, fid)


# Workloads, named by what they are.
SMALL_SINGLE_START = dict(  # one start, Gaussian data, L2 variance / L0 constraint
    name="gauss-100x500-F1-s10-r1", n=100, p=500, fid=1, s=10, r=1, tol=1e-8,
    maxit=500, seed=SEED_BASE + 0)
SPIKED_ALL8 = dict(  # all 8 formulations, 1024 random starts in one launch
    name="spiked-1000x10000-all8-r1024", n=1000, p=10000, thetas=(60.0, 40.0, 25.0),
    spike_nnz=50, s=50, r=1024, maxit=200, seed=SEED_BASE + 1)
SPIKED_BF16 = dict(
    name="spiked-5000x50000-F1F8-bf16-r256", n=5000, p=50000,
    thetas=(60.0, 40.0, 25.0), spike_nnz=50, s=100, r=256, maxit=200,
    fids=(8, 1), seed=SEED_BASE + 2)
SPIKED_LARGE = dict(
    name="spiked-20000x200000-F1-r64", n=20000, p=200000,
    thetas=(269.0, 223.0, 178.0, 141.0, 112.0), spike_nnz=200, s=200, r=64,
    maxit=200, fid=1, seed=SEED_BASE + 3)
