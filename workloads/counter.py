"""Counter-based synthetic data: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11) and the spiked model
built on it.

Any entry A[i, j] is a pure function of (seed, i, j), so the GPU library can
generate a matrix of any size in device memory and the host can regenerate
single columns of it bit for bit (this module is the host implementation;
the library has its own, written from the same published definition).  It
holds no arithmetic of the AM method.

Entry model: one Philox4x32-10 block per entry with counter (i, j, 0, 0)
and key (seed low 32 bits, seed high 32 bits); the four 32-bit outputs give
four uniform 24-bit integers w_0..w_3 (top 24 bits of each) and

    g = (sum(w) * 2^-24 - 2) * sqrt(3)          (FP64, rounded once to FP32)

a sum of four uniforms scaled to mean 0 and variance 1 (Irwin-Hall), used in
place of an exact Gaussian because it is computed exactly the same way on the
host and on the GPU (integer sums, a power-of-two scale, one rounded FP64
product).  The spiked matrix adds sum_k theta_k u_k[i] v_k[j] in FP64, left to
right in k, each term as (theta_k * u_k[i]) * v_k[j], then rounds once to
FP32.
"""
from __future__ import annotations

import dataclasses

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
SQRT3 = 1.7320508075688772  # the same literal is used by the GPU generator
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: (..., 4) uint32; key: (2,) or (..., 2)
    uint32.  Returns (..., 4) uint32."""
    c = [np.asarray(ctr[..., q], dtype=np.uint64) for q in range(4)]
    key = np.asarray(key, dtype=np.uint32)
    k0 = np.broadcast_to(key[..., 0], c[0].shape).astype(np.uint32)
    k1 = np.broadcast_to(key[..., 1], c[0].shape).astype(np.uint32)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0).astype(np.uint32)
            k1 = (k1 + W1).astype(np.uint32)
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0.astype(np.uint64), lo1,
             hi0 ^ c[3] ^ k1.astype(np.uint64), lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def _key(seed):
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([s & 0xFFFFFFFF, s >> 32], dtype=np.uint32)


def gaussian_entries(seed, rows, cols):
    """g[i, j] for the index arrays rows (length a) and cols (length b): an
    (a, b) float32 array."""
    return _gaussian64(seed, rows, cols).astype(np.float32)


def _gaussian64(seed, rows, cols):
    """The FP64 value of g[i, j] before its rounding to FP32."""
    rows = np.asarray(rows, dtype=np.uint32)
    cols = np.asarray(cols, dtype=np.uint32)
    R, C = np.meshgrid(rows, cols, indexing="ij")
    ctr = np.stack([R, C, np.zeros_like(R), np.zeros_like(R)], axis=-1)
    out = philox4x32_10(ctr, _key(seed))
    w = (out >> np.uint32(8)).astype(np.float64)
    ssum = w[..., 0] + w[..., 1] + w[..., 2] + w[..., 3]
    return (ssum * 2.0 ** -24 - 2.0) * SQRT3


@dataclasses.dataclass(frozen=True)
class SpikeFactors:
    thetas: np.ndarray   # (k,) float64
    U: np.ndarray        # (n, k) float64, unit columns
    V: np.ndarray        # (p, k) float64, unit columns, disjoint supports
    supports: tuple


def spike_factors(seed, n, p, thetas, spike_nnz):
    """Spike directions drawn on the host (PCG64): u_k = g / ||g||, v_k unit
    with spike_nnz N(0, 1) entries on disjoint uniform supports."""
    r = np.random.Generator(np.random.PCG64(int(seed) ^ 0x5A5A5A5A))
    k = len(thetas)
    U = np.zeros((n, k))
    V = np.zeros((p, k))
    perm = r.permutation(p)
    sups = []
    for t in range(k):
        u = r.standard_normal(n)
        U[:, t] = u / np.linalg.norm(u)
        sup = np.sort(perm[t * spike_nnz:(t + 1) * spike_nnz])
        vals = r.standard_normal(spike_nnz)
        V[sup, t] = vals / np.linalg.norm(vals)
        sups.append(sup)
    return SpikeFactors(np.asarray(thetas, dtype=np.float64), U, V, tuple(sups))


def spiked_columns(seed, n, cols, factors: SpikeFactors):
    """Columns `cols` of the spiked matrix, (n, len(cols)) float32."""
    cols = np.asarray(cols)
    acc = _gaussian64(seed, np.arange(n), cols)
    for t in range(len(factors.thetas)):
        acc = acc + (factors.thetas[t] * factors.U[:, t])[:, None] * factors.V[cols, t][None, :]
    return acc.astype(np.float32)


def spiked_matrix(seed, n, p, factors: SpikeFactors):
    """The whole n x p spiked matrix (column-major float32); small sizes."""
    return np.asfortranarray(spiked_columns(seed, n, np.arange(p), factors))
