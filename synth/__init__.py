"""Seeded synthetic inputs shared by the GPU path, the oracle, the tests and the bench.

This module holds no arithmetic of the method (no dimensions, ranks, orders or
matrix elements): only lattice topologies and seeded random numbers.

Seeding scheme (one fixed reading, since the paper states none):
  * numpy PCG64 through ``numpy.random.default_rng``;
  * the roles get fixed seeds: x -> 0, g -> 1, couplings -> 2, Lanczos start -> 3;
  * a vector is drawn in chunks of ``CHUNK`` rows, chunk ``c`` from
    ``default_rng([seed, c])``, so that any row range can be regenerated on its
    own and long vectors can be drawn by several threads;
  * FP32 inputs are the FP64 draws rounded to nearest;
  * a block of k columns is drawn as ``k*dim`` consecutive values in row-major
    ``[dim][k]`` order with the same chunking.
"""
from __future__ import annotations

import concurrent.futures as _fut
import os

import numpy as np

SEED_X = 0
SEED_G = 1
SEED_COUPLINGS = 2
SEED_V0 = 3

CHUNK = 1 << 24


def chain_bonds(L: int, distance: int = 1, periodic: bool = True):
    """Bonds (i, i+d) of a chain; with periodic boundaries (i, (i+d) mod L) for every i."""
    if periodic:
        if L <= 2 * distance:
            raise ValueError("periodic chain with L <= 2*d has repeated bonds")
        return [(i, (i + distance) % L) for i in range(L)]
    return [(i, i + distance) for i in range(L - distance)]


def j1j2_chain(L: int, j1: float, j2: float, delta: float):
    """Periodic J1-J2 XXZ chain: nearest-neighbour bonds (J1) then next-nearest (J2).

    Returns (bonds, jxy, jz) with jxy = J and jz = J*Delta per bond.
    """
    b1 = chain_bonds(L, 1)
    b2 = chain_bonds(L, 2)
    bonds = b1 + b2
    jxy = np.array([j1] * len(b1) + [j2] * len(b2), dtype=np.float64)
    jz = jxy * delta
    return bonds, jxy, jz


def xxz_chain(L: int, J: float = 1.0, delta: float = 1.0, periodic: bool = True):
    bonds = chain_bonds(L, 1, periodic)
    jxy = np.full(len(bonds), J, dtype=np.float64)
    return bonds, jxy, jxy * delta


def tilted_field_chain(L: int, jz: float = 1.0):
    """Open chain with Jxy = 1, Jz = jz on bonds (k, k+1), k < L-1, and the
    site-dependent field h_k = k on every site k (App. D's example model)."""
    bonds = chain_bonds(L, 1, periodic=False)
    jxy = np.ones(len(bonds), dtype=np.float64)
    return bonds, jxy, jxy * jz, np.arange(L, dtype=np.float64)


def random_couplings(num_bonds: int, seed: int = SEED_COUPLINGS,
                     j_range=(0.5, 1.5), delta_range=(0.0, 2.0)):
    """Per-bond J_b ~ U(j_range) and Delta_b ~ U(delta_range), drawn J first then Delta."""
    rng = np.random.default_rng(seed)
    J = rng.uniform(j_range[0], j_range[1], size=num_bonds)
    D = rng.uniform(delta_range[0], delta_range[1], size=num_bonds)
    return J, D


def gaussian(n_values: int, seed: int, dtype=np.float64, start: int = 0,
             threads: int | None = None) -> np.ndarray:
    """Values ``start .. start+n_values-1`` of the N(0,1) stream for ``seed``.

    Chunk c covers stream positions [c*CHUNK, (c+1)*CHUNK) and is drawn from
    ``default_rng([seed, c])`` in FP64; the result is then rounded to ``dtype``.
    """
    stop = start + n_values
    out = np.empty(n_values, dtype=np.float64)
    if n_values == 0:
        return out.astype(dtype)
    c0, c1 = start // CHUNK, (stop - 1) // CHUNK
    jobs = []
    for c in range(c0, c1 + 1):
        lo = max(start, c * CHUNK)
        hi = min(stop, (c + 1) * CHUNK)
        jobs.append((c, lo, hi))

    def run(job):
        c, lo, hi = job
        rng = np.random.default_rng([seed, c])
        full = rng.standard_normal(hi - c * CHUNK)
        out[lo - start:hi - start] = full[lo - c * CHUNK:]

    nthr = threads or min(len(jobs), max(1, min(16, os.cpu_count() or 1)))
    if nthr > 1 and len(jobs) > 1:
        with _fut.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(run, jobs))
    else:
        for j in jobs:
            run(j)
    if dtype == np.float64:
        return out
    return out.astype(dtype)


def vector(dim: int, seed: int = SEED_X, dtype=np.float64, k: int = 1) -> np.ndarray:
    """Seeded N(0,1) vector of ``dim`` rows (shape [dim] for k=1, else [dim, k])."""
    v = gaussian(dim * k, seed, dtype)
    return v if k == 1 else v.reshape(dim, k)


def random_states(Q: int, L: int, n: int, count: int, seed: int = 7) -> np.ndarray:
    """``count`` uniformly random words with digit sum n, as digit arrays [count, L].

    Q=2: a uniformly random n-subset of the sites (Fisher-Yates over site positions).
    Q>2: rejection sampling of uniform digit strings (only for small L).
    """
    rng = np.random.default_rng(seed)
    if Q == 2:
        keys = rng.random((count, L))
        order = np.argsort(keys, axis=1)
        digits = np.zeros((count, L), dtype=np.int64)
        rows = np.repeat(np.arange(count), n)
        digits[rows, order[:, :n].reshape(-1)] = 1
        return digits
    out = []
    got = 0
    while got < count:
        d = rng.integers(0, Q, size=(max(count, 1024) * 4, L))
        d = d[d.sum(axis=1) == n]
        out.append(d)
        got += len(d)
    return np.concatenate(out)[:count]


def pack_digits(digits: np.ndarray, Q: int) -> np.ndarray:
    """Pack digit rows into uint64 words, site 0 in the most significant field.

    This is the state encoding both sides use: ceil(log2 Q) bits per site, plain
    binary digits.
    """
    nbits = max(1, int(Q - 1).bit_length())
    digits = np.asarray(digits, dtype=np.uint64)
    L = digits.shape[-1]
    out = np.zeros(digits.shape[:-1], dtype=np.uint64)
    for i in range(L):
        out |= digits[..., i] << np.uint64(nbits * (L - 1 - i))
    return out


def random_local_matrix(Q: int, m: int, seed: int, density: float = 1.0) -> np.ndarray:
    """Seeded real Q^m x Q^m matrix with N(0,1) entries, kept only where the local digit
    strings of the row and the column have equal digit sums (the structure of a
    particle-number conserving term; local index sum_j d_j Q^(m-1-j)); ``density``
    keeps that fraction of those entries."""
    rng = np.random.default_rng([seed, Q, m])
    n = Q ** m
    sums = np.zeros(n, dtype=np.int64)
    for a in range(n):
        v, s = a, 0
        for _ in range(m):
            s += v % Q
            v //= Q
        sums[a] = s
    M = rng.standard_normal((n, n))
    mask = (sums[:, None] == sums[None, :]) & (rng.random((n, n)) < density)
    return np.where(mask, M, 0.0)


def random_local_matrix_dims(dims, seed: int, density: float = 1.0) -> np.ndarray:
    """The same on sites of local dimensions ``dims`` (one per listed site): an
    n x n matrix, n the product of the dims, local index the mixed-radix number of
    the digits with the first site most significant."""
    dims = [int(q) for q in dims]
    rng = np.random.default_rng([seed, len(dims)] + dims)
    n = int(np.prod(dims))
    sums = np.zeros(n, dtype=np.int64)
    for a in range(n):
        v, s = a, 0
        for q in reversed(dims):
            s += v % q
            v //= q
        sums[a] = s
    M = rng.standard_normal((n, n))
    mask = (sums[:, None] == sums[None, :]) & (rng.random((n, n)) < density)
    return np.where(mask, M, 0.0)
