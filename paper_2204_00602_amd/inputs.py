"""Seeded synthetic inputs for the SLOS hot path.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, imports nothing from the rest of the package, and is the
one module that both the library's tests/benchmarks and the CPU oracle's
checks take inputs from.

Workload recipe (the paper's workloads are Haar-random interferometers fed
with single photons, Sections 4.2.1-4.2.2 and the Appendix B.6 QML code):
  * haar_unitary: Z = (N(0,1) + i N(0,1)) / sqrt(2), Z = QR, U = Q diag(R_ii/|R_ii|)
    with numpy's PCG64 generator (the paper only says "Haar random" and uses
    a seeded generator that consumes 2 m^2 reals).
  * batch_instances: m ~ U{6..14}, n ~ U{2..min(7, m)}, photons placed one at a
    time into a uniformly chosen mode with occupancy < 2.
  * uniform_fock_states: distinct outputs drawn uniformly from S_{m,n}
    (stars and bars: a uniform (m-1)-subset of m+n-1 slots marks the bars).
"""
from __future__ import annotations

import math

import numpy as np


def haar_unitary(m: int, seed: int) -> np.ndarray:
    """m x m Haar-random unitary, complex128, from a seeded PCG64 stream."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = d / np.abs(d)
    return np.ascontiguousarray(q * ph[np.newaxis, :])


def first_modes_input(m: int, n: int) -> np.ndarray:
    """|1,...,1,0,...,0>: one photon in each of the first n modes."""
    t = np.zeros(m, dtype=np.int32)
    t[:n] = 1
    return t


def fourier_unitary(m: int) -> np.ndarray:
    """F[j, k] = exp(2 pi i j k / m) / sqrt(m)."""
    j = np.arange(m)
    return np.exp(2j * np.pi * np.outer(j, j) / m) / math.sqrt(m)


def periodic_input(m: int, n: int) -> np.ndarray:
    """One photon in each of modes 0, p, 2p, ..., (n-1)p with p = m // n."""
    assert m % n == 0
    t = np.zeros(m, dtype=np.int32)
    t[:: m // n] = 1
    return t


def random_input(m: int, n: int, rng: np.random.Generator, max_per_mode: int = 2) -> np.ndarray:
    """Place n photons one by one into a uniform mode among those with room left."""
    t = np.zeros(m, dtype=np.int32)
    for _ in range(n):
        free = np.nonzero(t < max_per_mode)[0]
        t[free[rng.integers(len(free))]] += 1
    return t


def batch_instances(count: int, seed: int, m_range=(6, 14), n_max: int = 7):
    """Uneven batch: list of (m, n, input_state, U) with m ~ U{6..14}, n ~ U{2..min(7,m)}."""
    rng = np.random.default_rng(seed)
    out = []
    for idx in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(2, min(n_max, m) + 1))
        t = random_input(m, n, rng)
        u = haar_unitary(m, seed * 1_000_003 + idx)
        out.append((m, n, t, u))
    return out


def uniform_fock_states(m: int, n: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct outputs drawn uniformly from S_{m,n} (count x m int32).

    Stars and bars: a uniform (m-1)-subset of the m+n-1 slots (the slots of the
    m-1 smallest of m+n-1 uniform keys) marks the bars, and the gaps between
    consecutive bars are the occupations.  Candidates are drawn in bulk and the
    first occurrence of each state is kept, in draw order.
    """
    rng = np.random.default_rng(seed)
    total = math.comb(m + n - 1, n)
    count = min(count, total)
    if m == 1:
        return np.full((count, 1), n, dtype=np.int32)
    rows = np.zeros((0, m), dtype=np.int32)
    while rows.shape[0] < count:
        need = count - rows.shape[0]
        draw = need + need // 4 + 64
        keys = rng.random((draw, m + n - 1))
        bars = np.sort(np.argpartition(keys, m - 2, axis=1)[:, :m - 1], axis=1)
        edges = np.concatenate((np.full((draw, 1), -1), bars, np.full((draw, 1), m + n - 1)), axis=1)
        occ = (np.diff(edges, axis=1) - 1).astype(np.int32)
        allr = np.concatenate((rows, occ))
        _, first = np.unique(allr, axis=0, return_index=True)
        rows = allr[np.sort(first)]
    return np.ascontiguousarray(rows[:count])


def bunched_fock_states(m: int, n: int, count: int) -> np.ndarray:
    """The `count` most bunched outputs (largest sum of s_j^2), ties by mode order."""
    rows = []
    # all photons in one mode, then n-1 + 1, then n-2 + 2 / n-2 + 1 + 1, ...
    for a in range(m):
        s = np.zeros(m, np.int32)
        s[a] = n
        rows.append(s)
    if n >= 2:
        for a in range(m):
            for b in range(m):
                if a != b:
                    s = np.zeros(m, np.int32)
                    s[a] = n - 1
                    s[b] = 1
                    rows.append(s)
    if n >= 4:
        for a in range(m):
            for b in range(m):
                if a != b:
                    s = np.zeros(m, np.int32)
                    s[a] = n - 2
                    s[b] = 2
                    rows.append(s)
    return np.asarray(rows[:count], dtype=np.int32).reshape(-1, m)


def mesh_phases(batch: int, n_mzi: int, seed: int) -> np.ndarray:
    """batch x (2 n_mzi) phases uniform in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * math.pi, size=(batch, 2 * n_mzi))
