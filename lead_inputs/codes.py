"""Seeded code descriptions (G, A, B, C_A, C_B).

A quantum Tanner code is fixed by a finite group G, two symmetric generating
sets A = A^-1 and B = B^-1 of equal size Delta that satisfy the Total
No-Conjugacy condition (ag != gb for all a, b, g; Section II-A), and two
classical local codes C_A, C_B of length Delta (Section II-B).  This module
only *samples* such descriptions; building the code from them is the job of
the decoder library and, independently, of the oracle.

Sampling rules (the paper fixes none beyond symmetry and TNC):

* A and B exclude the identity and are unions of involutions and
  {x, x^-1} pairs, drawn in a seeded random order (the order of A and B is
  the local coordinate order of every vertex view).
* TNC holds iff no element of B is conjugate to an element of A, so B is
  drawn from the conjugacy classes that A does not touch.
* C_A, C_B are random full-rank [Delta, k] codes given by a (generally not
  reduced) generator matrix, with minimum distance >= 2 and no all-zero
  coordinate (equivalently, dual distance >= 2), so that every local check
  of either type has weight >= 4.
"""
from __future__ import annotations

from dataclasses import dataclass, asdict

import numpy as np

from .groups import Group, by_name


@dataclass
class CodeSpec:
    group: str
    mul: np.ndarray      # uint16 [N, N]
    delta: int
    A: list              # ordered element indices
    B: list
    kA: int
    GA: list             # kA generator rows, bit c = coordinate c
    kB: int
    GB: list
    seed: int

    @property
    def order(self) -> int:
        return int(self.mul.shape[0])

    def describe(self) -> dict:
        d = asdict(self)
        d.pop("mul")
        return d


def _rank_rows(rows, width):
    rows = [int(r) for r in rows]
    rank = 0
    for col in range(width):
        piv = next((i for i in range(rank, len(rows)) if (rows[i] >> col) & 1), None)
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and (rows[i] >> col) & 1:
                rows[i] ^= rows[rank]
        rank += 1
    return rank


def local_code_ok(rows, width) -> bool:
    """Full rank, no codeword of weight 1, no all-zero coordinate."""
    k = len(rows)
    if _rank_rows(rows, width) != k:
        return False
    span_or = 0
    for r in rows:
        span_or |= r
    if span_or != (1 << width) - 1:
        return False
    for combo in range(1, 1 << k):
        w = 0
        for i in range(k):
            if (combo >> i) & 1:
                w ^= rows[i]
        if bin(w).count("1") < 2:
            return False
    return True


def sample_local_code(width: int, k: int, rng: np.random.Generator, tries: int = 10000):
    for _ in range(tries):
        rows = [int(x) for x in rng.integers(1, 1 << width, size=k)]
        if local_code_ok(rows, width):
            return rows
    raise RuntimeError(f"no [{width},{k}] local code found")


def sample_symmetric_set(group: Group, delta: int, rng: np.random.Generator, allowed: np.ndarray):
    """An ordered inverse-closed set of `delta` non-identity elements drawn
    from `allowed`, or None if the random fill does not close."""
    inv = group.inverse()
    e = group.identity
    units = []
    for x in range(group.order):
        if x == e or not allowed[x]:
            continue
        if inv[x] == x:
            units.append((x,))
        elif x < inv[x] and allowed[inv[x]]:
            units.append((x, int(inv[x])))
    order = rng.permutation(len(units))
    chosen = []
    for idx in order:
        u = units[idx]
        if len(chosen) + len(u) <= delta:
            chosen.extend(u)
        if len(chosen) == delta:
            break
    if len(chosen) != delta:
        return None
    return [int(chosen[i]) for i in rng.permutation(delta)]


def sample_generating_sets(group: Group, delta: int, rng: np.random.Generator, tries: int = 2000):
    cls = group.conjugacy_class_ids()
    all_ok = np.ones(group.order, dtype=bool)
    for _ in range(tries):
        A = sample_symmetric_set(group, delta, rng, all_ok)
        if A is None:
            continue
        used = set(int(cls[a]) for a in A)
        allowed_b = np.array([int(cls[x]) not in used for x in range(group.order)])
        B = sample_symmetric_set(group, delta, rng, allowed_b)
        if B is None:
            continue
        return A, B
    raise RuntimeError("no (A, B) pair satisfying TNC found")


def sample_code(group_name: str, delta: int, kA: int, kB: int, seed: int) -> CodeSpec:
    group = by_name(group_name)
    rng = np.random.default_rng(np.random.PCG64([0xC0DE, seed]))
    A, B = sample_generating_sets(group, delta, rng)
    GA = sample_local_code(delta, kA, rng)
    GB = sample_local_code(delta, kB, rng)
    return CodeSpec(group_name, group.mul, delta, A, B, kA, GA, kB, GB, seed)


def custom_code(group_name: str, delta: int, A, B, GA, GB) -> CodeSpec:
    group = by_name(group_name)
    return CodeSpec(group_name, group.mul, delta, list(A), list(B), len(GA), list(GA),
                    len(GB), list(GB), -1)


# Standard instances decoded by the tests and the benchmark.  Seeds were chosen
# so that each code has k >= 1 logical qubits (k is recorded beside the
# instance in tests/golden/instances.json, written by a script that uses the
# oracle only).
STANDARD = {
    # dihedral group of order 12, Delta = 4, [4,2] local codes, n = 96
    "T": ("D6", 4, 2, 2, 1),
    # A_5 (order 60), Delta = 6, [6,3] local codes, n = 1080
    "M": ("A5", 6, 3, 3, 1),
    # PSL(2,7) (order 168), Delta = 8, [8,4] local codes, n = 5376
    "L": ("PSL2_7", 8, 4, 4, 1),
}


def standard(name: str) -> CodeSpec:
    g, d, ka, kb, seed = STANDARD[name]
    return sample_code(g, d, ka, kb, seed)
