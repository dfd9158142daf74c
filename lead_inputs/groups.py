"""Finite groups given by multiplication tables.

A group of order N is a table ``mul`` (uint16, N x N) with ``mul[g, h]`` the
index of the product g*h.  These tables are the group input G of the code
construction (the left-right Cayley complex of Section II-A is built from a
finite group G and two symmetric generating sets A, B).

Three families are provided, matching the workloads that are decoded:

* ``dihedral(n)``: the dihedral group of order 2n (order 12 for n = 6),
* ``alternating5()``: A_5, the even permutations of five points (order 60),
* ``psl2(q)``: PSL(2, F_q) for a prime q (order 168 for q = 7),

plus ``cyclic(n)`` for tiny hand-checkable cases.  Element numbering is a
fixed, documented convention of each constructor; nothing downstream depends
on it beyond the table itself.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Group:
    name: str
    mul: np.ndarray  # uint16 [N, N]
    labels: list = field(default_factory=list)

    @property
    def order(self) -> int:
        return int(self.mul.shape[0])

    @property
    def identity(self) -> int:
        n = self.order
        for e in range(n):
            if np.array_equal(self.mul[e], np.arange(n)):
                return e
        raise ValueError("table has no left identity")

    def inverse(self) -> np.ndarray:
        e = self.identity
        inv = np.empty(self.order, dtype=np.int64)
        for g in range(self.order):
            inv[g] = int(np.nonzero(self.mul[g] == e)[0][0])
        return inv

    def conjugacy_class_ids(self) -> np.ndarray:
        """cls[g] = a label shared exactly by the elements conjugate to g."""
        n = self.order
        inv = self.inverse()
        cls = -np.ones(n, dtype=np.int64)
        nxt = 0
        for g in range(n):
            if cls[g] >= 0:
                continue
            # x g x^-1 for every x
            conj = self.mul[self.mul[np.arange(n), g], inv]
            cls[np.unique(conj)] = nxt
            nxt += 1
        return cls


def _table_from_elements(elems, product, key):
    index = {key(x): i for i, x in enumerate(elems)}
    n = len(elems)
    mul = np.empty((n, n), dtype=np.uint16)
    for i, x in enumerate(elems):
        for j, y in enumerate(elems):
            mul[i, j] = index[key(product(x, y))]
    return mul


def cyclic(n: int) -> Group:
    """Z_n with element k the residue k; mul[a, b] = a + b mod n."""
    a = np.arange(n)
    mul = ((a[:, None] + a[None, :]) % n).astype(np.uint16)
    return Group(f"Z{n}", mul, [str(k) for k in range(n)])


def elementary_abelian2(k: int) -> Group:
    """(Z_2)^k with element x the bit vector x; mul[x, y] = x xor y."""
    a = np.arange(1 << k)
    mul = (a[:, None] ^ a[None, :]).astype(np.uint16)
    return Group(f"E2_{k}", mul, [format(x, f"0{k}b") for x in range(1 << k)])


def dihedral(n: int) -> Group:
    """Dihedral group of order 2n.

    Element f*n + k is r^k s^f (r a rotation of order n, s a reflection), and
    (r^a s^f)(r^b s^g) = r^(a + (-1)^f b) s^(f xor g).
    """
    elems = [(k, f) for f in (0, 1) for k in range(n)]

    def prod(x, y):
        a, f = x
        b, g = y
        return ((a + (b if f == 0 else -b)) % n, f ^ g)

    mul = _table_from_elements(elems, prod, lambda x: x)
    labels = [("r^%d" % k) + ("s" if f else "") for k, f in elems]
    return Group(f"D{n}", mul, labels)


def alternating5() -> Group:
    """A_5 as even permutations of {0..4} in lexicographic order of their
    images; (g*h)(x) = g(h(x))."""
    elems = []
    for p in itertools.permutations(range(5)):
        inversions = sum(1 for i in range(5) for j in range(i + 1, 5) if p[i] > p[j])
        if inversions % 2 == 0:
            elems.append(p)

    def prod(g, h):
        return tuple(g[h[x]] for x in range(5))

    mul = _table_from_elements(elems, prod, lambda x: x)
    return Group("A5", mul, ["".join(map(str, p)) for p in elems])


def psl2(q: int) -> Group:
    """PSL(2, F_q) for a prime q: 2x2 matrices of determinant 1 modulo +-I.

    Each class {M, -M} is represented by the matrix whose first non-zero entry
    (in the order a, b, c, d) is at most (q-1)/2; classes are numbered in
    lexicographic order of that representative.
    """
    def canon(m):
        a, b, c, d = m
        first = next(x for x in m if x != 0)
        if first > (q - 1) // 2:
            m = tuple((-x) % q for x in m)
        return m

    reps = set()
    for a, b, c, d in itertools.product(range(q), repeat=4):
        if (a * d - b * c) % q == 1:
            reps.add(canon((a, b, c, d)))
    elems = sorted(reps)

    def prod(x, y):
        a, b, c, d = x
        e, f, g, h = y
        return canon(((a * e + b * g) % q, (a * f + b * h) % q,
                      (c * e + d * g) % q, (c * f + d * h) % q))

    mul = _table_from_elements(elems, prod, lambda x: x)
    return Group(f"PSL2_{q}", mul, [str(m) for m in elems])


def by_name(name: str) -> Group:
    if name.startswith("E2_"):
        return elementary_abelian2(int(name[3:]))
    if name.startswith("Z"):
        return cyclic(int(name[1:]))
    if name.startswith("D"):
        return dihedral(int(name[1:]))
    if name == "A5":
        return alternating5()
    if name.startswith("PSL2_"):
        return psl2(int(name[5:]))
    raise KeyError(name)
