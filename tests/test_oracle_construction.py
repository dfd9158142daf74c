"""Pins of the oracle's code construction (Section II) against the paper's
definitions, brute force and the Appendix-A worked example."""
import itertools
import json
import os

import numpy as np
import pytest

from conftest import code_pair
from lead_inputs import by_name, custom_code, standard, bitflip_packed, unpack_bits, pack_bits

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gf2_rank(M):
    """Row rank over GF(2) by plain Gaussian elimination (test-side code)."""
    M = (np.array(M, dtype=np.uint8) & 1).copy()
    rank = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = None
        for r in range(rank, rows):
            if M[r, c]:
                piv = r
                break
        if piv is None:
            continue
        M[[rank, piv]] = M[[piv, rank]]
        for r in range(rows):
            if r != rank and M[r, c]:
                M[r] ^= M[rank]
        rank += 1
    return rank


def square(mul, A, B, g, i, j):
    """The face {(g,0), (a g,1), (g b,1), (a g b,0)} of Sec. II-A."""
    a, b = A[i], B[j]
    ag = int(mul[a, g])
    return frozenset({(g, 0), (ag, 1), (int(mul[g, b]), 1), (int(mul[ag, b]), 0)})


@pytest.mark.parametrize("name", ["appendix", "Z5", "D3", "T", "M"])
def test_views_match_square_definition(name):
    """c-1: n = |G| Delta^2 / 2; the view of every vertex lists exactly the
    Delta^2 squares incident to it; every qubit lies in two V0 and two V1
    views."""
    spec, oc = code_pair(name)
    mul, A, B, D, N = spec.mul.astype(np.int64), spec.A, spec.B, spec.delta, spec.order
    assert oc.n == N * D * D // 2
    v0, v1 = oc.views(0), oc.views(1)
    q_to_sq = {}
    for g in range(N):
        for i in range(D):
            for j in range(D):
                sq = square(mul, A, B, g, i, j)
                assert len(sq) == 4                       # TNC: four distinct corners
                q = int(v0[g, i * D + j])
                assert q_to_sq.setdefault(q, sq) == sq
    assert len(q_to_sq) == oc.n and len(set(q_to_sq.values())) == oc.n
    # incidence: squares at each vertex
    at = {}
    for q, sq in q_to_sq.items():
        for vert in sq:
            at.setdefault(vert, set()).add(q)
    for g in range(N):
        assert set(v0[g].tolist()) == at[(g, 0)] and len(at[(g, 0)]) == D * D
        assert set(v1[g].tolist()) == at[(g, 1)] and len(at[(g, 1)]) == D * D
    for t in (v0, v1):
        counts = np.bincount(t.ravel(), minlength=oc.n)
        assert np.all(counts == 2)


def test_appendix_local_check_layout():
    """c-3: rep[3,1] with its dual gives exactly the rows of eq. (product)
    (a-major columns, reduced-echelon basis of the even-weight code)."""
    fx = json.load(open(os.path.join(GOLDEN, "appendix_a.json")))["local_check_layout"]
    _, oc = code_pair("appendix")
    want = np.array([[int(ch) for ch in row] for row in fx["rows"]], dtype=np.uint8)
    assert np.array_equal(oc.hloc(0), want)


def _in_span(vec, rows):
    rows = [int(r) for r in rows]
    for combo in range(1 << len(rows)):
        w = 0
        for i, r in enumerate(rows):
            if (combo >> i) & 1:
                w ^= r
        if w == vec:
            return True
    return False


def _is_rref(rows, width):
    piv = []
    for r in rows:
        bits = [c for c in range(width) if (r >> c) & 1]
        if not bits:
            return False
        piv.append(bits[0])
    if piv != sorted(piv) or len(set(piv)) != len(piv):
        return False
    for k, p in enumerate(piv):
        for k2, r in enumerate(rows):
            if k2 != k and (r >> p) & 1:
                return False
    return True


@pytest.mark.parametrize("name", ["appendix", "T", "M", "L"])
def test_local_checks_are_tensor_basis(name):
    """c-2 / reading of the check basis: every local Z row is u (x) v with
    u, v rows of the reduced-echelon bases of C_A, C_B (X rows: of the dual
    codes), rows ordered (u index) * kB + (v index); weights <= Delta^2."""
    spec, oc = code_pair(name)
    D = spec.delta
    for t in (0, 1):
        hl = oc.hloc(t)
        us, vs = [], []
        for row in hl:
            M = row.reshape(D, D)
            a_idx = np.nonzero(M.any(axis=1))[0]
            b_idx = np.nonzero(M.any(axis=0))[0]
            u = sum(1 << int(a) for a in a_idx)
            v = sum(1 << int(b) for b in b_idx)
            outer = np.outer([(u >> a) & 1 for a in range(D)], [(v >> b) & 1 for b in range(D)])
            assert np.array_equal(outer, M)
            us.append(u)
            vs.append(v)
            assert row.sum() <= D * D
        ua = list(dict.fromkeys(us))
        vb = list(dict.fromkeys(vs))
        ka, kb = (spec.kA, spec.kB) if t == 0 else (D - spec.kA, D - spec.kB)
        assert len(ua) == ka and len(vb) == kb and len(hl) == ka * kb
        assert [us[i] for i in range(0, len(us), kb)] == ua
        assert vs[:kb] == vb
        assert _is_rref(ua, D) and _is_rref(vb, D)
        for u in ua:
            if t == 0:
                assert _in_span(u, spec.GA)
            else:
                assert all(bin(u & g).count("1") % 2 == 0 for g in spec.GA)
        for v in vb:
            if t == 0:
                assert _in_span(v, spec.GB)
            else:
                assert all(bin(v & g).count("1") % 2 == 0 for g in spec.GB)
        assert gf2_rank(hl) == ka * kb


@pytest.mark.parametrize("name", ["appendix", "Z5", "D3", "T", "M"])
def test_global_rows_are_placed_local_checks_and_css(name):
    """Global check v*r + rho is local check rho placed on the view of v;
    CSS condition H_X H_Z^T = 0 (Sec. II-B)."""
    spec, oc = code_pair(name)
    for t in (0, 1):
        H, hl, view = oc.H(t), oc.hloc(t), oc.views(t)
        r = hl.shape[0]
        for v in range(spec.order):
            for rho in range(r):
                row = H[v * r + rho]
                want = np.zeros(oc.n, dtype=np.uint8)
                want[view[v][hl[rho] == 1]] = 1
                assert np.array_equal(row, want)
    HZ, HX = oc.H(0).astype(np.int64), oc.H(1).astype(np.int64)
    assert not np.any((HX @ HZ.T) % 2)


@pytest.mark.parametrize("name", ["Z5", "D3"])
def test_rank_and_logicals_brute_force(name):
    """c-4 / c-12 on codes small enough to enumerate F_2^n: rank from the
    kernel size, k = n - rank_X - rank_Z, and both logical tests agree with
    explicit rowspace membership."""
    spec, oc = code_pair(name)
    n = oc.n
    xs = np.arange(1 << n, dtype=np.int64)
    bits = ((xs[:, None] >> np.arange(n)) & 1).astype(np.int64)
    for t in (0, 1):
        H = oc.H(t).astype(np.int64)
        in_ker = ~np.any((bits @ H.T) % 2, axis=1)
        dim_ker = int(np.log2(in_ker.sum()))
        assert oc.info.rank[t] == n - dim_ker
    assert oc.k == n - oc.info.rank[0] - oc.info.rank[1]
    for t in (0, 1):
        H, Ho = oc.H(t).astype(np.int64), oc.H(1 - t).astype(np.int64)
        span = set()
        for combo in range(1 << Ho.shape[0]):
            sel = [(combo >> i) & 1 for i in range(Ho.shape[0])]
            vec = (np.array(sel) @ Ho) % 2
            span.add(int(sum(int(b) << q for q, b in enumerate(vec))))
        ker = xs[~np.any((bits @ H.T) % 2, axis=1)]
        res = pack_bits(((ker[:, None] >> np.arange(n)) & 1).astype(np.uint8))
        f0 = oc.logical_failure(res, t, route=0)
        f1 = oc.logical_failure(res, t, route=1)
        truth = np.array([int(x) not in span for x in ker])
        assert np.array_equal(f0, truth) and np.array_equal(f1, truth)
        assert oc.logicals(t).shape == (oc.k, n)


@pytest.mark.parametrize("name", ["appendix", "T", "M"])
def test_logical_basis(name):
    """Logical operators for check type t commute with the other type's
    stabilisers and are independent modulo H_t's rowspace; the two logical
    tests agree on residuals (other-type stabilisers plus other-type logicals,
    all in ker H_t), and flag exactly those with a logical component."""
    spec, oc = code_pair(name)
    rng = np.random.default_rng(5)
    for t in (0, 1):
        H, Ho, Lg, Lo = oc.H(t), oc.H(1 - t), oc.logicals(t), oc.logicals(1 - t)
        assert not np.any((Ho.astype(np.int64) @ Lg.T.astype(np.int64)) % 2)
        assert gf2_rank(np.vstack([H, Lg])) == oc.info.rank[t] + oc.k
        for _ in range(30):
            stab = (rng.integers(0, 2, Ho.shape[0]) @ Ho.astype(np.int64)) % 2
            lsel = rng.integers(0, 2, oc.k)
            res = (stab + lsel @ Lo.astype(np.int64)) % 2
            assert not np.any((H.astype(np.int64) @ res) % 2)
            packed = pack_bits(res[None].astype(np.uint8))
            f0 = oc.logical_failure(packed, t, 0)[0]
            f1 = oc.logical_failure(packed, t, 1)[0]
            assert f0 == f1 == bool(lsel.any())
            assert f1 == (gf2_rank(np.vstack([Ho, res])) > oc.info.rank[1 - t])


@pytest.mark.parametrize("name", ["T", "M"])
def test_syndrome_is_H_times_e(name):
    spec, oc = code_pair(name)
    e = bitflip_packed(64, oc.n, 0.05, seed=11)
    for t in (0, 1):
        s = oc.syndrome(e, t)
        want = (unpack_bits(e, oc.n).astype(np.int64) @ oc.H(t).T.astype(np.int64)) % 2
        assert np.array_equal(unpack_bits(s, oc.m(t)), want.astype(np.uint8))


def test_standard_instances_golden():
    """The standard instances keep their recorded structure, with k >= 1."""
    from oracle.oracle import OracleCode
    gold = json.load(open(os.path.join(GOLDEN, "instances.json")))
    for name, rec in gold.items():
        if name == "L":
            continue  # covered by the slower test below
        oc = OracleCode.from_spec(standard(name))
        assert (oc.n, list(oc.info.rank), oc.k, list(oc.info.eloc)) == \
            (rec["n"], rec["rank"], rec["k"], rec["eloc"])
        assert oc.k >= 1


def test_large_instance_golden():
    from oracle.oracle import OracleCode
    rec = json.load(open(os.path.join(GOLDEN, "instances.json")))["L"]
    oc = OracleCode.from_spec(standard("L"))
    assert (oc.n, list(oc.info.rank), oc.k, list(oc.info.eloc)) == \
        (rec["n"], rec["rank"], rec["k"], rec["eloc"])


def test_build_rejects_invalid_descriptions(oracle_mod):
    from oracle.oracle import OracleCode, OracleError
    g = by_name("Z5").mul
    cases = [
        ((g, 2, [1, 4], [1, 4], [0b11], [0b11]), -4),    # A = B in an abelian group: TNC fails
        ((g, 2, [1, 2], [2, 3], [0b11], [0b11]), -3),    # A not inverse-closed
        ((g, 2, [0, 4], [2, 3], [0b11], [0b11]), -3),    # identity in A
        ((by_name("D6").mul, 4, standard("T").A, standard("T").B, [0b0001, 0b0110], [0b0011, 0b1100]), -5),
        ((by_name("D6").mul, 4, standard("T").A, standard("T").B, [0b0011, 0b0011], [0b0011, 0b1100]), -5),
    ]
    for args, code in cases:
        with pytest.raises(OracleError) as ei:
            OracleCode(*args)
        assert ei.value.code == code
    bad = np.array(g, copy=True)
    bad[1, 1] = 3
    with pytest.raises(OracleError) as ei:
        OracleCode(bad, 2, [1, 4], [2, 3], [0b11], [0b11])
    assert ei.value.code == -2
