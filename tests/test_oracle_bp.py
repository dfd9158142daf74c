"""Pins of the oracle's decoder (Algorithm 1 with BP local and global
decoders) against brute force, closed forms, the Appendix-A example and
invariants of the method."""
import json
import os

import numpy as np
import pytest

from conftest import code_pair
from lead_inputs import bitflip_packed, unpack_bits, pack_bits, channel_llr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# computation-tree brute force (test-side, independent of the oracle's BP)
# ---------------------------------------------------------------------------

def _graph(H):
    checks = [list(np.nonzero(row)[0]) for row in H]
    var_checks = [list(np.nonzero(H[:, j])[0]) for j in range(H.shape[1])]
    return checks, var_checks


def computation_tree(H, s, lam, root, depth):
    """Unroll the Tanner graph of H from `root` through `depth` check
    layers.  Returns (priors of the variable copies, [(copies, s bit)])."""
    checks, var_checks = _graph(H)
    copies, cons = [float(lam[root])], []

    def expand(ci, var, parent, d):
        for c in var_checks[var]:
            if c == parent:
                continue
            members = [ci]
            for v2 in checks[c]:
                if v2 == var:
                    continue
                k = len(copies)
                copies.append(float(lam[v2]))
                members.append(k)
                if d + 1 < depth:
                    expand(k, v2, c, d + 1)
            cons.append((members, int(s[c])))

    expand(0, root, None, 0)
    return np.array(copies), cons


def tree_root_llr(copies, cons, kind):
    """Exact root LLR on a tree by enumerating every assignment.
    'sp': ln P(e_root=0 | checks) / P(e_root=1 | checks) with P(e) ~ exp(-sum lam e);
    'ms': min cost with e_root=1 minus min cost with e_root=0."""
    V = len(copies)
    x = np.arange(1 << V, dtype=np.int64)
    ok = np.ones(x.shape, dtype=bool)
    for members, sb in cons:
        mask = 0
        for m in members:
            mask |= 1 << m
        ok &= (np.bitwise_count(x & mask) & 1) == sb
    cost = np.zeros(x.shape, dtype=np.float64)
    for i, l in enumerate(copies):
        cost += l * ((x >> i) & 1)
    r0 = ok & ((x & 1) == 0)
    r1 = ok & ((x & 1) == 1)
    if kind == "ms":
        return cost[r1].min() - cost[r0].min()
    c0, c1 = cost[r0], cost[r1]
    m = min(c0.min(), c1.min())
    return np.log(np.exp(-(c0 - m)).sum()) - np.log(np.exp(-(c1 - m)).sum())


def _cases(H, depth, limit=20, max_copies=21):
    out = []
    for root in range(H.shape[1]):
        copies, cons = computation_tree(H, np.zeros(H.shape[0]), np.zeros(H.shape[1]), root, depth)
        if len(copies) <= max_copies:
            out.append(root)
    return out[:limit]


@pytest.mark.parametrize("name,t,depth", [("appendix", 0, 1), ("appendix", 0, 2), ("appendix", 1, 2),
                                          ("T", 0, 1), ("T", 1, 1), ("T_pairs", 0, 3)])
@pytest.mark.parametrize("kind", ["sp", "ms"])
def test_bp_equals_computation_tree_marginals(name, t, depth, kind):
    """c-5 / c-6: after `depth` iterations BP's posterior of a variable is
    the exact marginal (sum-product) or min-cost difference (min-sum, scale
    1) of that variable on its depth-`depth` computation tree; on a forest
    (T_pairs) this is the exact marginal of the code itself."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    H = oc.hloc(t)
    rng = np.random.default_rng(100 + depth)
    roots = _cases(H, depth)
    assert roots, "no computation tree small enough"
    p = o.params(bp=o.SUMPRODUCT if kind == "sp" else o.MINSUM, ms_scale=1.0, early_exit=0,
                 llr_clamp=1e6)
    for trial in range(3):
        lam = rng.uniform(-1.0, 4.0, size=H.shape[1])
        s = rng.integers(0, 2, size=H.shape[0]).astype(np.uint8)
        L, e, conv, it = o.bp(H, s, lam, depth, p)
        assert it == depth
        for root in roots:
            copies, cons = computation_tree(H, s, lam, root, depth)
            want = tree_root_llr(copies, cons, kind)
            assert abs(L[root] - want) < 1e-9 * max(1.0, abs(want)), (root, L[root], want)


def test_forest_view_equals_exact_local_marginals():
    """c-5 on a whole view: with pair local codes each local Tanner graph is
    a forest, so sum-product gives the exact posterior of every qubit of the
    view given its local syndrome (2^16 patterns enumerated)."""
    from oracle import oracle as o
    _, oc = code_pair("T_pairs")
    H = oc.hloc(0)
    n = H.shape[1]
    rng = np.random.default_rng(7)
    x = np.arange(1 << n, dtype=np.int64)
    bits = ((x[:, None] >> np.arange(n)) & 1).astype(np.float64)
    synd = (bits @ H.T.astype(np.float64)) % 2
    for _ in range(3):
        lam = rng.uniform(-0.5, 3.0, size=n)
        s = rng.integers(0, 2, size=H.shape[0]).astype(np.uint8)
        ok = np.all(synd == s, axis=1)
        logw = -(bits @ lam)
        L, e, conv, it = o.bp(H, s, lam, 4, o.params(bp=o.SUMPRODUCT, early_exit=0))
        for j in range(n):
            w0 = np.exp(logw[ok & (bits[:, j] == 0)])
            w1 = np.exp(logw[ok & (bits[:, j] == 1)])
            assert abs(L[j] - np.log(w0.sum() / w1.sum())) < 1e-9


@pytest.mark.parametrize("name", ["T", "M", "appendix"])
def test_first_iteration_is_scaled_single_check_min_cost(name):
    """c-7: after one min-sum iteration with scale beta, L_j = lam_j + beta *
    sum over checks c of j of the exact min-cost message of check c alone
    (brute force over each check's support)."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    rng = np.random.default_rng(3)
    for t in (0, 1):
        H = oc.hloc(t)
        for _ in range(3):
            lam = rng.uniform(-1.0, 4.0, size=H.shape[1])
            s = rng.integers(0, 2, size=H.shape[0]).astype(np.uint8)
            L, _, _, _ = o.bp(H, s, lam, 1, o.params(ms_scale=0.75, early_exit=0))
            want = lam.copy()
            for c in range(H.shape[0]):
                sup = list(np.nonzero(H[c])[0])
                w = len(sup)
                pats = ((np.arange(1 << w)[:, None] >> np.arange(w)) & 1)
                good = (pats.sum(axis=1) % 2) == s[c]
                for k, j in enumerate(sup):
                    others = [q for q in range(w) if q != k]
                    cost = pats[:, others] @ lam[[sup[q] for q in others]]
                    c1 = cost[good & (pats[:, k] == 1)].min()
                    c0 = cost[good & (pats[:, k] == 0)].min()
                    want[j] += 0.75 * (c1 - c0)
            want = np.clip(want, -30, 30)
            assert np.allclose(L, want, atol=1e-12)


def test_appendix_aggregation_example():
    """c-9: Appendix A, Phase 2: views v1 and v2 hold qubit 1 with 0.21 and
    0.25; alpha = 1 gives 0.23; the result is linear in alpha and its LLR is
    ln((1-p)/p)."""
    from oracle import oracle as o
    fx = json.load(open(os.path.join(GOLDEN, "appendix_a.json")))["aggregation"]
    view = np.array([fx["view_v1_qubits"], fx["view_v2_qubits"]]) - 1
    pv = np.array([fx["view_v1_p"], fx["view_v2_p"]])
    q = fx["qubit"] - 1
    phat, lam = o.aggregate(15, view, pv, fx["alpha"])
    assert abs(phat[q] - fx["expected_phat"]) < 1e-12
    assert abs(lam[q] - np.log((1 - 0.23) / 0.23)) < 1e-12
    for alpha in (0.5, 0.01):
        ph2, _ = o.aggregate(15, view, pv, alpha)
        assert np.allclose(ph2, alpha * phat, rtol=1e-12)
    # a qubit seen by a single view keeps that view's value
    assert abs(phat[1] - 0.12) < 1e-12 and abs(phat[12] - 0.50) < 1e-12


def _decode(oc, synd, lam, t=0, **kw):
    from oracle import oracle as o
    return oc.decode(synd, lam, t=t, p=o.params(**kw))


@pytest.mark.parametrize("name", ["T", "M"])
def test_boost_is_a_noop_for_bp_local_decoders(name):
    """c-8: with BP hard decisions e_j = 1 iff L_j < 0 iff p_j > 1/2, so the
    confidence boost max(p, 0.5) never changes anything."""
    spec, oc = code_pair(name)
    e = bitflip_packed(40, oc.n, 0.05, seed=2)
    lam = float(channel_llr(0.05))
    for t in (0, 1):
        s = oc.syndrome(e, t)
        a = _decode(oc, s, lam, t, max_iter_local=20, max_iter_global=20, boost=1)
        b = _decode(oc, s, lam, t, max_iter_local=20, max_iter_global=20, boost=0)
        for key in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("name", ["T", "M"])
@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_zero_syndrome_closed_form(name, alpha):
    """c-10: s = 0 with a uniform prior lam > 0: every local view converges
    after one iteration with L_j = lam (1 + beta d_j); Phase 2 gives
    p_i = alpha * mean of sigma(-L) over the two views; global BP converges
    after one iteration with L_i = lam'_i + beta sum_c min_{i' in c, i' != i} lam'_i';
    the estimate is e = 0."""
    spec, oc = code_pair(name)
    beta, lam = 0.75, float(channel_llr(0.05))
    for t in (0, 1):
        s = np.zeros((2, (oc.m(t) + 63) // 64), dtype=np.uint64)
        out = _decode(oc, s, lam, t, alpha=alpha, max_iter_local=10, max_iter_global=10)
        st = out["stats"]
        N = spec.order
        assert np.array_equal(st[:, 0], [1, 1]) and np.array_equal(st[:, 1], [1, 1])
        assert np.array_equal(st[:, 2], [N, N]) and np.array_equal(st[:, 3], [1, 1])
        assert np.array_equal(st[:, 4], [N, N])
        assert not out["ehat"].any()
        deg = oc.hloc(t).sum(axis=0)
        view = oc.views(t)
        psum = np.zeros(oc.n)
        for v in range(N):
            psum[view[v]] += 1.0 / (1.0 + np.exp(lam * (1 + beta * deg)))
        ph = alpha * psum / 2.0
        lamp = np.log(1 - ph) - np.log(ph)
        assert np.allclose(out["lam"][0], lamp, rtol=1e-12, atol=1e-12)
        H = oc.H(t)
        Lpost = lamp.copy()
        for row in H:
            sup = np.nonzero(row)[0]
            vals = lamp[sup]
            for k, i in enumerate(sup):
                Lpost[i] += beta * np.min(np.delete(vals, k))
        assert np.allclose(out["post"][0], np.clip(Lpost, -30, 30), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", ["T", "M"])
def test_converged_means_syndrome_reproduced(name):
    """c-11: converged => H e_hat = s (independent GF(2) product)."""
    spec, oc = code_pair(name)
    e = bitflip_packed(60, oc.n, 0.03, seed=4)
    lam = float(channel_llr(0.03))
    for t in (0, 1):
        s = oc.syndrome(e, t)
        out = _decode(oc, s, lam, t, max_iter_local=30, max_iter_global=30)
        conv = out["stats"][:, 0] == 1
        assert conv.any()
        sh = (unpack_bits(out["ehat"], oc.n).astype(np.int64) @ oc.H(t).T.astype(np.int64)) % 2
        same = np.all(sh == unpack_bits(s, oc.m(t)), axis=1)
        assert np.array_equal(conv, same)


def _left_kernel_vector(H):
    """A y with y^T H = 0 over GF(2), y != 0 (test-side elimination)."""
    Ht = (H.T.astype(np.uint8) & 1).copy()        # n x m ; want y in ker(Ht)
    rows, cols = Ht.shape
    piv_cols, r = [], 0
    M = Ht.copy()
    for c in range(cols):
        pr = next((i for i in range(r, rows) if M[i, c]), None)
        if pr is None:
            continue
        M[[r, pr]] = M[[pr, r]]
        for i in range(rows):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        piv_cols.append(c)
        r += 1
    free = next(c for c in range(cols) if c not in piv_cols)
    y = np.zeros(cols, dtype=np.uint8)
    y[free] = 1
    for i, pc in enumerate(piv_cols):
        y[pc] = M[i, free]
    assert not np.any((y.astype(np.int64) @ H.astype(np.int64)) % 2)
    return y


@pytest.mark.parametrize("name", ["T", "M"])
def test_invalid_syndrome_never_converges(name):
    """c-11: a syndrome outside the image of H cannot be reproduced, so no
    shot may report convergence."""
    spec, oc = code_pair(name)
    for t in (0, 1):
        y = _left_kernel_vector(oc.H(t))
        e = bitflip_packed(20, oc.n, 0.02, seed=8)
        s = unpack_bits(oc.syndrome(e, t), oc.m(t))
        j = int(np.nonzero(y)[0][0])
        s[:, j] ^= 1                                 # y . s = 1  =>  s not in im H
        out = _decode(oc, pack_bits(s), float(channel_llr(0.02)), t, max_iter_local=10,
                      max_iter_global=10)
        assert not out["stats"][:, 0].any()


def test_equivariance_under_centre_translation():
    """c-13: g -> x g with x central in D_6 maps square (g,a,b) to (xg,a,b)
    and check (g,rho) to (xg,rho); LEAD commutes with the relabelling."""
    spec, oc = code_pair("T")
    mul = spec.mul.astype(np.int64)
    N, D2 = spec.order, spec.delta ** 2
    centre = [x for x in range(N) if x != 0 and np.array_equal(mul[x, :], mul[:, x])]
    assert centre
    x = centre[0]
    e = bitflip_packed(50, oc.n, 0.06, seed=9)
    lam = float(channel_llr(0.06))
    for t in (0, 1):
        view = oc.views(t)
        r = oc.hloc(t).shape[0]
        qperm = np.empty(oc.n, dtype=np.int64)
        for g in range(N):
            qperm[view[g]] = view[mul[x, g]]
        cperm = np.array([mul[x, g] * r + rho for g in range(N) for rho in range(r)])
        eb = unpack_bits(e, oc.n)
        e2 = np.zeros_like(eb)
        e2[:, qperm] = eb
        s = oc.syndrome(e, t)
        s2 = oc.syndrome(pack_bits(e2), t)
        sb = unpack_bits(s, oc.m(t))
        assert np.array_equal(unpack_bits(s2, oc.m(t))[:, cperm], sb)
        a = _decode(oc, s, lam, t, max_iter_local=25, max_iter_global=25)
        b = _decode(oc, s2, lam, t, max_iter_local=25, max_iter_global=25)
        assert np.allclose(b["post"][:, qperm], a["post"], atol=1e-9)
        assert np.allclose(b["lam"][:, qperm], a["lam"], atol=1e-9)
        assert np.array_equal(unpack_bits(b["ehat"], oc.n)[:, qperm], unpack_bits(a["ehat"], oc.n))
        assert np.array_equal(a["stats"], b["stats"])


def test_local_stage_extracts_vertex_slices():
    """Phase 1 extraction (a1, a2): the local posteriors of view v equal BP on
    H_v with s_v = bits v*r .. v*r+r-1 of s and the priors of the qubits of
    Q(v); checked against depth-2 computation-tree brute force."""
    from oracle import oracle as o
    spec, oc = code_pair("appendix")
    rng = np.random.default_rng(21)
    H = oc.hloc(0)
    r = H.shape[0]
    roots = _cases(H, 2)
    lamq = rng.uniform(0.2, 3.0, size=oc.n)
    e = (rng.random((1, oc.n)) < 0.2).astype(np.uint8)
    s = oc.syndrome(pack_bits(e), 0)
    out = oc.decode(s, lamq[None, :], t=0, p=o.params(max_iter_local=2, ms_scale=1.0, early_exit=0,
                                                      stage=o.LOCAL), want_local=True)
    sb = unpack_bits(s, oc.m(0))[0]
    view = oc.views(0)
    for v in range(spec.order):
        sv = sb[v * r:(v + 1) * r]
        for root in roots:
            copies, cons = computation_tree(H, sv, lamq[view[v]], root, 2)
            assert abs(out["local"][0, v, root] - tree_root_llr(copies, cons, "ms")) < 1e-9


@pytest.mark.parametrize("name", ["T", "M"])
def test_iteration_count_is_first_success(name):
    """Stopping rule: with early exit, a run that reports t iterations and
    convergence has H e != s after t-1 iterations and reproduces, with early
    exit off and exactly t iterations, the same posterior; without early
    exit the count is the cap."""
    from oracle import oracle as o
    spec, oc = code_pair(name)
    H = oc.hloc(0)
    rng = np.random.default_rng(31)
    seen = set()
    for trial in range(300):
        lam = rng.uniform(0.5, 4.0, size=H.shape[1])
        err = np.zeros(H.shape[1], dtype=np.int64)
        err[rng.choice(H.shape[1], size=rng.integers(1, 4), replace=False)] = 1
        s = ((H.astype(np.int64) @ err) % 2).astype(np.uint8)
        L, e, conv, it = o.bp(H, s, lam, 40, o.params())
        L2, _, conv2, it2 = o.bp(H, s, lam, 40, o.params(early_exit=0))
        assert it2 == 40
        if not conv:
            assert it == 40
            continue
        seen.add(it)
        La, _, ca, ita = o.bp(H, s, lam, it, o.params(early_exit=0))
        assert ca and ita == it and np.array_equal(La, L)
        if it > 1:
            _, _, cb, _ = o.bp(H, s, lam, it - 1, o.params(early_exit=0))
            assert not cb
    assert any(t > 3 for t in seen), seen


# ---------------------------------------------------------------------------
# global BP alone (the single-stage baseline: channel priors, no local phase)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["T", "M"])
def test_global_bp_first_iteration_is_scaled_single_check_min_cost(name):
    """One global min-sum iteration on H_t: L_i = lam_i + beta * sum over the
    checks c of i of the exact min-cost message of check c alone (brute force
    over the check's support), for random syndromes and per-qubit priors."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    rng = np.random.default_rng(5)
    for t in (0, 1):
        H = oc.H(t)
        m, n = H.shape
        s = rng.integers(0, 2, size=(2, m)).astype(np.uint8)
        lam = rng.uniform(-1.0, 4.0, size=(2, n))
        synd = pack_bits(s)
        out = oc.global_bp(synd, lam, t=t, p=o.params(ms_scale=0.75, early_exit=0, max_iter_global=1))
        for shot in range(2):
            want = lam[shot].copy()
            for c in range(m):
                sup = list(np.nonzero(H[c])[0])
                w = len(sup)
                pats = ((np.arange(1 << w)[:, None] >> np.arange(w)) & 1)
                good = (pats.sum(axis=1) % 2) == s[shot, c]
                for k, j in enumerate(sup):
                    others = [q for q in range(w) if q != k]
                    cost = pats[:, others] @ lam[shot, [sup[q] for q in others]]
                    want[j] += 0.75 * (cost[good & (pats[:, k] == 1)].min() - cost[good & (pats[:, k] == 0)].min())
            assert np.allclose(out["post"][shot], np.clip(want, -30, 30), atol=1e-12)
            assert np.array_equal(unpack_bits(out["ehat"][shot:shot + 1], n)[0], (out["post"][shot] < 0).astype(np.uint8))
            assert out["stats"][shot, 1] == 1


@pytest.mark.parametrize("name", ["T", "M"])
def test_global_bp_zero_syndrome_closed_form(name):
    """s = 0 with a uniform prior lam > 0: global BP converges after one
    iteration with L_i = lam (1 + beta d_i), d_i the column weight of H_t."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    lam = float(channel_llr(0.05))
    for t in (0, 1):
        deg = oc.H(t).sum(axis=0)
        s = np.zeros((2, (oc.m(t) + 63) // 64), dtype=np.uint64)
        out = oc.global_bp(s, np.full(2, lam), t=t, p=o.params(ms_scale=0.75, max_iter_global=9))
        assert np.array_equal(out["stats"], [[1, 1], [1, 1]])
        assert np.allclose(out["post"], lam * (1 + 0.75 * deg), rtol=1e-12)
        assert not out["ehat"].any()


@pytest.mark.parametrize("mus", [(30.0, 30.0), (30.0, 25.0, 28.0), (12.0, 30.0, 30.0, 30.0, 29.5), (0.7, 30.0)])
def test_sum_product_message_at_saturation(mus):
    """One check: the sum-product message to a variable equals
    phi(sum phi(|mu|)) over the other edges, phi(x) = log1p(2 / expm1(x)) (the
    tanh rule's log-domain form, well-conditioned in double), to 1e-6 even
    where every |mu| sits at the clamp and 1 - prod tanh(mu/2) ~ 1e-12 (the
    oracle's extended-precision product resolves that distance to ~3e-7
    relative; a double-precision product would miss the message by ~3e-4)."""
    import math
    from oracle import oracle as O

    def phi(x):
        return math.log1p(2.0 / math.expm1(x))

    k = len(mus) + 1
    H = np.ones((1, k), dtype=np.uint8)
    lam = np.array([5.0] + list(mus))
    L, e, conv, it = O.bp(H, np.zeros(1, np.uint8), lam, 1,
                          O.params(bp=O.SUMPRODUCT, llr_clamp=1000.0, early_exit=0))
    want = phi(sum(phi(abs(m)) for m in mus))
    assert abs((L[0] - lam[0]) - want) <= 1e-6, (L[0] - lam[0], want)
