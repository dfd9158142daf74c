"""Pins of the oracle's local post-processing (OSD-0 on the views whose local
BP run did not reach H_v e_v = s_v; the paper's BP-LSD family of local
decoders): brute force over the information set, the stopping structure
inside LEAD, and the confidence boost it makes live."""
import numpy as np
import pytest

from conftest import code_pair
from lead_inputs import bitflip_packed, channel_llr


def _gf2_rank(rows):
    rows = [int(r) for r in rows if r]
    rank = 0
    while rows:
        piv = max(rows)
        top = piv.bit_length() - 1
        rows = [r ^ piv if (r >> top) & 1 else r for r in rows if r != piv]
        rows = [r for r in rows if r]
        rank += 1
    return rank


def _col_ints(H):
    return [int(sum(int(H[i, j]) << i for i in range(H.shape[0]))) for j in range(H.shape[1])]


def brute_osd0(H, s, L):
    """Information set = the first columns, in order of round(64 L)
    ascending (ties by position), that raise the GF(2) rank; the estimate is
    the one pattern on the information set whose syndrome is s (enumerated)."""
    cols = _col_ints(H)
    order = sorted(range(H.shape[1]), key=lambda j: (np.rint(64.0 * L[j]), j))
    info, chosen = [], []
    for j in order:
        if _gf2_rank(chosen + [cols[j]]) > len(chosen):
            chosen.append(cols[j])
            info.append(j)
    target = int(sum(int(s[i]) << i for i in range(H.shape[0])))
    sols = []
    for mask in range(1 << len(info)):
        acc = 0
        for b, j in enumerate(info):
            if (mask >> b) & 1:
                acc ^= cols[j]
        if acc == target:
            e = np.zeros(H.shape[1], dtype=np.uint8)
            for b, j in enumerate(info):
                e[j] = (mask >> b) & 1
            sols.append(e)
    return sols


@pytest.mark.parametrize("name", ["appendix", "T", "M"])
def test_osd0_is_the_information_set_solution(name):
    from oracle import oracle as o
    _, oc = code_pair(name)
    rng = np.random.default_rng(11)
    for t in (0, 1):
        H = oc.hloc(t)
        for trial in range(12):
            s = rng.integers(0, 2, size=H.shape[0]).astype(np.uint8)
            # reliabilities with ties (saturated values, equal keys) and distinct values
            L = np.round(rng.uniform(-3, 3, size=H.shape[1]), 1 if trial % 2 else 6)
            L[rng.random(H.shape[1]) < 0.2] = 30.0
            e, ok = o.osd0(H, s, L)
            sols = brute_osd0(H, s, L)
            assert ok and len(sols) == 1
            assert np.array_equal(e, sols[0])
            assert np.array_equal((H.astype(int) @ e) % 2, s)


def test_osd0_reports_unreachable_syndrome():
    from oracle import oracle as o
    H = np.array([[1, 1, 0], [1, 1, 0]], dtype=np.uint8)     # rank 1
    e, ok = o.osd0(H, np.array([1, 0], dtype=np.uint8), np.zeros(3))
    assert not ok and not e.any()


@pytest.mark.parametrize("name", ["T", "M"])
def test_local_osd_in_lead(name):
    """With OSD-0 every view ends with a local estimate: views BP resolved plus
    views OSD resolved = all views; shots whose views all converged under BP
    decode exactly as without OSD; elsewhere the boost can only lower the
    local LLRs it touches, so the regularised priors lambda' do not rise."""
    from oracle import oracle as o
    spec, oc = code_pair(name)
    T = {"T": 32, "M": 50}[name]
    shots = 40
    e = bitflip_packed(shots, oc.n, 0.05, seed=23)
    s = oc.syndrome(e)
    lam = np.full(shots, float(channel_llr(0.05)))
    base = oc.decode(s, lam, p=o.params(max_iter_local=T, max_iter_global=T))
    osd = oc.decode(s, lam, p=o.params(max_iter_local=T, max_iter_global=T, local_osd=1))
    N = spec.order
    assert np.array_equal(osd["stats"][:, 4] + osd["osd_views"], np.full(shots, N))
    assert np.array_equal(osd["stats"][:, 2:5], base["stats"][:, 2:5])   # BP runs unchanged
    same = osd["osd_views"] == 0
    assert (~same).any()
    if name == "T":
        assert same.any()
    for k in ("post", "lam"):
        assert np.array_equal(osd[k][same], base[k][same])
    assert np.all(osd["lam"] <= base["lam"] + 1e-12)
    assert np.any(osd["lam"] < base["lam"] - 1e-6)


def _greedy_information_set(H, L):
    """Columns in order of round(64 L) ascending (ties by position) that
    raise the GF(2) rank, with an incremental basis keyed by lowest set bit."""
    cols = _col_ints(H)
    order = sorted(range(H.shape[1]), key=lambda j: (np.rint(64.0 * L[j]), j))
    basis, info = {}, []
    for j in order:
        v = cols[j]
        while v:
            low = v & -v
            if low in basis:
                v ^= basis[low]
            else:
                basis[low] = v
                info.append(j)
                break
    return set(info)


@pytest.mark.parametrize("name", ["T", "M"])
def test_osd0_on_the_global_matrix(name):
    """OSD-0 on H_t (rank below the row count): the estimate reproduces the
    syndrome and lies on the greedy information set, where the solution is
    unique because those columns are independent."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    rng = np.random.default_rng(13)
    for t in (0, 1):
        H = oc.H(t)
        for trial in range(3):
            e0 = (rng.random(H.shape[1]) < 0.05).astype(np.uint8)
            s = (H.astype(np.int64) @ e0 % 2).astype(np.uint8)
            L = rng.uniform(-2, 5, size=H.shape[1])
            L[rng.random(H.shape[1]) < 0.3] = 30.0
            e, ok = o.osd0(H, s, L)
            assert ok
            assert np.array_equal((H.astype(np.int64) @ e) % 2, s)
            info = _greedy_information_set(H, L)
            assert set(np.nonzero(e)[0]) <= info
            assert len(info) == oc.info.rank[t]


@pytest.mark.parametrize("name", ["T", "M"])
def test_global_osd_in_lead(name):
    """With OSD-0 after global BP every shot ends with H e = s: shots global BP
    resolved are unchanged, the others report converged = 2."""
    from oracle import oracle as o
    spec, oc = code_pair(name)
    T = {"T": 32, "M": 50}[name]
    shots = 30
    e = bitflip_packed(shots, oc.n, 0.05, seed=29)
    s = oc.syndrome(e)
    lam = np.full(shots, float(channel_llr(0.05)))
    base = oc.decode(s, lam, p=o.params(max_iter_local=T, max_iter_global=T))
    gosd = oc.decode(s, lam, p=o.params(max_iter_local=T, max_iter_global=T, global_osd=1))
    conv = base["stats"][:, 0] == 1
    assert np.array_equal(gosd["stats"][conv, 0], base["stats"][conv, 0])
    assert np.all(gosd["stats"][~conv, 0] == 2) and (~conv).any()
    assert np.array_equal(gosd["ehat"][conv], base["ehat"][conv])
    assert np.array_equal(gosd["post"], base["post"])
    H = oc.H()
    from lead_inputs import unpack_bits
    eh = unpack_bits(gosd["ehat"], oc.n)
    sb = unpack_bits(s, oc.m())
    assert np.array_equal((eh.astype(np.int64) @ H.T) % 2, sb)


@pytest.mark.parametrize("name", ["T", "M"])
def test_global_osd_keeps_bp_on_unreachable_syndromes(name):
    """A syndrome outside the column space of H_t (random bits, rank < m) has
    no OSD-0 solution: the estimate and the stopping report stay BP's."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    rng = np.random.default_rng(31)
    shots = 6
    H = oc.H()
    sb = (rng.random((shots, H.shape[0])) < 0.3).astype(np.uint8)
    from lead_inputs import pack_bits
    s = pack_bits(sb)
    lam = np.full(shots, float(channel_llr(0.05)))
    base = oc.decode(s, lam, p=o.params(max_iter_local=10, max_iter_global=10))
    gosd = oc.decode(s, lam, p=o.params(max_iter_local=10, max_iter_global=10, global_osd=1))
    unreach = np.array([not o.osd0(H, sb[i], np.zeros(H.shape[1]))[1] for i in range(shots)])
    assert unreach.sum() >= shots // 2
    assert np.all(base["stats"][unreach, 0] == 0)
    assert np.array_equal(gosd["stats"][unreach], base["stats"][unreach])
    assert np.array_equal(gosd["ehat"][unreach], base["ehat"][unreach])


@pytest.mark.parametrize("name", ["T", "M"])
def test_global_bp_then_osd(name):
    """BP-OSD-0 on H_t alone: shots BP resolves are untouched; the others
    take the OSD-0 solution of H_t e = s ranked by BP's posteriors."""
    from oracle import oracle as o
    from lead_inputs import unpack_bits
    _, oc = code_pair(name)
    shots = 24
    e = bitflip_packed(shots, oc.n, 0.06, seed=37)
    s = oc.syndrome(e)
    lam = np.full(shots, float(channel_llr(0.06)))
    base = oc.global_bp(s, lam, p=o.params(max_iter_global=12))
    gosd = oc.global_bp(s, lam, p=o.params(max_iter_global=12, global_osd=1))
    conv = base["stats"][:, 0] == 1
    assert (~conv).any()
    assert np.array_equal(gosd["ehat"][conv], base["ehat"][conv])
    assert np.all(gosd["stats"][~conv, 0] == 2)
    assert np.array_equal(gosd["post"], base["post"])
    H = oc.H()
    sb = unpack_bits(s, oc.m())
    eh = unpack_bits(gosd["ehat"], oc.n)
    for i in np.nonzero(~conv)[0]:
        ref, ok = o.osd0(H, sb[i], base["post"][i])
        assert ok and np.array_equal(eh[i], ref)


def test_osd_weight_closed_form():
    """The sweep's cost of a bit is round(64 ln(1/p)) with p = 1/(1 + e^lam)."""
    import math
    from oracle import oracle as o
    for lam in (-30.0, -7.25, -1.0, -1e-9, 0.0, 0.3, 2.944438979, 9.5, 30.0):
        p = 1.0 / (1.0 + math.exp(lam))
        assert o.osd_weight(lam) == int(np.rint(64.0 * -math.log(p)))


def _sweep_by_brute_force(H, s, L, prior, order):
    """The combination sweep from its definition: information set S and the
    other columns T in rank order; candidate supports e_T = {}, {t} for every
    t in T, {a, b} for pairs among the first `order` columns of T; each
    completed on S by enumerating every pattern on S; the first candidate of
    least total cost wins."""
    from oracle import oracle as o
    rows, ncol = H.shape
    cols = _col_ints(H)
    ranked = sorted(range(ncol), key=lambda j: (np.rint(64.0 * L[j]), j))
    info = _greedy_information_set(H, L)
    S = [j for j in ranked if j in info]
    T = [j for j in ranked if j not in info]
    target = int(sum(int(s[i]) << i for i in range(rows)))
    w = [o.osd_weight(prior[j]) for j in range(ncol)]
    cands = [()] + [(t,) for t in T]
    lam = min(order, len(T))
    cands += [(T[x], T[y]) for x in range(lam) for y in range(x + 1, lam)]
    best, best_e = None, None
    for sup in cands:
        acc = target
        for t in sup:
            acc ^= cols[t]
        sol = None
        for mask in range(1 << len(S)):
            v = 0
            for b, j in enumerate(S):
                if (mask >> b) & 1:
                    v ^= cols[j]
            if v == acc:
                sol = mask
                break
        assert sol is not None
        e = np.zeros(ncol, dtype=np.uint8)
        for b, j in enumerate(S):
            e[j] = (sol >> b) & 1
        for t in sup:
            e[t] = 1
        c = sum(w[j] for j in range(ncol) if e[j])
        if best is None or c < best:
            best, best_e = c, e
    return best_e, best


@pytest.mark.parametrize("name", ["appendix", "T", "M"])
@pytest.mark.parametrize("order", [1, 3, 5])
def test_osd_cs_is_the_cheapest_candidate(name, order):
    """Combination sweep against brute force over its candidate set, on the
    local check matrices (rank below the number of columns)."""
    from oracle import oracle as o
    _, oc = code_pair(name)
    rng = np.random.default_rng(17 + order)
    for t in (0, 1):
        H = oc.hloc(t)
        if np.linalg.matrix_rank(H) > 14:
            continue
        for trial in range(4):
            e0 = (rng.random(H.shape[1]) < 0.2).astype(np.uint8)
            s = (H.astype(np.int64) @ e0 % 2).astype(np.uint8)
            L = rng.uniform(-3, 6, size=H.shape[1])
            prior = rng.uniform(-1, 5, size=H.shape[1])
            e, ok = o.osd(H, s, L, prior=prior, order=order)
            assert ok
            ref, _ = _sweep_by_brute_force(H, s, L, prior, order)
            assert np.array_equal(e, ref)
            e0_, _ = o.osd(H, s, L, order=0)
            assert np.array_equal(e0_, o.osd0(H, s, L)[0])
            c = lambda x: sum(o.osd_weight(prior[j]) for j in np.nonzero(x)[0])
            assert c(e) <= c(e0_)


@pytest.mark.parametrize("name", ["T", "M"])
def test_osd_cs_on_random_sparse_matrices(name):
    """Small random sparse matrices with dependent rows and columns: the sweep
    equals brute force and reproduces the syndrome."""
    from oracle import oracle as o
    rng = np.random.default_rng(101 if name == "T" else 202)
    for trial in range(12):
        rows, ncol = int(rng.integers(6, 11)), int(rng.integers(10, 17))
        H = (rng.random((rows, ncol)) < 0.3).astype(np.uint8)
        H[-1] = H[0] ^ H[1]
        e0 = (rng.random(ncol) < 0.25).astype(np.uint8)
        s = (H.astype(np.int64) @ e0 % 2).astype(np.uint8)
        L = np.round(rng.uniform(-2, 4, size=ncol) * 4) / 4   # exact ties included
        prior = rng.uniform(0, 4, size=ncol)
        for order in (0, 2, 3):
            e, ok = o.osd(H, s, L, prior=prior, order=order)
            assert ok and np.array_equal((H.astype(np.int64) @ e) % 2, s)
            if order:
                assert np.array_equal(e, _sweep_by_brute_force(H, s, L, prior, order)[0])


@pytest.mark.parametrize("name", ["T", "M"])
def test_global_osd_cs_in_lead(name):
    """LEAD with OSD-CS of order 3 after global BP: every unresolved shot takes
    the sweep's estimate on the global posteriors with lambda' as the prior,
    never costlier than OSD-0's; resolved shots are untouched."""
    from oracle import oracle as o
    from lead_inputs import unpack_bits
    _, oc = code_pair(name)
    T = {"T": 16, "M": 12}[name]
    shots = 16
    e = bitflip_packed(shots, oc.n, 0.06, seed=41)
    s = oc.syndrome(e)
    lam = np.full(shots, float(channel_llr(0.06)))
    kw = dict(max_iter_local=T, max_iter_global=T, global_osd=1)
    o0 = oc.decode(s, lam, p=o.params(**kw))
    o3 = oc.decode(s, lam, p=o.params(osd_order=3, **kw))
    assert np.array_equal(o3["post"], o0["post"]) and np.array_equal(o3["lam"], o0["lam"])
    assert np.array_equal(o3["stats"], o0["stats"])
    H = oc.H()
    sb = unpack_bits(s, oc.m())
    e3, e0 = unpack_bits(o3["ehat"], oc.n), unpack_bits(o0["ehat"], oc.n)
    res = o0["stats"][:, 0] == 2
    assert res.any()
    assert np.array_equal(e3[~res], e0[~res])
    for i in np.nonzero(res)[0]:
        ref, ok = o.osd(H, sb[i], o0["post"][i], prior=o0["lam"][i], order=3)
        assert ok and np.array_equal(e3[i], ref)
        c = lambda x: sum(o.osd_weight(o0["lam"][i][j]) for j in np.nonzero(x)[0])
        assert c(e3[i]) <= c(e0[i])


@pytest.mark.parametrize("order", [0, 3])
def test_local_osd_cs_in_lead(order):
    """LEAD's local post-processing at order lambda, rebuilt view by view from
    the oracle's own local posteriors: OSD with the view's channel priors as
    costs on every view whose BP missed its syndrome, the confidence boost on
    its errors, then the two-view aggregation of Algorithm 1 Phase 2."""
    from oracle import oracle as o
    from lead_inputs import unpack_bits
    _, oc = code_pair("T")
    shots, T = 12, 16
    e = bitflip_packed(shots, oc.n, 0.06, seed=43)
    s = oc.syndrome(e)
    lam = np.full(shots, float(channel_llr(0.06)))
    res = oc.decode(s, lam, p=o.params(max_iter_local=T, max_iter_global=T, local_osd=1, osd_order=order),
                    want_local=True)
    H = oc.hloc()
    view = oc.views()
    r, D2 = H.shape
    sb = unpack_bits(s, oc.m())
    n_osd = 0
    for i in range(shots):
        pv = np.zeros(view.shape)
        for v in range(view.shape[0]):
            sv = sb[i, v * r:(v + 1) * r]
            Lv = res["local"][i, v]
            ev = (Lv < 0).astype(np.uint8)
            conv = np.array_equal((H.astype(np.int64) @ ev) % 2, sv)
            p = 1.0 / (1.0 + np.exp(Lv))
            if not conv:
                eo, ok = o.osd(H, sv, Lv, prior=np.full(D2, lam[i]), order=order)
                if ok:
                    n_osd += 1
                    p = np.where(eo == 1, np.maximum(p, 0.5), p)
            pv[v] = p
        phat = np.zeros(oc.n)
        np.add.at(phat, view.ravel(), pv.ravel())
        phat = phat / 2.0
        ref = np.clip(np.log(1.0 - phat) - np.log(phat), -30.0, 30.0)
        assert np.allclose(res["lam"][i], ref, rtol=0, atol=1e-9)
    assert n_osd > 0
