"""OSD-0 after global BP (global_post = 1) on the GPU, against the oracle's
LEAD and global BP with OSD-0 on H_t, and across decode forms."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import (log, torch_dev, gpu_decoder, run_gpu, compare, oracle_decode_conditioned,
                        oracle_global_conditioned, bitflip_inputs)
from lead_inputs import pack_bits, standard, unpack_bits

pytestmark = pytest.mark.gpu

GLOBAL = 2


def _gpu_syndrome(dec, e):
    torch = torch_dev()
    s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint64)


def _check_osd_shots(orc, g, n, H, s):
    """Shots OSD-0 resolved: the same estimate bit for bit on both sides
    (well-conditioned shots), and H e = s for every shot reporting 2."""
    well = ~orc["ill"]
    osd = orc["stats"][:, 0] == 2
    eg, eo = unpack_bits(g["ehat"], n), unpack_bits(orc["ehat"], n)
    assert np.array_equal(eg[well & osd], eo[well & osd])
    sb = unpack_bits(s, H.shape[0])
    done = g["stats"][:, 0] == 2
    assert np.array_equal((eg[done].astype(np.int64) @ H.T) % 2, sb[done])
    return int((well & osd).sum())


@pytest.mark.parametrize("name,t,p,T,bp,min_well", [("T", 0, 0.08, 8, 0, 0.5), ("T", 1, 0.06, 12, 0, 0.5),
                                                    ("M", 0, 0.06, 8, 0, 0.3), ("M", 0, 0.04, 20, 0, 0.3),
                                                    ("M", 0, 0.06, 8, 1, 0.3)])
def test_global_osd_matches_oracle(name, t, p, T, bp, min_well):
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, global_post=1, bp=bp)
    e, s, lam = bitflip_inputs(oc, 160, p, seed=91, t=t)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_decode_conditioned(oc, s, lam, t=t, max_iter_local=T, max_iter_global=T, global_osd=1, bp=bp)
    res = compare(orc, g, oc.n)
    n_osd = _check_osd_shots(orc, g, oc.n, oc.H(t), s)
    well = ~orc["ill"]
    log(f"[global-osd] {name} t={t} p={p} T={T} bp={bp}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"well-conditioned share {well.mean():.2f}, OSD-resolved {int((orc['stats'][:, 0] == 2).sum())} "
        f"({n_osd} well-conditioned), worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert well.mean() >= min_well
    assert n_osd > 0


@pytest.mark.parametrize("name,p,T", [("T", 0.08, 8), ("M", 0.06, 12)])
def test_global_bp_osd_matches_oracle(name, p, T):
    """Stage GLOBAL with global_post: BP-OSD-0 on H_t alone."""
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, max_iter_global=T, stage=GLOBAL, global_post=1)
    e, s, lam = bitflip_inputs(oc, 160, p, seed=93)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0)
    orc = oracle_global_conditioned(oc, s, lam, max_iter_global=T, global_osd=1)
    res = compare(orc, {"post": g["post"], "ehat": g["ehat"], "stats": g["stats"][:, :2]}, oc.n, what=("post",))
    n_osd = _check_osd_shots(orc, g, oc.n, oc.H(0), s)
    log(f"[global-bp-osd] {name} p={p} T={T}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"OSD-resolved {int((orc['stats'][:, 0] == 2).sum())} ({n_osd} well-conditioned)")
    assert not res["unexplained"], res["detail"]
    assert n_osd > 0


def test_global_osd_paths_identical_and_limits():
    """Every kernel form, the fused kernel, outputs left to the decoder's own
    buffers, batches and the unreachable-syndrome case give the same bits;
    unsupported combinations are refused."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=12, max_iter_global=12, global_post=1, max_shots=2048)
    e, _, _ = bitflip_inputs(oc, 400, 0.06, seed=7)
    s = _gpu_syndrome(dec, e)
    rng = np.random.default_rng(3)
    s[:8] = pack_bits((rng.random((8, oc.m())) < 0.3).astype(np.uint8))[:, :s.shape[1]]   # invalid syndromes
    lam = np.full(400, 2.75, dtype=np.float32)
    runs = {}
    for key, sched in (("f2", dict(specialized=2)), ("f1", dict(specialized=1)), ("pre", dict(specialized=0)),
                       ("fused", dict(specialized=0, fused=1)), ("big", dict(specialized=2, global_osd_form=2))):
        dec.set_schedule(**sched)
        assert dec.get_schedule()["global_osd_form"] == (2 if key == "big" else 1)
        runs[key] = run_gpu(dec, s, lam, 0, lam=True)
    ref = runs["f2"]
    assert (ref["stats"][:, 0] == 2).any()
    for key, r in runs.items():
        for k in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(r[k], ref[k]), (key, k)
    # estimate alone: posteriors and statistics kept in the decoder's buffers
    dec.set_schedule(specialized=2)
    st = torch.from_numpy(s.view(np.int64)).cuda()
    pr = torch.from_numpy(lam).cuda()
    out = dec.alloc_outputs(400, post=False)
    out["stats"] = None
    dec.decode(st, pr, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out["ehat"].cpu().numpy().view(np.uint64), ref["ehat"])
    # graph replays of a batch, and the server
    out = dec.alloc_outputs(400, lam=True)
    gb = P.Batch([(dec, st, pr, out, P.LEAD_PRIOR_PER_SHOT)]).capture()
    for _ in range(2):
        out["stats"].zero_()
        gb.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out["ehat"].cpu().numpy().view(np.uint64), ref["ehat"])
        assert np.array_equal(out["stats"].cpu().numpy(), ref["stats"])
    server = P.Server([dec], max_batch_shots=128)
    tk = server.submit(0, s, lam)
    server.wait(tk)
    r = server.result(tk, 0, 400)
    server.close()
    assert np.array_equal(r["ehat"], ref["ehat"]) and np.array_equal(r["stats"], ref["stats"])
    # invalid syndromes keep BP's estimate and report
    _, base = gpu_decoder(spec, max_iter_local=12, max_iter_global=12, max_shots=2048)
    b = run_gpu(base, s, lam, 0, lam=True)
    H = oc.H()
    sb = unpack_bits(s, oc.m())
    from oracle import oracle as o
    for i in range(8):
        if not o.osd0(H, sb[i], np.zeros(oc.n))[1]:
            assert np.array_equal(ref["ehat"][i], b["ehat"][i]) and ref["stats"][i, 0] == b["stats"][i, 0]
    conv = b["stats"][:, 0] == 1
    assert np.array_equal(ref["ehat"][conv], b["ehat"][conv])
    # the plain per-round form on the compiled kernels, global OSD included
    dec.set_schedule(specialized=2)
    pa = dec.decode(st, pr, lam=True, plain=True)
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(pa[k].cpu().numpy().view(ref[k].dtype), ref[k]), k
    # limits
    with pytest.raises(P.LeadError, match="UNSUPPORTED"):
        gpu_decoder(spec, global_post=1, stage=1)
    with pytest.raises(P.LeadError, match="ARG"):
        dec.set_schedule(global_osd_form=3)


@pytest.mark.parametrize("name,t,p,T,order", [("T", 0, 0.08, 8, 3), ("T", 1, 0.06, 12, 3), ("M", 0, 0.06, 8, 3),
                                             ("M", 0, 0.04, 20, 3), ("M", 0, 0.06, 8, 1), ("M", 0, 0.06, 8, 8)])
def test_global_osd_cs_matches_oracle(name, t, p, T, order):
    """Combination sweep of order lambda after global BP (the paper's global
    decoder runs it at order 3), against the oracle."""
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, global_post=1, osd_order=order)
    e, s, lam = bitflip_inputs(oc, 160, p, seed=95, t=t)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_decode_conditioned(oc, s, lam, t=t, max_iter_local=T, max_iter_global=T, global_osd=1,
                                    osd_order=order)
    res = compare(orc, g, oc.n)
    n_osd = _check_osd_shots(orc, g, oc.n, oc.H(t), s)
    # the sweep changes some estimates relative to OSD-0
    o0 = oracle_decode_conditioned(oc, s, lam, t=t, k=0, max_iter_local=T, max_iter_global=T, global_osd=1)
    changed = int((o0["ehat"] != orc["ehat"]).any(axis=1).sum())
    log(f"[global-osd-cs] {name} t={t} p={p} T={T} order={order}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"OSD-resolved {int((orc['stats'][:, 0] == 2).sum())} ({n_osd} well-conditioned), "
        f"{changed} estimates differ from OSD-0")
    assert not res["unexplained"], res["detail"]
    assert n_osd > 0 and changed > 0


def test_global_bp_osd_cs_matches_oracle():
    """Stage GLOBAL: BP followed by OSD-CS of order 3 on H_t alone, costs from
    the channel prior."""
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_global=12, stage=GLOBAL, global_post=1, osd_order=3)
    e, s, lam = bitflip_inputs(oc, 160, 0.06, seed=97)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0)
    orc = oracle_global_conditioned(oc, s, lam, max_iter_global=12, global_osd=1, osd_order=3)
    res = compare(orc, {"post": g["post"], "ehat": g["ehat"], "stats": g["stats"][:, :2]}, oc.n, what=("post",))
    n_osd = _check_osd_shots(orc, g, oc.n, oc.H(0), s)
    log(f"[global-bp-osd-cs] M: {res['bad']} differ, {res['tie']} ill-conditioned, {n_osd} well-conditioned OSD shots")
    assert not res["unexplained"], res["detail"]
    assert n_osd > 0


def test_global_osd_cs_forms_identical_and_limits():
    import paper_2605_17796_amd as P
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=10, max_iter_global=10, global_post=1, osd_order=3, max_shots=1024)
    e, _, _ = bitflip_inputs(oc, 300, 0.06, seed=9)
    s = _gpu_syndrome(dec, e)
    lam = np.full(300, 2.75, dtype=np.float32)
    runs = {}
    for key, sched in (("f2", dict(specialized=2)), ("f1", dict(specialized=1)), ("pre", dict(specialized=0)),
                       ("fused", dict(specialized=0, fused=1)), ("big", dict(specialized=2, global_osd_form=2))):
        dec.set_schedule(**sched)
        runs[key] = run_gpu(dec, s, lam, 0, lam=key != "pre")
    for key, r in runs.items():
        for k in ("ehat", "post", "stats"):
            assert np.array_equal(r[k], runs["f2"][k]), (key, k)
    with pytest.raises(P.LeadError, match="ARG"):
        gpu_decoder(spec, global_post=1, osd_order=9)
    with pytest.raises(P.LeadError, match="ARG"):
        gpu_decoder(spec, osd_order=3)


@pytest.mark.parametrize("name,t,order,stage", [("T", 0, 0, 0), ("T", 1, 3, 0), ("M", 0, 0, 0), ("M", 0, 3, 0),
                                                ("M", 0, 3, GLOBAL), ("M", 1, 8, 0)])
def test_global_osd_matrix_in_memory_identical(name, t, order, stage):
    """The global OSD kernel with [H_t | s] in device memory (persistent
    workgroups, panel elimination) gives the bits of the kernel with the
    rows in registers, for OSD-0 and the combination sweep, in LEAD and after
    global BP alone."""
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=10, max_iter_global=10, global_post=1, osd_order=order,
                            stage=stage, max_shots=1024)
    e, _, _ = bitflip_inputs(oc, 700, 0.06, seed=11, t=t)
    s = _gpu_syndrome(dec, e)
    lam = np.full(700, 2.75, dtype=np.float32)
    dec.set_schedule(global_osd_form=1)
    reg = run_gpu(dec, s, lam, 0, lam=True)
    dec.set_schedule(global_osd_form=2)
    big = run_gpu(dec, s, lam, 0, lam=True)
    n2 = int((reg["stats"][:, 0] == 2).sum())
    log(f"[global-osd-hbm] {name} t={t} order={order} stage={stage}: {n2} of 700 shots resolved by OSD")
    assert n2 > 0
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(reg[k], big[k]), k


@pytest.mark.parametrize("t,order", [(0, 0), (1, 0), (0, 3), (1, 3)])
def test_global_osd_psl27_matches_oracle(t, order):
    """PSL(2,7) (m = 2688, n = 5376): global OSD-0 and OSD-CS of order 3 with
    the matrix in device memory, against the oracle, with caps short enough
    for the shots to stay well-conditioned (3 + 3 rounds, depolarising
    p = 0.03 with the marginal prior 2p/3)."""
    from lead_inputs import channel_llr, depolarizing_packed
    spec, oc = code_pair("L")
    shots, p, T = 24, 0.03, 3
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, global_post=1, osd_order=order,
                            max_shots=shots)
    assert dec.get_schedule()["global_osd_form"] == 2
    xs, zs = depolarizing_packed(shots, oc.n, p, seed=131)
    e = xs if t == 0 else zs
    s = _gpu_syndrome(dec, e)
    assert np.array_equal(s, oc.syndrome(e, t))
    lam = np.full(shots, float(channel_llr(2 * p / 3)), dtype=np.float32)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_decode_conditioned(oc, s, lam, t=t, k=2, max_iter_local=T, max_iter_global=T, global_osd=1,
                                    osd_order=order)
    res = compare(orc, g, oc.n)
    n_osd = _check_osd_shots(orc, g, oc.n, oc.H(t), s)
    log(f"[global-osd] L t={t} order={order}: {res['bad']} differ, {res['tie']} ill-conditioned, OSD-resolved "
        f"{int((orc['stats'][:, 0] == 2).sum())} ({n_osd} well-conditioned), worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert n_osd >= shots // 2
