"""OSD-0 local post-processing (local_post = 1) on the kernels compiled for
the code, against the oracle's LEAD with OSD-0, and across kernel forms."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import (log, torch_dev, gpu_decoder, run_gpu, compare, oracle_decode_conditioned, bitflip_inputs)

pytestmark = pytest.mark.gpu


def _gpu_syndrome(dec, e):
    torch = torch_dev()
    s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name,t,p,T,bp,min_well", [("T", 0, 0.05, 32, 0, 0.6), ("T", 1, 0.03, 32, 0, 0.6),
                                                    ("M", 0, 0.02, 50, 0, 0.3), ("M", 0, 0.05, 8, 0, 0.3),
                                                    ("T", 0, 0.05, 32, 1, 0.6), ("M", 0, 0.02, 50, 1, 0.3)])
def test_local_osd_matches_oracle(name, t, p, T, bp, min_well):
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, local_post=1, bp=bp)
    e, s, lam = bitflip_inputs(oc, 160, p, seed=81, t=t)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_decode_conditioned(oc, s, lam, t=t, max_iter_local=T, max_iter_global=T, local_osd=1, bp=bp)
    res = compare(orc, g, oc.n)
    well = ~orc["ill"]
    assert np.array_equal(g["stats"][well, 7], orc["osd_views"][well])
    log(f"[osd] {name} t={t} p={p} T={T} bp={bp}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"well-conditioned share {well.mean():.2f}, OSD views per shot {orc['osd_views'].mean():.1f}, "
        f"worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert well.mean() >= min_well


def test_local_osd_forms_identical_and_limits():
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=50, max_iter_global=50, local_post=1, max_shots=2048)
    e, s, lam = bitflip_inputs(oc, 400, 0.05, seed=5)
    s = _gpu_syndrome(dec, e)
    runs = {}
    for form in (2, 1):
        dec.set_schedule(specialized=form)
        assert dec.get_schedule()["specialized"] == form
        runs[form] = run_gpu(dec, s, lam, 0, lam=True)
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(runs[1][k], runs[2][k]), k
    # the precompiled kernels have no OSD-0: schedules keep the compiled form
    dec.set_schedule(specialized=0, fused=1)
    sc = dec.get_schedule()
    assert sc["fused"] == 0 and sc["specialized"] in (1, 2)
    st = torch.from_numpy(s.view(np.int64)).cuda()
    pr = torch.from_numpy(lam).cuda()
    # the plain per-round form runs the compiled kernels, local OSD included
    pa = dec.decode(st, pr, lam=True, plain=True)
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(pa[k].cpu().numpy().view(runs[2][k].dtype), runs[2][k]), k
    with pytest.raises(P.LeadError, match="UNSUPPORTED"):
        gpu_decoder(spec, local_post=1, stage=2)


@pytest.mark.parametrize("name,t,p,T,order,mode", [("T", 0, 0.05, 32, 3, 0), ("M", 0, 0.05, 8, 3, 0),
                                                  ("M", 0, 0.02, 50, 8, 0), ("T", 1, 0.05, 16, 3, 2)])
def test_local_osd_cs_matches_oracle(name, t, p, T, order, mode):
    """Local OSD with the combination sweep (costs from the view's channel
    priors), per-shot and per-qubit priors, against the oracle."""
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, local_post=1, osd_order=order)
    e, s, lam = bitflip_inputs(oc, 160, p, seed=83, t=t)
    s = _gpu_syndrome(dec, e)
    prior = lam
    if mode == 2:
        rng = np.random.default_rng(5)
        prior = np.log(1 / rng.uniform(0.02, 0.08, (160, oc.n)) - 1).astype(np.float32)
    g = run_gpu(dec, s, prior, mode, lam=True)
    orc = oracle_decode_conditioned(oc, s, prior.astype(np.float64), t=t, max_iter_local=T, max_iter_global=T,
                                    local_osd=1, osd_order=order)
    o0 = oracle_decode_conditioned(oc, s, prior.astype(np.float64), t=t, k=0, max_iter_local=T, max_iter_global=T,
                                   local_osd=1)
    res = compare(orc, g, oc.n)
    well = ~orc["ill"]
    assert np.array_equal(g["stats"][well, 7], orc["osd_views"][well])
    changed = int((np.abs(o0["lam"] - orc["lam"]).max(axis=1) > 0).sum())
    log(f"[osd-cs local] {name} t={t} p={p} T={T} order={order} mode={mode}: {res['bad']} differ, "
        f"{res['tie']} ill-conditioned, {changed} shots whose lambda' the sweep changes")
    assert not res["unexplained"], res["detail"]
    assert well.mean() >= 0.3 and changed > 0


def test_local_and_global_osd_cs_forms_identical():
    """Local and global OSD with the sweep together: every kernel form gives
    the same bits."""
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=12, max_iter_global=12, local_post=1, global_post=1, osd_order=3,
                            max_shots=1024)
    e, _, _ = bitflip_inputs(oc, 300, 0.05, seed=13)
    s = _gpu_syndrome(dec, e)
    lam = np.full(300, 2.94, dtype=np.float32)
    runs = {}
    for form in (2, 1):
        dec.set_schedule(specialized=form)
        runs[form] = run_gpu(dec, s, lam, 0, lam=True)
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(runs[1][k], runs[2][k]), k
    assert (runs[2]["stats"][:, 0] == 2).any() and runs[2]["stats"][:, 7].sum() > 0
