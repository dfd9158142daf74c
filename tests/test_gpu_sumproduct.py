"""Sum-product BP (both stages, log-domain check update on the kernels
compiled for the code) against the oracle's sum-product LEAD, and its
limits."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import (log, torch_dev, gpu_decoder, run_gpu, compare, oracle_decode_conditioned, bitflip_inputs)
from lead_inputs import channel_llr, uniform_p

pytestmark = pytest.mark.gpu

SP = 1


def _gpu_syndrome(dec, e):
    torch = torch_dev()
    s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name,t,p,T,alpha,min_well", [("T", 0, 0.05, 32, 1.0, 0.6), ("T", 1, 0.03, 32, 0.5, 0.6),
                                                       ("M", 0, 0.02, 50, 1.0, 0.4), ("M", 0, 0.05, 8, 1.0, 0.4),
                                                       ("M", 1, 0.01, 50, 0.1, 0.2)])
def test_sum_product_matches_oracle(name, t, p, T, alpha, min_well):
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, alpha=alpha, bp=SP)
    assert dec.get_schedule()["specialized"] == 3
    e, s, lam = bitflip_inputs(oc, 160, p, seed=71, t=t)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_decode_conditioned(oc, s, lam, t=t, max_iter_local=T, max_iter_global=T, alpha=alpha, bp=SP)
    res = compare(orc, g, oc.n)
    well = 1 - orc["ill"].mean()
    log(f"[sum-product] {name} t={t} p={p} T={T} alpha={alpha}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"well-conditioned share {well:.2f}, worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert well >= min_well


@pytest.mark.parametrize("name,p,T", [("T", 0.05, 32), ("M", 0.05, 50)])
def test_sum_product_fixed_point_variants_equal(name, p, T):
    """The fixed-point exit on both stages (1), on local runs only (2: the
    Phases 2-3 kernel compiled without the comparison) and off (0) give the
    same outputs bit for bit; only the fixed-point statistics differ."""
    torch = torch_dev()
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, max_iter_local=T, max_iter_global=T, bp=SP, fixed_point_stop=1)
    e, _, lamv = bitflip_inputs(oc, 400, p, seed=83)
    s = torch.from_numpy(_gpu_syndrome(dec, e).view(np.int64)).cuda()
    lam = torch.from_numpy(lamv).cuda()
    runs = {}
    for fp in (1, 2, 0):
        dec.set_params(max_iter_local=T, max_iter_global=T, bp=SP, fixed_point_stop=fp)
        runs[fp] = dec.decode(s, lam, lam=True)
    torch.cuda.synchronize()
    for fp in (2, 0):
        for k in ("ehat", "post", "lam"):
            assert torch.equal(runs[fp][k], runs[1][k]), (fp, k)
        assert torch.equal(runs[fp]["stats"][:, :5], runs[1]["stats"][:, :5]), fp
    assert torch.equal(runs[2]["stats"][:, 5], runs[1]["stats"][:, 5])
    assert int(runs[2]["stats"][:, 6].abs().sum()) == 0 and int(runs[0]["stats"][:, 5:7].abs().sum()) == 0
    st = runs[1]["stats"].cpu().numpy()
    log(f"[sum-product] {name} p={p}: fixed_point_stop 1/2/0 bit-identical; shots with a global fixed point "
        f"{(st[:, 6] > 0).mean():.3f}")


def test_sum_product_batched_and_served_equal_alone():
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=50, max_iter_global=50, bp=SP, max_shots=4096)
    ps = uniform_p(300, 0.02, 0.08, 4)
    e, _, _ = bitflip_inputs(oc, 300, 0.05, seed=4)
    s = torch.from_numpy(_gpu_syndrome(dec, e).view(np.int64)).cuda()
    pr = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
    a = dec.decode(s, pr, lam=True)
    out = dec.alloc_outputs(300, lam=True)
    g = P.Batch([(dec, s, pr, out, P.LEAD_PRIOR_PER_SHOT)]).capture()
    g.replay()
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(a[k], out[k]), k
    server = P.Server([dec], max_batch_shots=128)
    tk = server.submit(0, s.cpu().numpy().view(np.uint64), pr.cpu().numpy())
    server.wait(tk)
    r = server.result(tk, 0, 300)
    server.close()
    assert np.array_equal(r["ehat"], a["ehat"].cpu().numpy().view(np.uint64))
    assert np.array_equal(r["stats"], a["stats"].cpu().numpy())


@pytest.mark.parametrize("name,p,T", [("T", 0.05, 10), ("M", 0.03, 12)])
def test_sum_product_global_only_matches_oracle(name, p, T):
    """Sum-product global BP alone (stage GLOBAL, channel priors), at caps
    short enough that FP32 rounding is not amplified beyond the tolerance on
    shots that do not converge (global BP alone leaves many of them)."""
    from gpu_common import oracle_global_conditioned
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, max_iter_global=T, stage=2, bp=SP)
    e, s, lam = bitflip_inputs(oc, 200, p, seed=73)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0, lam=True)
    assert np.array_equal(g["lam"], np.broadcast_to(lam[:, None], g["lam"].shape))
    orc = oracle_global_conditioned(oc, s, lam, max_iter_global=T, bp=SP)
    res = compare(orc, {"post": g["post"], "ehat": g["ehat"], "stats": g["stats"][:, :2]}, oc.n, what=("post",))
    log(f"[sum-product global-only] {name} p={p} T={T}: {res['bad']} differ, {res['tie']} ill-conditioned")
    assert not res["unexplained"], res["detail"]
    assert res["tie"] <= 0.6 * res["shots"]


@pytest.mark.parametrize("t,T,shots,min_well", [(0, 4, 48, 0.9), (1, 4, 48, 0.7), (0, 10, 96, 0.15)])
def test_sum_product_psl27_matches_oracle(t, T, shots, min_well):
    """Sum-product LEAD on the PSL(2,7) views (156 edges on the Z checks,
    182 on the X checks: one register per message, one wave per SIMD),
    depolarising p = 0.03 with the marginal prior 2p/3, against the oracle.
    At 10 + 10 rounds most shots are no longer determined to the tolerance
    by FP32-sized rounding (the share is reported; every well-conditioned
    shot must match)."""
    from lead_inputs import depolarizing_packed
    spec, oc = code_pair("L")
    p = 0.03
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, bp=SP, max_shots=shots)
    assert dec.get_schedule()["specialized"] == 3
    xs, zs = depolarizing_packed(shots, oc.n, p, seed=137)
    e = xs if t == 0 else zs
    s = _gpu_syndrome(dec, e)
    lam = np.full(shots, float(channel_llr(2 * p / 3)), dtype=np.float32)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_decode_conditioned(oc, s, lam, t=t, max_iter_local=T, max_iter_global=T, bp=SP)
    res = compare(orc, g, oc.n)
    well = 1 - orc["ill"].mean()
    conv = float((orc["stats"][:, 0] == 1).mean())
    log(f"[sum-product] L t={t} p={p} T={T}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"well-conditioned share {well:.2f}, converged {conv:.2f}, worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert well >= min_well


def test_sum_product_plain_form_and_flavour_switch():
    """The plain per-round form runs sum-product on its compiled round
    kernel (bit-identical to lead_decode); the precompiled kernels have no
    sum-product, so schedules keep the compiled form."""
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, bp=SP, max_iter_local=20, max_iter_global=20)
    e, s, lamv = bitflip_inputs(oc, 200, 0.06, seed=5)
    s = torch.from_numpy(_gpu_syndrome(dec, e).view(np.int64)).cuda()
    lam = torch.from_numpy(lamv).cuda()
    a = dec.decode(s, lam, lam=True)
    b = dec.decode(s, lam, lam=True, plain=True)
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(a[k], b[k]), k
    dec.set_schedule(specialized=0, fused=1)
    assert dec.get_schedule()["specialized"] == 3 and dec.get_schedule()["fused"] == 0
    # switching flavours on a live decoder
    dec.set_params(bp=0)
    assert dec.get_schedule()["specialized"] in (1, 2)
    dec.set_params(bp=SP)
    assert dec.get_schedule()["specialized"] == 3
