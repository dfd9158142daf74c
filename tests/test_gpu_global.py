"""Global BP alone (stage GLOBAL: the channel priors are the prior of the
global BP and there is no local phase; the single-stage decoder LEAD is
compared against) matches the oracle's global BP, and every decode form
gives the same bits."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import (log, torch_dev, gpu_decoder, run_gpu, compare, oracle_global_conditioned,
                        bitflip_inputs)
from lead_inputs import channel_llr, uniform_p

pytestmark = pytest.mark.gpu

GLOBAL = 2


def _gpu_syndrome(dec, e):
    torch = torch_dev()
    s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name,t,p,T,min_well", [("T", 0, 0.05, 32, 0.6), ("T", 1, 0.03, 32, 0.6),
                                                 ("M", 0, 0.05, 8, 0.5), ("M", 0, 0.02, 50, 0.5)])
def test_global_only_matches_oracle(name, t, p, T, min_well):
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_global=T, stage=GLOBAL)
    e, s, lam = bitflip_inputs(oc, 200, p, seed=61, t=t)
    s = _gpu_syndrome(dec, e)
    g = run_gpu(dec, s, lam, 0, lam=True)
    orc = oracle_global_conditioned(oc, s, lam, t=t, max_iter_global=T)
    # lambda' of the GLOBAL stage is the channel prior itself
    assert np.array_equal(g["lam"], np.broadcast_to(lam[:, None], g["lam"].shape))
    res = compare(orc, {"post": g["post"], "ehat": g["ehat"], "stats": g["stats"][:, :2]}, oc.n,
                  what=("post",))
    well = 1 - orc["ill"].mean()
    log(f"[global-only] {name} t={t} p={p} T={T}: {res['bad']} differ, {res['tie']} ill-conditioned, "
        f"well-conditioned share {well:.2f}, worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert well >= min_well
    # local statistics are zero: there is no local phase
    assert not g["stats"][:, 2:6].any()


def test_global_only_forms_identical():
    """Plain per-round launches, batched graph replay and the default call give
    the same bits in the GLOBAL stage."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_global=50, stage=GLOBAL, max_shots=4096)
    ps = uniform_p(500, 0.02, 0.08, 3)
    e, _, _ = bitflip_inputs(oc, 500, 0.05, seed=3)
    s = torch.from_numpy(_gpu_syndrome(dec, e).view(np.int64)).cuda()
    pr = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
    a = dec.decode(s, pr, lam=True)
    b = dec.decode(s, pr, lam=True, plain=True)
    out = dec.alloc_outputs(500, lam=True)
    g = P.Batch([(dec, s, pr, out, P.LEAD_PRIOR_PER_SHOT)]).capture()
    g.replay()
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(a[k], out[k]), k


@pytest.mark.parametrize("name,mode", [("T", 0), ("M", 0), ("M", 1), ("M", 2), ("L", 0)])
def test_global_only_specialised_equals_fused(name, mode):
    """Stage GLOBAL on the per-shot kernel compiled for the code (both check
    state forms) and on the fused precompiled kernel: the same bits, for every
    prior mode."""
    spec, oc = code_pair(name)
    T = {"T": 32, "M": 50, "L": 20}[name]
    shots = {"T": 700, "M": 300, "L": 40}[name]
    code, dec = gpu_decoder(spec, max_iter_global=T, stage=GLOBAL, max_shots=1024)
    e, _, _ = bitflip_inputs(oc, shots, 0.04, seed=5 + mode)
    s = _gpu_syndrome(dec, e)
    rng = np.random.default_rng(mode)
    prior = {0: channel_llr(uniform_p(shots, 0.02, 0.06, 8)).astype(np.float32),
             1: channel_llr(rng.uniform(0.02, 0.06, oc.n)).astype(np.float32),
             2: channel_llr(rng.uniform(0.02, 0.06, (shots, oc.n))).astype(np.float32)}[mode]
    runs = {}
    for key, sched in (("f2", dict(specialized=2)), ("f1", dict(specialized=1)), ("fused", dict(specialized=0, fused=1))):
        dec.set_schedule(**sched)
        runs[key] = run_gpu(dec, s, prior, mode, lam=True)
    for key in ("f1", "fused"):
        for k in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(runs["f2"][k], runs[key][k]), (key, k)
    log(f"[global-only forms] {name} mode={mode}: {shots} shots identical, converged "
        f"{runs['f2']['stats'][:, 0].mean():.3f}")
