"""The persistent Phases 2-3 kernel for codes whose views span several waves
(lead_schedule.global_tiles = 1: workgroups of 512 lanes holding three
PSL(2,7) shots, each slot taking the next shot from a device counter when its
shot ends) against the per-shot kernel (global_tiles = 2): the same outputs
bit for bit -- e_hat, L_post, lambda' and every statistic -- for both check
types, both min-sum forms, the two prior modes and stage GLOBAL, on batch
sizes that leave slots and workgroups empty (1, 2 shots), fill one round of
slots (768 on 256 compute units) and need refills (2000 shots)."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder
from lead_inputs import bitflip_packed, channel_llr, uniform_p

pytestmark = pytest.mark.gpu


def _decode(dec, synd, prior, mode, tiles, form):
    torch = torch_dev()
    dec.set_schedule(specialized=form, global_tiles=tiles)
    sc = dec.get_schedule()
    assert sc["specialized"] == form and sc["global_tiles"] == tiles, sc
    out = dec.decode(synd, prior, mode=mode, lam=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("t,form", [(0, 2), (0, 1), (1, 2), (1, 1)])
def test_tiles_equal_per_shot_kernel(t, form):
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("L")
    shots_max = 2000
    code, dec = gpu_decoder(spec, t=t, max_iter_local=24, max_iter_global=24, max_shots=shots_max)
    ps = uniform_p(shots_max, 0.01, 0.05, 40 + t)
    e = bitflip_packed(shots_max, oc.n, ps, 40 + t)
    synd_all = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    prior_shot = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
    prior_qubit = torch.from_numpy(channel_llr(np.linspace(0.01, 0.05, oc.n)).astype(np.float32)).cuda()
    for shots in (1, 2, 769, 2000):
        for mode, prior in ((P.LEAD_PRIOR_PER_SHOT, prior_shot[:shots]), (P.LEAD_PRIOR_SHARED, prior_qubit)):
            if mode == P.LEAD_PRIOR_SHARED and shots not in (2, 2000):
                continue
            synd = synd_all[:shots]
            ref = _decode(dec, synd, prior, mode, 2, form)
            got = _decode(dec, synd, prior, mode, 1, form)
            for key in ("ehat", "post", "lam", "stats"):
                assert np.array_equal(got[key], ref[key]), (shots, mode, key)
    conv = float((ref["stats"][:, 0] == 1).mean())
    log(f"[tiles] PSL(2,7) t={t} form {form}: persistent kernel equals the per-shot kernel on 1/2/769/2000 shots "
        f"(converged {conv:.3f})")


def test_tiles_stage_global_and_fixed_point_off():
    """Global BP alone (lambda' = the channel prior, no Phase 1) and runs to
    the cap with the fixed-point exit off."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("L")
    shots = 900
    ps = uniform_p(shots, 0.02, 0.06, 77)
    e = bitflip_packed(shots, oc.n, ps, 77)
    for kw in (dict(stage=P.LEAD_STAGE_GLOBAL), dict(fixed_point_stop=0), dict(early_exit=0, fixed_point_stop=0)):
        code, dec = gpu_decoder(spec, t=0, max_iter_local=16, max_iter_global=16, max_shots=shots, **kw)
        synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
        prior = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
        ref = _decode(dec, synd, prior, P.LEAD_PRIOR_PER_SHOT, 2, 2)
        got = _decode(dec, synd, prior, P.LEAD_PRIOR_PER_SHOT, 1, 2)
        for key in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(got[key], ref[key]), (kw, key)
        log(f"[tiles] {kw}: persistent kernel equals the per-shot kernel on {shots} shots")


@pytest.mark.parametrize("t", [0, 1])
def test_forms_equal_on_psl27(t):
    """Form 1 (compressed check state in both phases) and form 2 (the Phase 1
    queue kernel with the messages of the lowest-degree checks in LDS, the
    persistent Phases 2-3 kernel with the mixed state) give the same bits,
    lambda' (the Phase 1 posteriors aggregated) included."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("L")
    shots = 1500
    code, dec = gpu_decoder(spec, t=t, max_iter_local=64, max_iter_global=24, max_shots=shots)
    ps = uniform_p(shots, 0.01, 0.05, 90 + t)
    e = bitflip_packed(shots, oc.n, ps, 90 + t)
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    prior = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
    r1 = _decode(dec, synd, prior, P.LEAD_PRIOR_PER_SHOT, 1, 1)
    r2 = _decode(dec, synd, prior, P.LEAD_PRIOR_PER_SHOT, 1, 2)
    for key in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(r1[key], r2[key]), key
    log(f"[tiles] PSL(2,7) t={t}: forms 1 and 2 identical on {shots} shots (64 local rounds)")
