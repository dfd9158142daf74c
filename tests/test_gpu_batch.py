"""Batched decoding: several requests of different codes, shot counts and
priors in one call or one graph launch give, for every shot, exactly the
outputs of decoding that request alone."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder
from lead_inputs import bitflip_packed, channel_llr, uniform_p

pytestmark = pytest.mark.gpu

ROUNDS = {"T": 32, "M": 50, "L": 64}


def _request(dec, oc, shots, seed, p_lo=0.02, p_hi=0.08):
    """Syndromes of errors drawn with a per-shot p ~ U[p_lo, p_hi], per-shot
    channel LLR priors."""
    torch = torch_dev()
    ps = uniform_p(shots, p_lo, p_hi, seed)
    e = bitflip_packed(shots, oc.n, ps, seed)
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    prior = torch.from_numpy(channel_llr(ps)).cuda()
    return synd, prior


def _alone(dec, synd, prior):
    torch = torch_dev()
    out = dec.decode(synd, prior, lam=True)
    torch.cuda.synchronize()
    return {k: v.clone() for k, v in out.items()}


def _decoders(names):
    decs = {}
    for name in names:
        spec, oc = code_pair(name)
        T = ROUNDS[name]
        code, dec = gpu_decoder(spec, max_iter_local=T, max_iter_global=T, max_shots=4096)
        decs[name] = (code, dec, oc)
    return decs


def test_mixed_batch_equals_alone():
    import paper_2605_17796_amd as P
    torch = torch_dev()
    decs = _decoders(["T", "M", "L"])
    sizes = {"T": 1000, "M": 301, "L": 7}
    entries, alone = [], {}
    for i, (name, (code, dec, oc)) in enumerate(decs.items()):
        synd, prior = _request(dec, oc, sizes[name], seed=100 + i)
        alone[name] = _alone(dec, synd, prior)
        out = dec.alloc_outputs(sizes[name], lam=True)
        entries.append((dec, synd, prior, out, P.LEAD_PRIOR_PER_SHOT))
    batch = P.Batch(entries)
    batch.run()
    torch.cuda.synchronize()
    for (dec, synd, prior, out, mode), name in zip(entries, decs):
        for k in ("ehat", "post", "lam", "stats"):
            assert torch.equal(out[k], alone[name][k]), (name, k)
    log("[batch] T/M/L mixed batch (1000/301/7 shots, p~U[0.02,0.08]) equals per-code decodes")


def test_same_decoder_items_run_in_order():
    import paper_2605_17796_amd as P
    torch = torch_dev()
    decs = _decoders(["M"])
    code, dec, oc = decs["M"]
    reqs = [_request(dec, oc, n, seed=200 + n) for n in (33, 1, 64)]
    alone = [_alone(dec, s, p) for s, p in reqs]
    entries = [(dec, s, p, dec.alloc_outputs(int(s.shape[0]), lam=True), P.LEAD_PRIOR_PER_SHOT) for s, p in reqs]
    P.Batch(entries).run()
    torch.cuda.synchronize()
    for (d, s, p, out, m), ref in zip(entries, alone):
        for k in ("ehat", "post", "lam", "stats"):
            assert torch.equal(out[k], ref[k]), k


def test_graph_replays_match_eager():
    """Capture once, then replay with refilled inputs; eager decodes and
    synchronisations run between replays; every replay is checked."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    decs = _decoders(["T", "M"])
    sizes = {"T": 257, "M": 96}
    bufs = {}
    entries = []
    for name, (code, dec, oc) in decs.items():
        synd, prior = _request(dec, oc, sizes[name], seed=300)
        out = dec.alloc_outputs(sizes[name], lam=True)
        bufs[name] = (synd, prior, out)
        entries.append((dec, synd, prior, out, P.LEAD_PRIOR_PER_SHOT))
    batch = P.Batch(entries).capture()
    for rep in range(4):
        refs = {}
        for i, (name, (code, dec, oc)) in enumerate(decs.items()):
            synd_new, prior_new = _request(dec, oc, sizes[name], seed=400 + 10 * rep + i)
            refs[name] = _alone(dec, synd_new, prior_new)        # eager work between replays
            bufs[name][0].copy_(synd_new)
            bufs[name][1].copy_(prior_new)
        torch.cuda.synchronize()
        batch.replay()
        torch.cuda.synchronize()
        for name in decs:
            out = bufs[name][2]
            for k in ("ehat", "post", "lam", "stats"):
                assert torch.equal(out[k], refs[name][k]), (rep, name, k)
    log("[batch] graph replays x4 with refilled inputs equal the eager decodes")


@pytest.mark.parametrize("name", ["T", "M"])
def test_autotune_keeps_results(name):
    torch = torch_dev()
    decs = _decoders([name])
    code, dec, oc = decs[name]
    synd, prior = _request(dec, oc, 2000, seed=500)
    before = _alone(dec, synd, prior)
    best = dec.autotune(synd, prior)
    after = _alone(dec, synd, prior)
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(before[k], after[k]), k
    assert dec.get_schedule() == best
    log(f"[autotune] {name}: {best}")
