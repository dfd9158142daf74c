"""Fused batch (lead_batch_fused_*): requests of codes of different sizes
(D6 / A5 / PSL(2,7): Delta = 4 / 6 / 8), check types, kernel forms, prior
modes, stages and shot counts decoded by one persistent Phase 1 launch and
one Phases 2-3 launch, replayed as a graph.  Every request's outputs equal
its lone lead_decode bit for bit, on every replay with refilled inputs."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder
from lead_inputs import bitflip_packed, channel_llr, uniform_p

pytestmark = pytest.mark.gpu

ROUNDS = {"T": 32, "M": 50, "L": 64}


def _inputs(dec, oc, shots, seed, t=0, shared=False):
    torch = torch_dev()
    ps = uniform_p(shots, 0.02, 0.08, seed)
    e = bitflip_packed(shots, oc.n, ps, seed)
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    if shared:   # one prior per qubit, shared by the shots
        prior = torch.from_numpy(channel_llr(np.linspace(0.03, 0.07, oc.n)).astype(np.float32)).cuda()
    else:
        prior = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
    return synd, prior


def _run(entries, reps=2):
    """Fused launches (with inputs refilled between replays) against each
    request decoded alone."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    fused_entries, refs = [], []
    for dec, synd, prior, mode, oc, t, seed in entries:
        out = dec.alloc_outputs(int(synd.shape[0]), lam=True)
        fused_entries.append((dec, synd, prior, out, mode))
    fb = P.FusedBatch(fused_entries)
    for rep in range(reps):
        # refill every request's inputs (new shots), then replay
        for k, (dec, synd, prior, mode, oc, t, seed) in enumerate(entries):
            s2, p2 = _inputs(dec, oc, int(synd.shape[0]), seed + 100 * (rep + 1), t, shared=mode != 0)
            synd.copy_(s2)
            if mode == 0:
                prior.copy_(p2)
            for v in fused_entries[k][3].values():
                if v is not None:
                    v.fill_(-9)
        torch.cuda.synchronize()
        fb.launch()
        torch.cuda.synchronize()
        for k, (dec, synd, prior, mode, oc, t, seed) in enumerate(entries):
            ref = dec.decode(synd, prior, mode=mode, lam=True)
            torch.cuda.synchronize()
            out = fused_entries[k][3]
            for key in ("ehat", "post", "lam", "stats"):
                assert torch.equal(out[key], ref[key]), (rep, k, key)
    return fused_entries


def test_fused_mixed_codes_equal_alone():
    """The mixed workload: D6, A5 and PSL(2,7) with uneven shot counts and
    per-shot p ~ U[0.02, 0.08]."""
    entries = []
    for i, (name, shots) in enumerate((("T", 1000), ("M", 3000), ("L", 300))):
        spec, oc = code_pair(name)
        code, dec = gpu_decoder(spec, max_iter_local=ROUNDS[name], max_iter_global=ROUNDS[name], max_shots=shots)
        synd, prior = _inputs(dec, oc, shots, seed=700 + i)
        entries.append((dec, synd, prior, 0, oc, 0, 700 + i))
    fe = _run(entries)
    conv = [float((e[3]["stats"][:, 0] == 1).float().mean()) for e in fe]
    log(f"[fused] D6 1000 / A5 3000 / PSL(2,7) 300 shots, 2 replays equal the lone decodes; converged {conv}")


def test_fused_forms_modes_stages():
    """Kernel forms (compressed, one register per message, sum-product),
    check types, a prior per qubit, stage GLOBAL, and PSL(2,7)'s X-check
    views, all in one fused batch."""
    import paper_2605_17796_amd as P
    specs = [("T", 0, 2, 0, {}, 400), ("M", 0, 1, 0, dict(stage=2), 900), ("M", 1, 2, 1, {}, 700),
             ("L", 0, 2, 0, {}, 150), ("T", 0, 3, 0, dict(bp=1), 500), ("L", 1, 2, 0, {}, 120)]
    entries = []
    for i, (name, t, form, mode, kw, shots) in enumerate(specs):
        spec, oc = code_pair(name)
        T = 12 if name == "L" else ROUNDS[name]
        code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, max_shots=shots, **kw)
        if form != 3:
            dec.set_schedule(specialized=form)
        assert dec.get_schedule()["specialized"] == form
        synd, prior = _inputs(dec, oc, shots, seed=800 + i, t=t, shared=mode != 0)
        entries.append((dec, synd, prior, mode, oc, t, 800 + i))
    _run(entries, reps=1)
    log("[fused] six requests of mixed forms, check types, prior modes and stages equal their lone decodes")


def test_fused_shared_decoder_and_limits():
    """Two requests of one decoder in one fused batch (each has its own
    workspace); OSD post-processing and more than 8 requests are refused."""
    import paper_2605_17796_amd as P
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, max_iter_local=32, max_iter_global=32, max_shots=600)
    entries = []
    for i, shots in enumerate((600, 250)):
        synd, prior = _inputs(dec, oc, shots, seed=900 + i)
        entries.append((dec, synd, prior, 0, oc, 0, 900 + i))
    _run(entries)
    torch = torch_dev()
    synd, prior = _inputs(dec, oc, 10, seed=950)
    out = dec.alloc_outputs(10)
    _, odec = gpu_decoder(spec, max_shots=10, global_post=1)
    with pytest.raises(P.LeadError, match="UNSUPPORTED"):
        P.FusedBatch([(odec, synd, prior, out, 0)])
    with pytest.raises(P.LeadError, match="UNSUPPORTED"):
        P.FusedBatch([(dec, synd, prior, out, 0)] * 9)
    log("[fused] two requests of one decoder equal their lone decodes; limits refused")
