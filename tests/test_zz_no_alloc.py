"""lead_decode_noalloc: the decode for callers that cannot allocate, with its
buffers in the library's static device scratch.  Through the C ABI, two
calls in a row (the second with fewer shots, so stale scratch contents from
the first would show) give outputs identical bit for bit to lead_decode's on
the same decoder; batches beyond the scratch are refused before anything is
enqueued."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder
from lead_inputs import bitflip_packed, channel_llr

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


def _inputs(dec, oc, shots, p, seed):
    torch = torch_dev()
    e = bitflip_packed(shots, oc.n, p, seed)
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    prior = torch.full((shots,), float(channel_llr(p)), dtype=torch.float32, device="cuda")
    return synd, prior


def _pair(dec, synd, prior, post=True, lam=True, stats=True):
    """(lead_decode outputs, lead_decode_noalloc outputs) on the same inputs."""
    torch = torch_dev()
    shots = int(synd.shape[0])
    ref = dec.decode(synd, prior, out=dec.alloc_outputs(shots, post=post, lam=lam, stats=stats))
    out = dec.alloc_outputs(shots, post=post, lam=lam, stats=stats)
    # poison the outputs so that anything left unwritten shows
    for v in out.values():
        if v is not None:
            v.fill_(-7)
    got = dec.decode(synd, prior, out=out, noalloc=True)
    torch.cuda.synchronize()
    return ref, got


def _same(ref, got, what):
    for k, v in ref.items():
        if v is None:
            continue
        a, b = v.cpu().numpy(), got[k].cpu().numpy()
        assert a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{what}: {k} differs"


@pytest.mark.parametrize("name,T,sizes", [("M", 50, (3000, 700)), ("L", 8, (600, 150)), ("T", 32, (2000, 333))])
def test_noalloc_matches_decode(name, T, sizes):
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, max_shots=max(sizes), max_iter_local=T, max_iter_global=T)
    for k, shots in enumerate(sizes):
        log(f"[noalloc] {name} call {k + 1}: {shots} shots, {T}+{T} rounds")
        synd, prior = _inputs(dec, oc, shots, 0.05 if name != "L" else 0.02, seed=300 + k)
        ref, got = _pair(dec, synd, prior)
        _same(ref, got, f"{name} call {k + 1}")
        conv = float((ref["stats"][:, 0] != 0).float().mean())
        log(f"[noalloc] {name} call {k + 1}: identical to lead_decode ({conv:.3f} converged)")


def test_noalloc_global_osd_buffers_from_scratch():
    """With global OSD (order 3) and no posterior / statistics / lambda'
    outputs, the OSD's buffers come from the scratch too."""
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_shots=2000, max_iter_local=20, max_iter_global=20, global_post=1,
                            osd_order=3)
    for k, shots in enumerate((1200, 300)):
        synd, prior = _inputs(dec, oc, shots, 0.05, seed=400 + k)
        ref, got = _pair(dec, synd, prior, post=False, lam=False, stats=False)
        _same(ref, got, f"OSD call {k + 1}")
        log(f"[noalloc] M global OSD-CS3 call {k + 1}: {shots} shots identical to lead_decode")


def test_noalloc_capacity_refused():
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_shots=9000)
    per_shot = 4 * 60 * 36 + 8 * 60
    cap = (SCRATCH - 2048) // per_shot
    synd = torch.zeros((cap + 1, dec.synd_words), dtype=torch.int64, device="cuda")
    prior = torch.full((cap + 1,), 3.0, dtype=torch.float32, device="cuda")
    out = dec.alloc_outputs(cap + 1)
    out["ehat"].fill_(-7)
    with pytest.raises(P.LeadError) as ei:
        dec.decode(synd, prior, out=out, noalloc=True)
    assert P.STATUS_NAMES[ei.value.status] == "LEAD_E_CAPACITY"
    assert f"at most {cap} shots" in str(ei.value)
    torch.cuda.synchronize()
    assert int((out["ehat"] != -7).sum()) == 0, "a refused call enqueued work"
    # exactly at the limit it runs (zero syndromes decode to zero at once)
    dec.decode(synd[:cap], prior[:cap], out={k: (v[:cap] if v is not None else None) for k, v in out.items()},
               noalloc=True)
    torch.cuda.synchronize()
    assert int(out["ehat"][:cap].abs().sum()) == 0
    log(f"[noalloc] A5: {cap + 1} shots refused (capacity {cap}), {cap} decoded")
