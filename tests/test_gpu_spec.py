"""Kernels compiled for one code (check masks and local position map as
compile-time constants) give outputs bit-identical to the precompiled
kernels, for every code size, check type, prior mode and stopping rule."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder, run_gpu
from lead_inputs import bitflip_packed, channel_llr, uniform_p

pytestmark = pytest.mark.gpu

ROUNDS = {"T": 32, "M": 50, "L": 64, "appendix": 16}


def _inputs(dec, oc, shots, seed, t):
    torch = torch_dev()
    ps = uniform_p(shots, 0.02, 0.08, seed)
    e = bitflip_packed(shots, oc.n, ps, seed)
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return synd.cpu().numpy().view(np.uint64), ps


def _priors(mode, ps, n, seed):
    if mode == 0:
        return channel_llr(ps).astype(np.float32)
    rng = np.random.default_rng(seed)
    if mode == 1:
        return channel_llr(rng.uniform(0.02, 0.08, n)).astype(np.float32)
    return channel_llr(rng.uniform(0.02, 0.08, (ps.shape[0], n))).astype(np.float32)


def _forms(dec, synd, prior, mode, eloc):
    """Outputs under every kernel form: specialised with one register per
    message (views of at most 192 edges; the per-shot kernel keeps the
    compressed state on the highest-degree checks above 128), specialised with
    the compressed check state, precompiled split, precompiled fused."""
    runs = {}
    for form in (2, 1, 0):
        dec.set_schedule(specialized=form)
        want = form if form != 2 or eloc <= 192 else 1
        assert dec.get_schedule()["specialized"] == want
        runs[form] = run_gpu(dec, synd, prior, mode, lam=True)
    dec.set_schedule(fused=1)
    runs["fused"] = run_gpu(dec, synd, prior, mode, lam=True)
    return runs


CASES = [("T", 0, 0, {}), ("T", 1, 2, {}), ("M", 0, 0, {}), ("M", 1, 0, {}), ("M", 0, 1, {}), ("M", 0, 2, {}),
         ("M", 0, 0, dict(early_exit=0)), ("M", 0, 0, dict(fixed_point_stop=0)), ("M", 0, 0, dict(alpha=0.1)),
         ("M", 0, 0, dict(stage=1)), ("L", 0, 0, {}), ("L", 1, 1, {}), ("appendix", 0, 0, {}),
         ("appendix", 1, 2, {}), ("M", 0, 0, dict(llr_clamp=4.0)), ("L", 0, 0, dict(llr_clamp=4.0)),
         ("T", 1, 0, dict(llr_clamp=2.0))]


@pytest.mark.parametrize("name,t,mode,params", CASES)
def test_specialised_equals_precompiled(name, t, mode, params):
    spec, oc = code_pair(name)
    T = ROUNDS[name]
    kw = dict(max_iter_local=T, max_iter_global=T)
    kw.update(params)
    code, dec = gpu_decoder(spec, t=t, max_shots=4096, **kw)
    shots = {"T": 777, "M": 301, "L": 41, "appendix": 257}[name]
    synd, ps = _inputs(dec, oc, shots, seed=900 + shots + 7 * t + mode, t=t)
    prior = _priors(mode, ps, oc.n, seed=31 + mode)
    runs = _forms(dec, synd, prior, mode, code.info.eloc[t])
    keys = ("lam", "stats") if params.get("stage") == 1 else ("ehat", "post", "lam", "stats")
    a = runs[2]
    for form in (1, 0, "fused"):
        for k in keys:
            assert np.array_equal(a[k], runs[form][k]), (k, form)
    log(f"[spec] {name} t={t} mode={mode} {params}: {shots} shots bit-identical over every kernel form "
        f"(converged {a['stats'][:, 0].mean():.3f})")


def test_specialised_ragged_and_chunked():
    """Shot counts that leave the last workgroup partly empty, and a batch
    decoded in 13334-shot chunks."""
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, max_shots=40000)
    synd, ps = _inputs(dec, oc, 40000, seed=5, t=0)
    prior = channel_llr(ps).astype(np.float32)
    dec.set_schedule(chunk_shots=16384)
    full = run_gpu(dec, synd, prior, 0, lam=True)
    dec.set_schedule()
    for n_sub in (1, 4, 5, 6, 11):
        part = run_gpu(dec, synd[:n_sub], prior[:n_sub], 0, lam=True)
        for k in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(part[k], full[k][:n_sub]), (n_sub, k)
    for form in (1, 0):
        dec.set_schedule(specialized=form)
        ref = run_gpu(dec, synd, prior, 0, lam=True)
        for k in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(full[k], ref[k]), (form, k)


def test_phase_timing():
    """Per-phase device time of the work-queue form: one pair of timed
    launches per workspace chunk, none while a graph is being captured."""
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, max_shots=40000)
    synd, ps = _inputs(dec, oc, 40000, seed=8, t=0)
    s = torch.from_numpy(synd.view(np.int64)).cuda()
    prior = torch.from_numpy(channel_llr(ps).astype(np.float32)).cuda()
    dec.set_schedule(chunk_shots=32768)
    assert dec.get_schedule()["chunk_shots"] == 32768
    dec.time_phases(True)
    out = dec.decode(s, prior)
    pt = dec.phase_times()
    assert pt["local_launches"] == 2 and pt["global_launches"] == 2      # two equal chunks of 20000
    assert pt["local_ms"] > 0 and pt["global_ms"] > 0
    g = P.Batch([(dec, s, prior, out, P.LEAD_PRIOR_PER_SHOT)]).capture()
    g.replay()
    torch.cuda.synchronize()
    assert dec.phase_times()["global_launches"] == 2
    dec.time_phases(False)
    dec.decode(s, prior, out=out)
    torch.cuda.synchronize()
    assert dec.phase_times()["global_launches"] == 0
    log(f"[timing] T 40000 shots: {pt}")
