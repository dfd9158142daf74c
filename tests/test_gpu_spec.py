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


def _both(dec, synd, prior, mode):
    dec.set_schedule(specialized=1)
    assert dec.get_schedule()["specialized"] == 1
    a = run_gpu(dec, synd, prior, mode, lam=True)
    dec.set_schedule(specialized=0)
    assert dec.get_schedule()["specialized"] == 0
    b = run_gpu(dec, synd, prior, mode, lam=True)
    dec.set_schedule(fused=1)
    c = run_gpu(dec, synd, prior, mode, lam=True)
    return a, b, c


CASES = [("T", 0, 0, {}), ("T", 1, 2, {}), ("M", 0, 0, {}), ("M", 1, 0, {}), ("M", 0, 1, {}), ("M", 0, 2, {}),
         ("M", 0, 0, dict(early_exit=0)), ("M", 0, 0, dict(fixed_point_stop=0)), ("M", 0, 0, dict(alpha=0.1)),
         ("M", 0, 0, dict(stage=1)), ("L", 0, 0, {}), ("L", 1, 1, {}), ("appendix", 0, 0, {}),
         ("appendix", 1, 2, {})]


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
    a, b, c = _both(dec, synd, prior, mode)
    keys = ("lam", "stats") if params.get("stage") == 1 else ("ehat", "post", "lam", "stats")
    for k in keys:
        assert np.array_equal(a[k], b[k]), (k, "specialised vs precompiled split")
        assert np.array_equal(a[k], c[k]), (k, "specialised vs precompiled fused")
    log(f"[spec] {name} t={t} mode={mode} {params}: {shots} shots bit-identical "
        f"(converged {a['stats'][:, 0].mean():.3f})")


def test_specialised_ragged_and_chunked():
    """Shot counts that leave the last workgroup partly empty, and a batch
    above the 32768-shot workspace."""
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, max_shots=40000)
    synd, ps = _inputs(dec, oc, 40000, seed=5, t=0)
    prior = channel_llr(ps).astype(np.float32)
    full = run_gpu(dec, synd, prior, 0, lam=True)
    for n_sub in (1, 4, 5, 6, 11):
        part = run_gpu(dec, synd[:n_sub], prior[:n_sub], 0, lam=True)
        for k in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(part[k], full[k][:n_sub]), (n_sub, k)
    dec.set_schedule(specialized=0)
    ref = run_gpu(dec, synd, prior, 0, lam=True)
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(full[k], ref[k]), k
