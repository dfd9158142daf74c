"""GPU parity: the HIP decoder through the C ABI against the FP64 oracle on
the same seeded inputs.

Bar: posteriors (L_post) and regularised priors (lambda') within
|Delta LLR| <= 1e-3; hard decisions bit-exact except where the oracle's
|L_post| < 1e-3; per-shot statistics (convergence, iteration counts,
converged local views) identical.  Every well-conditioned shot must meet the
bar; ill-conditioned shots (the oracle's own result moves under FP32-sized
rounding perturbations, see gpu_common) are counted, each case keeps a
minimum share of well-conditioned shots, and the logical error rate covers
them statistically."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import (LLR_TOL, TAU, log, torch_dev, gpu_decoder, oracle_params, run_gpu, compare,
                        bitflip_inputs, oracle_decode_conditioned)
from lead_inputs import bitflip_packed, unpack_bits, pack_bits, channel_llr, depolarizing_packed

pytestmark = pytest.mark.gpu


def _gpu_syndrome(dec, e):
    torch = torch_dev()
    s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint64)


def _decode_both(name, t, shots, p, seed, stage=0, mode=0, prior=None, **kw):
    spec, oc = code_pair(name)
    params = dict(max_iter_local=kw.pop("Tl", 32), max_iter_global=kw.pop("Tg", 32), stage=stage, **kw)
    code, dec = gpu_decoder(spec, t=t, **params)
    e = bitflip_packed(shots, oc.n, p, seed)
    s_orc = oc.syndrome(e, t)
    s_gpu = _gpu_syndrome(dec, e)
    assert np.array_equal(s_gpu, s_orc), "syndrome kernel differs from the oracle"
    if prior is None:
        prior = np.full(shots, float(channel_llr(p)), dtype=np.float32)
    gpu = run_gpu(dec, s_gpu, prior, mode, lam=True)
    orc = oracle_decode_conditioned(oc, s_orc, prior.astype(np.float64), t=t, **params)
    return oc, gpu, orc


def _report(tag, r, min_well=0.5):
    log(f"[parity] {tag}: shots={r['shots']} differ={r['bad']} ill-conditioned={r['tie']} "
        f"differ&ill={r['bad_tie']} unexplained={len(r['unexplained'])} worst_ok={r['worst_ok']:.2e}")
    for line in r["detail"]:
        log("    " + line)
    assert not r["unexplained"], r["detail"]
    assert r["shots"] - r["tie"] >= min_well * r["shots"], "too few well-conditioned shots to compare"


@pytest.mark.parametrize("name", ["T", "M", "L"])
@pytest.mark.parametrize("t", [0, 1])
def test_syndrome_kernel_bit_exact(name, t):
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t)
    shots = 37 if name == "L" else 301
    for p in (0.0, 0.05, 0.5):
        e = bitflip_packed(shots, oc.n, p, seed=5)
        assert np.array_equal(_gpu_syndrome(dec, e), oc.syndrome(e, t)), (name, t, p)


@pytest.mark.parametrize("name,shots", [("T", 400), ("M", 120), ("appendix", 300)])
@pytest.mark.parametrize("p", [0.02, 0.05])
def test_local_stage_parity(name, shots, p):
    """Phases 1-2 (stage LOCAL): lambda' and the local statistics."""
    Tl = 50 if name == "M" else 32
    oc, gpu, orc = _decode_both(name, 0, shots, p, seed=11, stage=1, Tl=Tl)
    r = compare(orc, gpu, oc.n, what=("lam",), check_ehat=False)
    _report(f"local {name} p={p}", r)


@pytest.mark.parametrize("name,shots,p", [("T", 1000, 0.05), ("T", 1000, 0.02), ("M", 150, 0.05),
                                          ("M", 150, 0.02), ("appendix", 500, 0.05)])
def test_full_decode_parity(name, shots, p):
    T = 50 if name == "M" else 32
    oc, gpu, orc = _decode_both(name, 0, shots, p, seed=13, Tl=T, Tg=T)
    _report(f"full {name} p={p} T={T}", compare(orc, gpu, oc.n))


@pytest.mark.parametrize("name,t,shots,p,T", [("T", 0, 1000, 0.05, 8), ("T", 1, 1000, 0.05, 8),
                                              ("M", 0, 150, 0.05, 8), ("M", 1, 150, 0.05, 4),
                                              ("L", 0, 16, 0.03, 3), ("L", 1, 16, 0.03, 2),
                                              ("appendix", 1, 400, 0.05, 8)])
def test_short_cap_parity(name, t, shots, p, T):
    """Short iteration caps: the rounding amplification of non-converging
    min-sum (about beta * (column degree - 1) per iteration: x2 for T, x4 for
    M's X checks, x6 for L) stays below the tolerance, so nearly every shot is
    well-conditioned and the whole pipeline (both check types, every code) is
    compared shot by shot."""
    oc, gpu, orc = _decode_both(name, t, shots, p, seed=53, Tl=T, Tg=T)
    _report(f"T={T} {name} type={t} p={p}", compare(orc, gpu, oc.n), min_well=0.8)


@pytest.mark.parametrize("name,p,min_well", [("T", 0.015, 0.8), ("M", 0.01, 0.2)])
def test_x_checks_parity(name, p, min_well):
    oc, gpu, orc = _decode_both(name, 1, 300 if name == "T" else 100, p, seed=17, Tl=32, Tg=32)
    _report(f"X-checks {name}", compare(orc, gpu, oc.n), min_well=min_well)


@pytest.mark.parametrize("name,shots,clamp", [("T", 600, 3.0), ("M", 150, 4.0)])
def test_small_clamp_parity(name, shots, clamp):
    """A clamp that many |mu| exceed: the kernels clamp the two minima of
    each check rather than every mu, which must give the oracle's messages
    (it clamps every mu) wherever the clamp decides the minimum."""
    T = 20
    oc, gpu, orc = _decode_both(name, 0, shots, 0.05, seed=37, Tl=T, Tg=T, llr_clamp=clamp)
    _report(f"clamp={clamp} {name}", compare(orc, gpu, oc.n), min_well=0.3)


@pytest.mark.parametrize("alpha", [0.5, 0.01])
def test_alpha_parity(alpha):
    oc, gpu, orc = _decode_both("T", 0, 500, 0.05, seed=19, alpha=alpha)
    _report(f"alpha={alpha}", compare(orc, gpu, oc.n))


@pytest.mark.parametrize("mode", [1, 2])
def test_prior_modes(mode):
    """SHARED (one LLR per qubit) and FULL (per shot and qubit) priors."""
    spec, oc = code_pair("T")
    rng = np.random.default_rng(23)
    shots = 300
    if mode == 1:
        prior = np.log((1 - 0.04) / 0.04) + rng.uniform(-0.5, 0.5, size=oc.n).astype(np.float32)
        prior_o = np.broadcast_to(prior.astype(np.float64), (shots, oc.n))
    else:
        prior = rng.uniform(1.5, 4.5, size=(shots, oc.n)).astype(np.float32)
        prior_o = prior.astype(np.float64)
    code, dec = gpu_decoder(spec)
    e = bitflip_packed(shots, oc.n, 0.05, seed=29)
    s = _gpu_syndrome(dec, e)
    gpu = run_gpu(dec, s, prior.astype(np.float32), mode, lam=True)
    orc = oracle_decode_conditioned(oc, oc.syndrome(e), np.ascontiguousarray(prior_o))
    _report(f"prior mode {mode}", compare(orc, gpu, oc.n))


def test_early_exit_off_and_caps():
    oc, gpu, orc = _decode_both("T", 0, 300, 0.05, seed=31, early_exit=0, Tl=7, Tg=9)
    _report("early_exit=0", compare(orc, gpu, oc.n))
    assert np.all(gpu["stats"][:, 1] == 9) and np.all(gpu["stats"][:, 3] == 7)


def test_zero_syndrome_and_ragged_batches():
    """s = 0 gives e_hat = 0 after one global iteration; batch sizes that
    leave a partial workgroup (T packs 5 shots per workgroup) and a single
    shot decode like the same shots inside a large batch."""
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec)
    lam = float(channel_llr(0.05))
    z = np.zeros((7, 1), dtype=np.uint64)
    g = run_gpu(dec, z, np.full(7, lam, np.float32), 0)
    assert not g["ehat"].any() and np.all(g["stats"][:, 0] == 1) and np.all(g["stats"][:, 1] == 1)
    e, s, lamv = bitflip_inputs(oc, 23, 0.05, seed=37)
    s = _gpu_syndrome(dec, e)
    full = run_gpu(dec, s, lamv, 0, lam=True)
    for n_sub in (1, 4, 5, 6, 11):
        part = run_gpu(dec, s[:n_sub], lamv[:n_sub], 0, lam=True)
        for k in ("ehat", "post", "lam", "stats"):
            assert np.array_equal(part[k], full[k][:n_sub]), (n_sub, k)
    # zero shots is a no-op
    out = dec.decode(torch.zeros((0, 1), dtype=torch.int64, device="cuda"),
                     torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert out["ehat"].shape[0] == 0


@pytest.mark.parametrize("sched", [dict(shots_per_workgroup=2), dict(shots_per_workgroup=3),
                                   dict(shots_per_workgroup=4), dict(fused=1), dict(fused=1, shots_per_workgroup=4),
                                   dict(local_chunk=64), dict(local_chunk=4096, local_waves=7),
                                   dict(specialized=0), dict(specialized=0, local_chunk=64),
                                   dict(specialized=1)])
def test_schedule_does_not_change_results(sched):
    """Launch geometry (shots per workgroup, Phase 1 fused into the per-shot
    kernel or run from a work queue, queue chunk, wave count) leaves every
    output bit-identical (M: 60 lanes per shot, up to 4 shots per 256-lane
    group)."""
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=50, max_iter_global=50)
    e, s, lamv = bitflip_inputs(oc, 50, 0.05, seed=41)
    s = _gpu_syndrome(dec, e)
    ref = run_gpu(dec, s, lamv, 0, lam=True)
    dec.set_schedule(**sched)
    got = run_gpu(dec, s, lamv, 0, lam=True)
    for k in ("ehat", "post", "lam", "stats"):
        assert np.array_equal(got[k], ref[k]), k


def test_chunked_large_batch():
    """Batches decoded in one launch and chunk by chunk (32768-shot chunks)
    give the same results as shot-by-shot sub-batches."""
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, max_shots=70000)
    e = bitflip_packed(70000, oc.n, 0.05, seed=77)
    synd = torch.from_numpy(_gpu_syndrome(dec, e).view(np.int64)).cuda()
    lam = torch.full((70000,), float(channel_llr(0.05)), dtype=torch.float32, device="cuda")
    big = dec.decode(synd, lam, lam=True)
    dec.set_schedule(chunk_shots=32768)
    chunked = dec.decode(synd, lam, lam=True)
    idx = [0, 1, 32767, 32768, 32769, 65535, 65536, 69999]
    part = dec.decode(synd[idx].contiguous(), lam[idx].contiguous(), lam=True)
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(big[k], chunked[k]), k
        assert torch.equal(big[k][idx], part[k]), k


def _wilson(k, n, z=1.96):
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return c - h, c + h


@pytest.mark.parametrize("name,shots,p,T", [("T", 4000, 0.05, 32)])
def test_logical_error_rate_in_oracle_ci(name, shots, p, T):
    """c-14: over all shots, ill-conditioned ones included, the GPU's logical
    error rate (failure = not converged, or residual a non-trivial logical)
    lies in the oracle's Wilson 95% interval on the same shots."""
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, max_iter_local=T, max_iter_global=T)
    e = bitflip_packed(shots, oc.n, p, seed=61)
    s = _gpu_syndrome(dec, e)
    lam = np.full(shots, float(channel_llr(p)), dtype=np.float32)
    gpu = run_gpu(dec, s, lam, 0)
    orc = oc.decode(oc.syndrome(e), lam.astype(np.float64), p=oracle_params(max_iter_local=T, max_iter_global=T))
    fail_g = (gpu["stats"][:, 0] == 0) | oc.logical_failure(gpu["ehat"] ^ e)
    fail_o = (orc["stats"][:, 0] == 0) | oc.logical_failure(orc["ehat"] ^ e)
    lo, hi = _wilson(int(fail_o.sum()), shots)
    log(f"[ler] {name} p={p}: oracle {fail_o.mean():.4f} CI [{lo:.4f}, {hi:.4f}] gpu {fail_g.mean():.4f}")
    assert lo <= fail_g.mean() <= hi


def test_determinism():
    spec, oc = code_pair("M")
    code, dec = gpu_decoder(spec, max_iter_local=50, max_iter_global=50)
    e, s, lamv = bitflip_inputs(oc, 200, 0.05, seed=47)
    s = _gpu_syndrome(dec, e)
    a = run_gpu(dec, s, lamv, 0, lam=True)
    b = run_gpu(dec, s, lamv, 0, lam=True)
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_argument_errors():
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair("T")
    code, dec = gpu_decoder(spec, max_shots=8)
    s = torch.zeros((9, 1), dtype=torch.int64, device="cuda")
    lam = torch.zeros(9, dtype=torch.float32, device="cuda")
    with pytest.raises(P.LeadError) as ei:
        dec.decode(s, lam)
    assert P.STATUS_NAMES[ei.value.status] == "LEAD_E_CAPACITY"
    with pytest.raises(P.LeadError):
        P.lead_decode(dec._h, 2, None, 1, None, 0, None, 0, None, None, None, None)
    with pytest.raises((P.LeadError, ValueError)):
        dec.decode(torch.zeros((2, 0), dtype=torch.int64, device="cuda"), lam[:2])
    with pytest.raises(P.LeadError):
        P.Decoder(code, alpha=0.0)


@pytest.mark.parametrize("name,t,shots,p,T,kw", [
    ("T", 0, 301, 0.05, 32, {}), ("T", 1, 200, 0.05, 32, dict(specialized=1)), ("M", 0, 97, 0.05, 50, {}),
    ("M", 0, 64, 0.02, 50, dict(specialized=1)), ("M", 1, 120, 0.03, 50, {}), ("M", 0, 150, 0.05, 20, dict(bp=1)),
    ("M", 0, 150, 0.05, 20, dict(stage=2)), ("M", 0, 150, 0.05, 12, dict(local_post=1, global_post=1, osd_order=3)),
    ("L", 0, 40, 0.02, 16, {}), ("L", 1, 40, 0.02, 16, {}), ("L", 0, 24, 0.02, 8, dict(bp=1)),
    ("M", 0, 64, 0.05, 50, dict(specialized=0)), ("L", 0, 5, 0.02, 16, dict(specialized=0))])
def test_plain_form_bit_identical(name, t, shots, p, T, kw):
    """lead_decode_plain (one launch per global round, state in HBM, host
    convergence check) returns exactly what lead_decode returns: on the
    kernels compiled for the code (its per-round kernels, every form, BP
    flavour, stage and post-processing) and on the precompiled kernels
    (specialized = 0: min-sum without OSD)."""
    kw = dict(kw)
    form = kw.pop("specialized", None)
    spec, oc = code_pair(name)
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, **kw)
    if form is not None:
        dec.set_schedule(specialized=form)
        assert dec.get_schedule()["specialized"] == form
    e, _, lamv = bitflip_inputs(oc, shots, p, seed=71, t=t)
    s = _gpu_syndrome(dec, e)
    torch = torch_dev()
    synd = torch.from_numpy(s.view(np.int64)).cuda()
    lam = torch.from_numpy(lamv).cuda()
    a = dec.decode(synd, lam, lam=True)
    b = dec.decode(synd, lam, lam=True, plain=True)
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(a[k], b[k]), k
    log(f"[plain] {name} t={t} {kw} form={dec.get_schedule()['specialized']}: {shots} shots bit-identical, "
        f"conv={float((a['stats'][:, 0] != 0).float().mean()):.3f}")


@pytest.mark.parametrize("name,shots,p,T", [("T", 500, 0.05, 32), ("M", 300, 0.05, 50), ("M", 300, 0.02, 50),
                                            ("L", 8, 0.02, 64)])
def test_fixed_point_stop_is_exact(name, shots, p, T):
    """Ending a BP run whose message state reproduces itself gives exactly the
    outputs and reported counts of running every iteration to the cap: the
    test on local and global runs (fixed_point_stop = 1), on local runs only
    (2: the Phases 2-3 kernel compiled without the per-message comparison)
    and none (0), on the compiled kernels and in the plain form."""
    import paper_2605_17796_amd as P
    spec, oc = code_pair(name)
    torch = torch_dev()
    code, dec = gpu_decoder(spec, max_iter_local=T, max_iter_global=T, fixed_point_stop=1)
    e, _, lamv = bitflip_inputs(oc, shots, p, seed=73)
    synd = torch.from_numpy(_gpu_syndrome(dec, e).view(np.int64)).cuda()
    lam = torch.from_numpy(lamv).cuda()
    a = dec.decode(synd, lam, lam=True)
    pa = dec.decode(synd, lam, lam=True, plain=True)
    dec.set_params(max_iter_local=T, max_iter_global=T, fixed_point_stop=2)
    c = dec.decode(synd, lam, lam=True)
    pc = dec.decode(synd, lam, lam=True, plain=True)
    dec.set_params(max_iter_local=T, max_iter_global=T, fixed_point_stop=0)
    b = dec.decode(synd, lam, lam=True)
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam"):
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(pa[k], b[k]), k
        assert torch.equal(c[k], b[k]), k
        assert torch.equal(pc[k], b[k]), k
    for r in (a, pa, c, pc):
        assert torch.equal(r["stats"][:, :5], b["stats"][:, :5])
    # the local fixed-view counts of 1 and 2 agree; 2 reports no global fixed point
    for r in (c, pc):
        assert torch.equal(r["stats"][:, 5], a["stats"][:, 5])
        assert int(r["stats"][:, 6].abs().sum()) == 0
    assert int(b["stats"][:, 5:7].abs().sum()) == 0
    with pytest.raises(P.LeadError):
        dec.set_params(max_iter_local=T, max_iter_global=T, fixed_point_stop=3)
    st = a["stats"].cpu().numpy()
    log(f"[fixed] {name} p={p}: local views stopped at a fixed point {st[:, 5].sum() / (shots * code.info.order):.3f}, "
        f"shots with a global fixed point {(st[:, 6] > 0).mean():.3f} (mean iteration "
        f"{st[st[:, 6] > 0, 6].mean() if (st[:, 6] > 0).any() else 0:.1f})")
