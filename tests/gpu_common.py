"""Shared helpers of the GPU tests: run the HIP decoder and the oracle on the
same seeded inputs and compare them."""
import sys

import numpy as np

from lead_inputs import bitflip_packed, unpack_bits, channel_llr

# |Delta LLR| bound between the FP32 GPU posteriors and the FP64 oracle.
LLR_TOL = 1e-3
# Conditioning.  Min-sum BP that does not converge is an expanding map on
# loopy graphs: a rounding difference grows by a factor ~2-4 per iteration, so
# after a few dozen iterations any two correct implementations with different
# rounding (FP32 vs FP64, or two FP64 summation orders) may disagree by O(1).
# The oracle is therefore re-run K times with every computed value perturbed
# by a relative PERTURB (a few FP32 ulps, Monte Carlo arithmetic); a shot
# whose FP64 result moves by more than ILL_TOL, or whose hard decisions or
# statistics change, is ill-conditioned.  Ill-conditioned shots are counted
# and reported, and covered statistically (logical error rate); every
# well-conditioned shot must meet the bar.
PERTURB = 2.4e-7
K_PERTURB = 3
ILL_TOL = LLR_TOL / 4
TAU = 1e-4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    return torch


def gpu_decoder(spec, t=0, max_shots=1 << 17, **params):
    import paper_2605_17796_amd as P
    code = P.Code.from_spec(spec)
    return code, P.Decoder(code, t=t, max_shots=max_shots, **params)


def oracle_params(**kw):
    from oracle import oracle as o
    m = dict(alpha=1.0, ms_scale=0.75, max_iter_local=32, max_iter_global=32, llr_clamp=30.0, early_exit=1,
             stage=0, boost=1)
    m.update(kw)
    return o.params(**m)


def run_gpu(dec, synd_np, prior_np, mode, lam=False, post=True):
    torch = torch_dev()
    synd = torch.from_numpy(synd_np.view(np.int64)).cuda()
    prior = torch.from_numpy(np.ascontiguousarray(prior_np, dtype=np.float32)).cuda()
    out = dec.decode(synd, prior, mode=mode, lam=lam, post=post)
    torch.cuda.synchronize()
    res = {}
    for k, v in out.items():
        if v is None:
            continue
        a = v.cpu().numpy()
        res[k] = a.view(np.uint64) if k == "ehat" else a
    return res


def compare(orc, gpu, n, what=("post", "lam"), tol=LLR_TOL, tau=TAU, check_ehat=True, check_stats=True):
    """Per-shot comparison.  Returns a dict of counts; `unexplained` lists the
    shots that disagree although their oracle margin is >= tau, and `detail`
    describes the first few of them."""
    shots = orc["stats"].shape[0]
    bad = np.zeros(shots, dtype=bool)
    reason = [[] for _ in range(shots)]
    worst = 0.0
    for key in what:
        if key not in gpu:
            continue
        d = np.abs(gpu[key].astype(np.float64) - orc[key])
        per = d.max(axis=1)
        for i in np.nonzero(per > tol)[0]:
            reason[i].append(f"{key} max|d|={per[i]:.3g} at {int(d[i].argmax())}")
        bad |= per > tol
        worst = max(worst, float(per[per <= tol].max()) if np.any(per <= tol) else 0.0)
    if check_ehat and "ehat" in gpu:
        eg = unpack_bits(gpu["ehat"], n)
        eo = unpack_bits(orc["ehat"], n)
        near0 = np.abs(orc["post"]) < tol
        diff = (eg != eo) & ~near0
        for i in np.nonzero(diff.any(axis=1))[0]:
            reason[i].append(f"ehat differs at {int(diff[i].sum())} bits")
        bad |= diff.any(axis=1)
    if check_stats and "stats" in gpu:
        st = gpu["stats"][:, :5]
        so = orc["stats"]
        if "ehat" not in gpu:   # LOCAL stage: no global fields
            st, so = st[:, 2:], so[:, 2:]
        sd = np.any(st != so, axis=1)
        for i in np.nonzero(sd)[0]:
            reason[i].append(f"stats gpu={st[i].tolist()} oracle={so[i].tolist()}")
        bad |= sd
    tie = orc["ill"] if "ill" in orc else orc["margin"] < tau
    unexplained = np.nonzero(bad & ~tie)[0].tolist()
    detail = [f"shot {i} margin={orc['margin'][i]:.2e} spread={orc.get('spread', np.zeros(shots))[i]:.2e}: "
              + "; ".join(reason[i]) for i in unexplained[:6]]
    return dict(shots=shots, bad=int(bad.sum()), tie=int(tie.sum()), bad_tie=int((bad & tie).sum()),
                unexplained=unexplained, worst_ok=worst, detail=detail)


def oracle_decode_conditioned(oc, synd, prior, t=0, k=K_PERTURB, **kw):
    """Plain oracle decode plus a per-shot `ill` flag from K perturbed runs."""
    ref = oc.decode(synd, prior, t=t, p=oracle_params(**kw))
    n = oc.n
    ill = np.zeros(synd.shape[0], dtype=bool)
    spread = np.zeros(synd.shape[0])
    e_ref = unpack_bits(ref["ehat"], n)
    near0 = np.abs(ref["post"]) < LLR_TOL
    for i in range(k):
        pk = oc.decode(synd, prior, t=t, p=oracle_params(perturb=PERTURB, perturb_seed=i + 1, **kw))
        d = np.maximum(np.abs(pk["post"] - ref["post"]).max(axis=1), np.abs(pk["lam"] - ref["lam"]).max(axis=1))
        spread = np.maximum(spread, d)
        ill |= d > ILL_TOL
        ill |= np.any((unpack_bits(pk["ehat"], n) != e_ref) & ~near0, axis=1)
        ill |= np.any(pk["stats"] != ref["stats"], axis=1)
    ref["ill"] = ill
    ref["spread"] = spread
    return ref


def bitflip_inputs(oc, shots, p, seed, t=0):
    e = bitflip_packed(shots, oc.n, p, seed)
    s = oc.syndrome(e, t)
    lam = np.full(shots, float(channel_llr(p)), dtype=np.float32)
    return e, s, lam


def oracle_global_conditioned(oc, synd, prior, t=0, k=K_PERTURB, **kw):
    """Oracle global BP alone (channel priors, no local phase) with the
    per-shot `ill` flag from K perturbed runs, in the layout compare()
    expects (stats columns converged, iterations)."""
    ref = oc.global_bp(synd, prior, t=t, p=oracle_params(**kw))
    n = oc.n
    e_ref = unpack_bits(ref["ehat"], n)
    near0 = np.abs(ref["post"]) < LLR_TOL
    ill = np.zeros(synd.shape[0], dtype=bool)
    spread = np.zeros(synd.shape[0])
    for i in range(k):
        pk = oc.global_bp(synd, prior, t=t, p=oracle_params(perturb=PERTURB, perturb_seed=i + 1, **kw))
        d = np.abs(pk["post"] - ref["post"]).max(axis=1)
        spread = np.maximum(spread, d)
        ill |= d > ILL_TOL
        ill |= np.any((unpack_bits(pk["ehat"], n) != e_ref) & ~near0, axis=1)
        ill |= np.any(pk["stats"] != ref["stats"], axis=1)
    ref["ill"] = ill
    ref["spread"] = spread
    ref["margin"] = np.full(synd.shape[0], np.inf)
    return ref
