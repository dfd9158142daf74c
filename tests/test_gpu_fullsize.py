"""The full-size workloads in the launch configuration the benchmark times:
10^5 A5 shots decoded in one launch per kernel (eager and as a replayed
graph, with the benchmark's parameters) and 10^5 PSL(2,7) shots; sampled
shots against the oracle, properties that hold at any size on every shot."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder, compare, oracle_decode_conditioned
from lead_inputs import bitflip_packed, channel_llr

pytestmark = pytest.mark.gpu


def _decode_full(name, shots, p, T, seed):
    import paper_2605_17796_amd as P
    torch = torch_dev()
    spec, oc = code_pair(name)
    # the benchmark's setting: the fixed-point exit on local runs only (the
    # Phases 2-3 kernel without the fixed-point test)
    code, dec = gpu_decoder(spec, max_shots=shots, max_iter_local=T, max_iter_global=T, fixed_point_stop=2)
    e = bitflip_packed(20_000, oc.n, p, seed)            # 20000 error draws, repeated
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda()).repeat(shots // 20_000, 1).contiguous()
    lam = torch.full((shots,), float(channel_llr(p)), dtype=torch.float32, device="cuda")
    eager = dec.decode(synd, lam, lam=True)
    out = dec.alloc_outputs(shots, lam=True)
    graph = P.Batch([(dec, synd, lam, out, P.LEAD_PRIOR_PER_SHOT)]).capture()
    graph.replay()
    torch.cuda.synchronize()
    for k in ("ehat", "post", "lam", "stats"):
        assert torch.equal(eager[k], out[k]), k
    return oc, code, dec, synd, out


def _properties(dec, synd, out, T, order, n):
    """Converged shots reproduce their syndrome, the others do not; the
    statistics stay in range."""
    st = out["stats"].cpu().numpy()
    back = dec.syndrome(out["ehat"]).cpu().numpy()
    same = np.all(back == synd.cpu().numpy(), axis=1)
    conv = st[:, 0] == 1
    assert np.array_equal(same, conv)
    assert np.all((st[:, 1] >= 0) & (st[:, 1] <= T))
    assert np.all((st[:, 3] >= 0) & (st[:, 3] <= T))
    assert np.all(st[:, 2] <= st[:, 3] * order) and np.all(st[:, 4] <= order)
    post = out["post"].cpu().numpy()
    assert np.all(np.isfinite(post))
    # decisions are the signs of the posteriors
    eh = np.unpackbits(out["ehat"].cpu().numpy().view(np.uint8), axis=1, bitorder="little")[:, :n]
    assert np.array_equal(eh.astype(bool), post < 0)
    return conv.mean()


@pytest.mark.parametrize("name,p,T,samples", [("M", 0.05, 50, 48), ("L", 0.03, 64, 0), ("L", 0.03, 3, 12)])
def test_full_size_sampled_parity(name, p, T, samples):
    """PSL(2,7) at its 64-round cap amplifies FP32 rounding by about 6 per
    non-converging round, so shot-by-shot parity there is not determined to
    the tolerance (its shots are ill-conditioned; the logical error rate test
    covers them): the sampled comparison runs the same launch at 3 rounds."""
    shots = 100_000
    oc, code, dec, synd, out = _decode_full(name, shots, p, T, seed=2024)
    conv = _properties(dec, synd, out, T, code.info.order, oc.n)
    if samples == 0:
        log(f"[full-size] {name} T={T}: {shots} shots, converged {conv:.3f}; properties hold on every shot")
        return
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(shots, size=samples, replace=False))
    s = synd.cpu().numpy().view(np.uint64)[idx]
    g = {k: out[k].cpu().numpy()[idx] for k in ("ehat", "post", "lam", "stats")}
    g["ehat"] = g["ehat"].view(np.uint64)
    lam = np.full(samples, float(channel_llr(p)))
    orc = oracle_decode_conditioned(oc, s, lam, max_iter_local=T, max_iter_global=T)
    res = compare(orc, g, oc.n)
    log(f"[full-size] {name}: {shots} shots, converged {conv:.3f}; {samples} sampled: {res['bad']} differ, "
        f"{res['tie']} ill-conditioned, worst ok |dLLR| {res['worst_ok']:.2e}")
    assert not res["unexplained"], res["detail"]
    assert res["tie"] <= samples // 2
