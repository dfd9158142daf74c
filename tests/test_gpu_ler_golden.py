"""Statistical parity at the full iteration caps (c-14): the GPU decodes the
same seeded 10^4-shot workloads as the stored FP64 oracle outcomes
(tests/golden/outcomes_*.json, written by tests/golden/make_outcomes.py from
the oracle alone).

Workloads: the A5 code under bit flips at p = 0.02 and 0.05 with 50 + 50
rounds, and the PSL(2,7) code under depolarising noise at p = 0.01, 0.02,
0.03 and 0.05 with 64 + 64 rounds (X and Z errors decoded independently with
the marginal prior 2p/3).

Two correct decoders that round differently need not agree shot by shot
where min-sum does not converge: a rounding difference grows by about
beta*(d-1) per iteration (x6 on PSL(2,7)), so after dozens of iterations the
two runs of a shot are unrelated.  The stored files therefore also hold the
outcomes of a second correct decoder, the oracle with every computed value
perturbed by a few FP32 ulps.  The checks, per check type and metric
(logical failure, converged, global iterations):
  * paired: the mean per-shot difference GPU - oracle lies within z standard
    errors of zero (z = 3.1: a 5 % family-wise level over the 24 checks, by
    Bonferroni); the perturbed oracle passes the same test against the
    plain one, which shows the bar is what a correct decoder meets;
  * the spec bar: the GPU's logical error rate lies in the oracle's
    Wilson 95 % interval, asserted wherever the perturbed oracle's rate lies
    in it too (where it does not, a correct decoder misses the interval, and
    the paired test stands alone);
  * on A5, where every shot is well-conditioned at these caps, the outcomes
    are identical shot by shot."""
import os
import sys

import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_outcomes as G  # noqa: E402

pytestmark = pytest.mark.gpu


def _wilson(k, n, z=1.96):
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return c - h, c + h


Z_PAIRED = 3.1


def _paired(tag, xg, xo, xp, what):
    """|mean(xg - xo)| <= Z se; the perturbed oracle xp must pass as well."""
    for name, x in (("gpu", xg), ("perturbed oracle", xp)):
        d = x.astype(np.float64) - xo.astype(np.float64)
        se = d.std(ddof=1) / np.sqrt(d.size) if np.any(d != 0) else 0.0
        log(f"[golden] {tag} {what}: {name} - oracle = {d.mean():+.4f} (se {se:.4f}, "
            f"{int((d != 0).sum())} shots differ)")
        assert abs(d.mean()) <= Z_PAIRED * se + 1e-12, f"{tag} {what}: {name}"


@pytest.mark.parametrize("point", list(G.POINTS))
def test_gpu_outcomes_in_oracle_intervals(point):
    torch = torch_dev()
    ref = G.load(point)
    code_name, noise, p, T, seed = G.POINTS[point]
    assert ref["shots"] == G.SHOTS and ref["seed"] == seed and ref["max_iter_global"] == T
    spec, parts, lam = G.point_inputs(point)
    spec_c, oc = code_pair(code_name)
    shots = G.SHOTS
    fails = []
    for (t, e), rp in zip(parts, ref["parts"]):
        assert rp["check_type"] == t
        pp = rp["perturbed"]
        code, dec = gpu_decoder(spec_c, t=t, max_iter_local=T, max_iter_global=T, max_shots=shots)
        synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
        prior = torch.from_numpy(lam).cuda()
        out = dec.decode(synd, prior, post=False)
        torch.cuda.synchronize()
        st = out["stats"].cpu().numpy()
        ehat = out["ehat"].cpu().numpy().view(np.uint64)
        conv = st[:, 0] != 0
        fail = ~conv | oc.logical_failure(ehat ^ e, t)
        ig = st[:, 1].astype(np.int64)
        tag = f"{point} {'XZ'[t]} errors"
        same = (conv == rp["conv"]) & (fail == rp["fail"]) & (ig == rp["iters_g"])
        same_p = (pp["conv"] == rp["conv"]) & (pp["fail"] == rp["fail"]) & (pp["iters_g"] == rp["iters_g"])
        log(f"[golden] {tag}: same (converged, failure, I_g) as the oracle on {same.mean():.4f} of {shots} shots "
            f"(perturbed oracle: {same_p.mean():.4f})")
        if code_name == "M":
            assert same.all(), f"{tag}: {int((~same).sum())} shots differ"
        _paired(tag, fail, rp["fail"], pp["fail"], "logical failure")
        _paired(tag, conv, rp["conv"], pp["conv"], "converged")
        _paired(tag, ig, rp["iters_g"], pp["iters_g"], "global iterations")
        lo, hi = _wilson(int(rp["fail"].sum()), shots)
        inside_p = lo <= pp["fail"].mean() <= hi
        log(f"[golden] {tag} logical error rate: oracle {rp['fail'].mean():.4f} CI [{lo:.4f}, {hi:.4f}] "
            f"gpu {fail.mean():.4f} perturbed oracle {pp['fail'].mean():.4f}")
        if inside_p:
            assert lo <= fail.mean() <= hi, f"{tag} logical error rate outside the oracle's interval"
        fails.append((fail, rp["fail"], pp["fail"]))
    if len(fails) == 2:
        fg, fo, fp = (fails[0][i] | fails[1][i] for i in range(3))
        _paired(f"{point} either part", fg, fo, fp, "logical failure")
