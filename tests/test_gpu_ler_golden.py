"""Statistical parity at the full iteration caps (c-14): the GPU decodes the
same seeded 10^4-shot workloads as the stored FP64 oracle outcomes
(tests/golden/outcomes_*.json, written by tests/golden/make_outcomes.py from
the oracle alone), and its logical error rate and converged share lie in the
oracle's Wilson 95 % intervals and its mean global iteration count in the
oracle's normal 95 % interval, for every check type and for the depolarising
pair (a shot fails if either part fails).

Workloads: the A5 code under bit flips at p = 0.02 and 0.05 with 50 + 50
rounds, and the PSL(2,7) code under depolarising noise at p = 0.01, 0.02,
0.03 and 0.05 with 64 + 64 rounds (X and Z errors decoded independently with
the marginal prior 2p/3).  Per-shot agreement of (converged, failure, global
iterations) is reported beside the intervals; shots whose min-sum runs are
ill-conditioned (rounding differences grow by a factor of beta*(d-1) per
iteration) may differ one by one, which the intervals absorb."""
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


def _mean_ci(x, z=1.96):
    x = np.asarray(x, dtype=np.float64)
    h = z * x.std(ddof=1) / np.sqrt(x.size) if x.size > 1 else 0.0
    return x.mean() - h, x.mean() + h


def _check(tag, fg, fo, what):
    lo, hi = _wilson(int(fo.sum()), fo.size)
    log(f"[golden] {tag} {what}: oracle {fo.mean():.4f} CI [{lo:.4f}, {hi:.4f}] gpu {fg.mean():.4f}")
    assert lo <= fg.mean() <= hi, f"{tag} {what}"


@pytest.mark.parametrize("point", list(G.POINTS))
def test_gpu_outcomes_in_oracle_intervals(point):
    torch = torch_dev()
    ref = G.load(point)
    code_name, noise, p, T, seed = G.POINTS[point]
    assert ref["shots"] == G.SHOTS and ref["seed"] == seed and ref["max_iter_global"] == T
    spec, parts, lam = G.point_inputs(point)
    spec_c, oc = code_pair(code_name)
    shots = G.SHOTS
    fails_g, fails_o = [], []
    for (t, e), rp in zip(parts, ref["parts"]):
        assert rp["check_type"] == t
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
        log(f"[golden] {tag}: same (converged, failure, I_g) on {same.mean():.4f} of {shots} shots")
        _check(tag, fail, rp["fail"], "logical error rate")
        _check(tag, conv, rp["conv"], "converged share")
        lo, hi = _mean_ci(rp["iters_g"])
        log(f"[golden] {tag} mean I_g: oracle {rp['iters_g'].mean():.3f} CI [{lo:.3f}, {hi:.3f}] gpu {ig.mean():.3f}")
        assert lo <= ig.mean() <= hi, f"{tag} mean I_g"
        fails_g.append(fail)
        fails_o.append(rp["fail"])
    if len(fails_g) == 2:
        _check(f"{point} either part", fails_g[0] | fails_g[1], fails_o[0] | fails_o[1], "logical error rate")
