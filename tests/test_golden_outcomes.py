"""The stored oracle outcomes (tests/golden/outcomes_*.json) are what the
oracle computes: arrays of the stated size, consistent with the stopping rule
(a run that does not converge reports the cap; failure includes every shot
that does not converge), and a sample of shots re-decoded now by the oracle
reproduces its stored outcome exactly."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_outcomes as G  # noqa: E402


@pytest.mark.parametrize("point", list(G.POINTS))
def test_stored_outcomes_consistent(point):
    ref = G.load(point)
    code, noise, p, T, seed = G.POINTS[point]
    assert (ref["code"], ref["noise"], ref["p"], ref["max_iter_global"], ref["seed"]) == (code, noise, p, T, seed)
    assert len(ref["parts"]) == (1 if noise == "bitflip" else 2)
    for part in ref["parts"]:
        assert part["perturbed"]["perturb"] == G.PERTURB
        for x in (part, part["perturbed"]):
            conv, fail, ig = x["conv"], x["fail"], x["iters_g"]
            assert conv.size == fail.size == ig.size == x["iters_l_sum"].size == G.SHOTS
            assert np.all(fail[~conv]), "a shot that does not converge is a failure"
            assert np.all(ig[~conv] == T), "a run that does not converge reports the cap"
            assert np.all((ig >= 1) & (ig <= T))
            assert abs(x["summary"]["failure"] - fail.mean()) < 1e-12


@pytest.mark.parametrize("point", list(G.POINTS))
def test_stored_outcomes_reproduced_by_oracle(point):
    from oracle import oracle as O
    ref = G.load(point)
    code, noise, p, T, seed = G.POINTS[point]
    idx = np.arange(0, 12 if code == "L" else 60)
    spec, parts, lam = G.point_inputs(point, int(idx[-1]) + 1)
    oc = O.OracleCode.from_spec(spec)
    for (t, e), part in zip(parts, ref["parts"]):
        e = e[idx]
        o = oc.decode(oc.syndrome(e, t), lam[idx].astype(np.float64), t=t,
                      p=O.params(max_iter_local=T, max_iter_global=T))
        conv = o["stats"][:, 0] != 0
        fail = ~conv | oc.logical_failure(o["ehat"] ^ e, t)
        assert np.array_equal(conv, part["conv"][idx])
        assert np.array_equal(fail, part["fail"][idx])
        assert np.array_equal(o["stats"][:, 1], part["iters_g"][idx])
        assert np.array_equal(o["stats"][:, 2], part["iters_l_sum"][idx])
