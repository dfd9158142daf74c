"""Depolarising noise on the PSL(2,7) code (n = 5376): X and Z parts decoded
independently, X errors with the Z checks and Z errors with the X checks,
each with the marginal prior 2p/3.  Over all shots the GPU's logical error
rate of each part, and of the pair, lies in the oracle's Wilson 95 % interval
on the same shots."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder, run_gpu, oracle_params
from lead_inputs import channel_llr, depolarizing_packed

pytestmark = pytest.mark.gpu


def _wilson(k, n, z=1.96):
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return c - h, c + h


def test_depolarising_logical_error_rate_in_oracle_ci():
    torch = torch_dev()
    spec, oc = code_pair("L")
    p, shots, T = 0.02, 200, 64
    xs, zs = depolarizing_packed(shots, oc.n, p, seed=17)
    lam = np.full(shots, float(channel_llr(2 * p / 3)), dtype=np.float32)
    fails_g, fails_o = [], []
    for t, e in ((0, xs), (1, zs)):
        code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, max_shots=shots)
        s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
        torch.cuda.synchronize()
        s = s.cpu().numpy().view(np.uint64)
        assert np.array_equal(s, oc.syndrome(e, t))
        g = run_gpu(dec, s, lam, 0)
        o = oc.decode(s, lam.astype(np.float64), t=t, p=oracle_params(max_iter_local=T, max_iter_global=T))
        fg = (g["stats"][:, 0] == 0) | oc.logical_failure(g["ehat"] ^ e, t)
        fo = (o["stats"][:, 0] == 0) | oc.logical_failure(o["ehat"] ^ e, t)
        lo, hi = _wilson(int(fo.sum()), shots)
        log(f"[depolarising] L p={p} {'XZ'[t]} errors: oracle {fo.mean():.3f} CI [{lo:.3f}, {hi:.3f}] "
            f"gpu {fg.mean():.3f}; same outcome on {(fg == fo).mean():.3f} of shots")
        assert lo <= fg.mean() <= hi
        fails_g.append(fg)
        fails_o.append(fo)
    fg, fo = fails_g[0] | fails_g[1], fails_o[0] | fails_o[1]
    lo, hi = _wilson(int(fo.sum()), shots)
    log(f"[depolarising] L p={p} either part fails: oracle {fo.mean():.3f} CI [{lo:.3f}, {hi:.3f}] gpu {fg.mean():.3f}")
    assert lo <= fg.mean() <= hi
