"""Serving loop: requests admitted while others are on the GPU are packed
into launch slots with other requests, and each result equals the result of
decoding that request alone."""
import threading

import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder
from lead_inputs import bitflip_packed, channel_llr, uniform_p, unpack_bits

pytestmark = pytest.mark.gpu

ROUNDS = {"T": 32, "M": 50, "L": 64}


def _setup(names, max_shots=8192):
    out = []
    for name in names:
        spec, oc = code_pair(name)
        code, dec = gpu_decoder(spec, max_iter_local=ROUNDS[name], max_iter_global=ROUNDS[name],
                                max_shots=max_shots)
        out.append((name, code, dec, oc))
    return out


def _request(dec, oc, shots, seed):
    torch = torch_dev()
    ps = uniform_p(shots, 0.02, 0.08, seed)
    e = bitflip_packed(shots, oc.n, ps, seed)
    synd = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return synd.cpu().numpy().view(np.uint64), channel_llr(ps).astype(np.float32)


def _alone(dec, synd, prior):
    torch = torch_dev()
    out = dec.decode(torch.from_numpy(synd.view(np.int64)).cuda(), torch.from_numpy(prior).cuda())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("posteriors", [False, True])
def test_each_served_result_equals_alone(posteriors):
    import paper_2605_17796_amd as P
    decs = _setup(["T", "M", "L"])
    server = P.Server([d for _, _, d, _ in decs], max_batch_shots=512, max_slots_per_decoder=3,
                      return_posteriors=posteriors)
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(40):
        k = int(rng.integers(0, 3))
        name, code, dec, oc = decs[k]
        shots = int(rng.integers(1, 1300 if name != "L" else 40))
        synd, prior = _request(dec, oc, shots, seed=1000 + i)
        reqs.append((k, synd, prior, server.submit(k, synd, prior)))
    for k, synd, prior, ticket in reqs:
        server.wait(ticket)
        got = server.result(ticket, k, synd.shape[0])
        ref = _alone(decs[k][2], synd, prior)
        assert np.array_equal(got["ehat"], ref["ehat"].view(np.uint64))
        assert np.array_equal(got["stats"], ref["stats"])
        if posteriors:
            assert np.array_equal(got["post"], ref["post"])
        assert got["done_ns"] >= got["submit_ns"]
    st = server.stats()
    server.close()
    assert st["completed"] == 40 and st["submitted"] == 40
    log(f"[server] 40 mixed requests (posteriors={posteriors}) equal their alone decodes; {st}")


def test_concurrent_submitters():
    import paper_2605_17796_amd as P
    decs = _setup(["T", "M"])
    server = P.Server([d for _, _, d, _ in decs], max_batch_shots=256)
    results = {}
    errors = []

    def client(k, base):
        name, code, dec, oc = decs[k]
        try:
            for i in range(10):
                synd, prior = _request(dec, oc, 50 + 37 * i, seed=base + i)
                t = server.submit(k, synd, prior)
                results[(k, i)] = (synd, prior, t)
        except Exception as exc:            # noqa: BLE001
            errors.append(exc)

    ths = [threading.Thread(target=client, args=(k, 5000 + 100 * k)) for k in (0, 1)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errors
    for (k, i), (synd, prior, t) in results.items():
        server.wait(t)
        got = server.result(t, k, synd.shape[0])
        ref = _alone(decs[k][2], synd, prior)
        assert np.array_equal(got["ehat"], ref["ehat"].view(np.uint64))
        assert np.array_equal(got["stats"], ref["stats"])
    server.close()


def test_server_argument_errors():
    import paper_2605_17796_amd as P
    decs = _setup(["T"])
    server = P.Server([decs[0][2]])
    with pytest.raises(P.LeadError):
        server.submit(3, np.zeros((1, 1), np.uint64), np.zeros(1, np.float32))
    with pytest.raises(P.LeadError):
        server.poll(12345)
    server.close()
