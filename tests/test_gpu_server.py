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


def _slot_bytes(P, decs, **kw):
    """Device bytes of one slot per decoder (a server with room for exactly
    that reports them)."""
    server = P.Server([d for _, _, d, _ in decs], mem_budget_bytes=1 << 40, max_slots_per_decoder=1, **kw)
    st = server.stats()
    server.close()
    return st["slot_bytes"]


def test_admission_by_device_memory():
    """A budget that cannot hold one slot per decoder is refused; a budget of
    exactly one slot per decoder serves with those slots alone; a budget with
    room for one more slot gives it to whichever decoder has shots waiting,
    freeing another decoder's idle extra slot when the budget is full; every
    result equals its lone decode."""
    import paper_2605_17796_amd as P
    decs = _setup(["T", "M"])
    base = _slot_bytes(P, decs, max_batch_shots=256)
    with pytest.raises(P.LeadError) as ei:
        P.Server([d for _, _, d, _ in decs], mem_budget_bytes=base - 1, max_batch_shots=256)
    assert P.STATUS_NAMES[ei.value.status] == "LEAD_E_CAPACITY" and "one launch slot per decoder" in str(ei.value)
    # exactly one slot per decoder: the server never grows
    server = P.Server([d for _, _, d, _ in decs], mem_budget_bytes=base, max_batch_shots=256,
                      max_slots_per_decoder=4)
    st0 = server.stats()
    assert st0["slots"] == 2 and st0["slot_bytes"] == base
    reqs = []
    for i in range(12):
        k = i % 2
        name, code, dec, oc = decs[k]
        synd, prior = _request(dec, oc, 300, seed=4000 + i)
        reqs.append((k, synd, prior, server.submit(k, synd, prior)))
    for k, synd, prior, t in reqs:
        server.wait(t)
        got = server.result(t, k, synd.shape[0])
        ref = _alone(decs[k][2], synd, prior)
        assert np.array_equal(got["ehat"], ref["ehat"].view(np.uint64)) and np.array_equal(got["stats"], ref["stats"])
    st = server.stats()
    server.close()
    assert st["slots"] == 2 and st["slots_created"] == 2 and st["slot_bytes"] <= base
    # room for one more A5 slot (the larger one): a burst of A5 requests
    # takes it, then a burst of D6 requests takes it back after it idles
    bm = _slot_bytes(P, decs[1:], max_batch_shots=256)
    server = P.Server([d for _, _, d, _ in decs], mem_budget_bytes=base + bm, max_batch_shots=256,
                      max_slots_per_decoder=2)
    st = server.stats()
    assert st["slots"] == 3 and st["slot_bytes"] <= base + bm
    for k in (1, 0):
        name, code, dec, oc = decs[k]
        batch = []
        for i in range(8):
            synd, prior = _request(dec, oc, 400, seed=5000 + 10 * k + i)
            batch.append((synd, prior, server.submit(k, synd, prior)))
        for synd, prior, t in batch:
            server.wait(t)
            got = server.result(t, k, synd.shape[0])
            ref = _alone(dec, synd, prior)
            assert np.array_equal(got["ehat"], ref["ehat"].view(np.uint64))
            assert np.array_equal(got["stats"], ref["stats"])
        assert server.stats()["slot_bytes"] <= base + bm
    st = server.stats()
    server.close()
    log(f"[server] admission: one slot per decoder {base} B, budget +1 A5 slot: {st}")
    assert st["evictions"] >= 1 and st["slots_created"] >= 4


def test_back_pressure_oversize_and_close():
    """Pending shots (submitted, not yet released) are bounded: a request
    larger than the bound is refused as oversize, one that would exceed it
    while others are pending is refused as busy and accepted once results
    are collected; refused submits queue nothing.  After lead_server_close
    (which waits for the admitted requests) submits are refused with
    LEAD_E_CLOSED and earlier results remain available."""
    import paper_2605_17796_amd as P
    decs = _setup(["M"])
    name, code, dec, oc = decs[0]
    server = P.Server([dec], max_batch_shots=512, max_pending_shots=1000)
    synd, prior = _request(dec, oc, 1001, seed=6000)
    with pytest.raises(P.LeadError) as ei:
        server.submit(0, synd, prior)
    assert P.STATUS_NAMES[ei.value.status] == "LEAD_E_CAPACITY" and "oversize" in str(ei.value)
    t1 = server.submit(0, synd[:700], prior[:700])
    with pytest.raises(P.LeadError) as ei:
        server.submit(0, synd[700:1001], prior[700:1001])   # 700 + 301 > 1000
    assert P.STATUS_NAMES[ei.value.status] == "LEAD_E_CAPACITY" and "busy" in str(ei.value)
    assert server.stats()["pending_shots"] == 700 and server.stats()["submitted"] == 1
    server.wait(t1)
    r1 = server.result(t1, 0, 700)
    t2 = server.submit(0, synd[700:1001], prior[700:1001])
    server.drain()
    assert server.poll(t2)
    with pytest.raises(P.LeadError) as ei:
        server.submit(0, synd[:10], prior[:10])
    assert P.STATUS_NAMES[ei.value.status] == "LEAD_E_CLOSED"
    r2 = server.result(t2, 0, 301)
    st = server.stats()
    server.close()
    ref = _alone(dec, synd, prior)
    assert np.array_equal(np.concatenate([r1["ehat"], r2["ehat"]]), ref["ehat"].view(np.uint64))
    assert st["refused"] == 2 and st["pending_shots"] == 0 and st["completed"] == 2
    log(f"[server] back-pressure and close: {st}")
