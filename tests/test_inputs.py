"""The seeded input generators: groups, generating sets, local codes, noise."""
import numpy as np
import pytest

from lead_inputs import (by_name, standard, pack_bits, unpack_bits, bitflip_packed,
                         depolarizing_packed, channel_llr, STANDARD)
from lead_inputs.codes import local_code_ok


@pytest.mark.parametrize("name,order,classes", [("D6", 12, 6), ("A5", 60, 5), ("PSL2_7", 168, 6),
                                                ("E2_3", 8, 8), ("Z5", 5, 5), ("D3", 6, 3)])
def test_group_tables(name, order, classes):
    g = by_name(name)
    assert g.order == order
    mul = g.mul.astype(np.int64)
    # Latin square, identity, associativity (brute force)
    assert all(len(set(row)) == order for row in mul)
    e = g.identity
    assert np.array_equal(mul[e], np.arange(order)) and np.array_equal(mul[:, e], np.arange(order))
    lhs = mul[mul[:, :, None], np.arange(order)[None, None, :]]           # (a b) c
    rhs = mul[np.arange(order)[:, None, None], mul[None, :, :]]            # a (b c)
    assert np.array_equal(lhs, rhs)
    assert len(set(g.conjugacy_class_ids())) == classes


@pytest.mark.parametrize("name", list(STANDARD))
def test_standard_instances_follow_sampling_rules(name):
    spec = standard(name)
    g = by_name(spec.group)
    inv = g.inverse()
    cls = g.conjugacy_class_ids()
    for S in (spec.A, spec.B):
        assert len(S) == spec.delta and len(set(S)) == spec.delta
        assert g.identity not in S
        assert set(int(inv[x]) for x in S) == set(S)
    # TNC: a g != g b for all a, b, g
    mul = g.mul.astype(np.int64)
    for a in spec.A:
        for b in spec.B:
            assert not np.any(mul[a, :] == mul[:, b])
    assert not set(cls[spec.A]) & set(cls[spec.B])
    assert local_code_ok(spec.GA, spec.delta) and local_code_ok(spec.GB, spec.delta)
    assert standard(name).A == spec.A  # deterministic


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    for n in (1, 63, 64, 65, 540, 1080):
        bits = rng.integers(0, 2, size=(7, n), dtype=np.uint8)
        w = pack_bits(bits)
        assert w.shape == (7, (n + 63) // 64)
        assert np.array_equal(unpack_bits(w, n), bits)
        # LSB-first convention
        i = n - 1
        assert ((w[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)).astype(np.uint8).tolist() == bits[:, i].tolist()


def test_noise_rates_and_determinism():
    e = bitflip_packed(4000, 1080, 0.05, seed=3)
    rate = unpack_bits(e, 1080).mean()
    assert abs(rate - 0.05) < 0.002
    assert np.array_equal(e, bitflip_packed(4000, 1080, 0.05, seed=3))
    assert not np.array_equal(e, bitflip_packed(4000, 1080, 0.05, seed=4))
    xs, zs = depolarizing_packed(4000, 96, 0.03, seed=1)
    bx, bz = unpack_bits(xs, 96), unpack_bits(zs, 96)
    assert abs((bx | bz).mean() - 0.03) < 0.003
    assert abs((bx & bz).mean() - 0.01) < 0.002
    assert np.isclose(float(channel_llr(0.05)), np.log(19.0), rtol=1e-7)


def test_device_noise_packing_and_rates():
    """The GPU-side generators (run here on the CPU device) pack bits exactly
    like pack_bits and draw flips at the stated rates; depolarising X and Z
    parts overlap on Y errors only (rate p/3)."""
    import torch
    from lead_inputs.noise_device import _pack, bitflip_packed_device, depolarizing_packed_device
    from lead_inputs import pack_bits, unpack_bits
    rng = np.random.default_rng(0)
    for n in (1, 63, 64, 65, 1080, 5376):
        bits = rng.random((7, n)) < 0.3
        got = _pack(torch.from_numpy(bits)).numpy().view(np.uint64)
        assert np.array_equal(got, pack_bits(bits.astype(np.uint8)))
    e = bitflip_packed_device(4000, 1080, 0.05, seed=3, device="cpu").numpy().view(np.uint64)
    rate = unpack_bits(e, 1080).mean()
    assert abs(rate - 0.05) < 4 * np.sqrt(0.05 * 0.95 / (4000 * 1080))
    ps = np.linspace(0.02, 0.08, 2000)
    e = unpack_bits(bitflip_packed_device(2000, 1080, ps, seed=4, device="cpu").numpy().view(np.uint64), 1080)
    assert np.corrcoef(e.mean(axis=1), ps)[0, 1] > 0.8
    xs, zs = depolarizing_packed_device(3000, 1080, 0.06, seed=5, device="cpu")
    x = unpack_bits(xs.numpy().view(np.uint64), 1080)
    z = unpack_bits(zs.numpy().view(np.uint64), 1080)
    tot = 3000 * 1080
    for r, want in ((x.mean(), 0.04), (z.mean(), 0.04), ((x & z).mean(), 0.02)):
        assert abs(r - want) < 4 * np.sqrt(want * (1 - want) / tot)
    # distinct draws per shot, same draws for the same seed
    a = bitflip_packed_device(50, 1080, 0.05, seed=9, device="cpu")
    b = bitflip_packed_device(50, 1080, 0.05, seed=9, device="cpu")
    assert torch.equal(a, b) and len({tuple(r) for r in a.tolist()}) == 50
