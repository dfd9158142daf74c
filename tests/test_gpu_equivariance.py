"""c-13 on the GPU: the decoder commutes with the translations of the
Cayley complex that preserve its local structure (Sec. I: the code's
topological symmetry).  g -> x g with x commuting with every element of A
maps square (g, a, b) to (x g, a, b) and check (g, rho) to (x g, rho);
g -> g y with y commuting with every element of B does the same on the
right.  Decoding the relabelled syndrome on the GPU and mapping the outputs
back gives the outputs of the original decode bit for bit, on every shot
(stronger than the 1e-3 bar): each view's arithmetic depends only on local
positions, lambda' is symmetric in the two views of a qubit, and a qubit's
two occurrences add the same two partial sums (IEEE addition commutes), so
no rounding depends on the vertex labels."""
import numpy as np
import pytest

from conftest import code_pair
from gpu_common import log, torch_dev, gpu_decoder, run_gpu
from lead_inputs import bitflip_packed, channel_llr, pack_bits, unpack_bits

pytestmark = pytest.mark.gpu


def _gpu_syndrome(dec, e):
    torch = torch_dev()
    s = dec.syndrome(torch.from_numpy(e.view(np.int64)).cuda())
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name,t,side,elem,T,shots", [("T", 0, "left", 3, 32, 300), ("T", 1, "left", 3, 32, 300),
                                                      ("T", 0, "right", 1, 32, 300), ("T", 1, "right", 2, 32, 300),
                                                      ("L", 0, "left", 21, 64, 200), ("L", 1, "right", 21, 64, 200)])
def test_gpu_decoder_commutes_with_translations(name, t, side, elem, T, shots):
    spec, _ = code_pair(name)
    mul = spec.mul.astype(np.int64)
    N = spec.order
    gens = spec.A if side == "left" else spec.B
    assert all(mul[elem, a] == mul[a, elem] for a in gens), "element does not commute with the generators"
    code, dec = gpu_decoder(spec, t=t, max_iter_local=T, max_iter_global=T, max_shots=shots)
    view = code.views(t)
    r = code.info.r[t]
    image = (lambda g: mul[elem, g]) if side == "left" else (lambda g: mul[g, elem])
    qperm = np.empty(code.n, dtype=np.int64)
    for g in range(N):
        qperm[view[g]] = view[image(g)]
    assert np.array_equal(np.sort(qperm), np.arange(code.n))
    cperm = np.array([image(g) * r + rho for g in range(N) for rho in range(r)])
    p = 0.06 if name == "T" else 0.02
    e = bitflip_packed(shots, code.n, p, seed=17)
    eb = unpack_bits(e, code.n)
    e2 = np.zeros_like(eb)
    e2[:, qperm] = eb
    s = _gpu_syndrome(dec, e)
    s2 = _gpu_syndrome(dec, pack_bits(e2))
    m = code.m(t)
    assert np.array_equal(unpack_bits(s2, m)[:, cperm], unpack_bits(s, m))
    lam = np.full(shots, float(channel_llr(p)), dtype=np.float32)
    a = run_gpu(dec, s, lam, 0, lam=True)
    b = run_gpu(dec, s2, lam, 0, lam=True)
    for k in ("post", "lam"):
        assert np.array_equal(b[k][:, qperm], a[k]), k
    assert np.array_equal(unpack_bits(b["ehat"], code.n)[:, qperm], unpack_bits(a["ehat"], code.n))
    assert np.array_equal(a["stats"], b["stats"])
    conv = float((a["stats"][:, 0] == 1).mean())
    log(f"[equivariance] {name} t={t} {side} x{elem}: {shots} shots bit-identical after relabelling "
        f"(converged {conv:.2f})")
