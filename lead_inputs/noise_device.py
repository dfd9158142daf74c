"""Seeded channel noise drawn on the GPU (for throughput runs of 10^5..10^6
distinct shots, where host draws would take minutes).

Same noise models as lead_inputs.noise -- i.i.d. bit flips with probability
p per qubit (p scalar or per shot), and depolarising noise (X, Y, Z each with
probability p/3) -- drawn from torch's seeded GPU generator in shot chunks,
so every shot is a distinct draw.  The draws differ from the host PCG64
streams of lead_inputs.noise (the tests compare against the oracle with
those); only the distribution is the same.  Bit packing is LSB-first: bit i
of a row lives in word i // 64 at position i % 64.  No decoding arithmetic.
"""
from __future__ import annotations

CHUNK_ELEMS = 1 << 28   # uniforms per chunk (1 GiB of float32)


def _pack(bits):
    """bool [S, n] on the GPU -> int64 [S, ceil(n/64)] packed LSB-first."""
    import torch
    s, n = bits.shape
    w = (n + 63) // 64
    if w * 64 != n:
        bits = torch.nn.functional.pad(bits, (0, w * 64 - n))
    b = bits.view(s, w, 2, 32).to(torch.int64)
    weights = torch.ones(32, dtype=torch.int64, device=bits.device) << torch.arange(32, device=bits.device)
    halves = (b * weights).sum(dim=3)                     # [S, w, 2], each < 2^32
    return halves[:, :, 0] | (halves[:, :, 1] << 32)


def _chunks(shots, n):
    step = max(1, CHUNK_ELEMS // max(n, 1))
    for s0 in range(0, shots, step):
        yield s0, min(shots, s0 + step)


def bitflip_packed_device(shots: int, n: int, p, seed: int, device="cuda"):
    """Packed i.i.d. bit-flip errors [shots, ceil(n/64)] int64 on `device`;
    `p` is a float or a per-shot sequence/tensor."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty((shots, (n + 63) // 64), dtype=torch.int64, device=device)
    pt = None if isinstance(p, (int, float)) else torch.as_tensor(p, dtype=torch.float32, device=device)
    for s0, s1 in _chunks(shots, n):
        u = torch.rand((s1 - s0, n), generator=g, device=device)
        thr = float(p) if pt is None else pt[s0:s1, None]
        out[s0:s1] = _pack(u < thr)
        del u
    return out


def depolarizing_packed_device(shots: int, n: int, p: float, seed: int, device="cuda"):
    """Depolarising noise: packed (x_part, z_part) int64 tensors; a Y error
    sets both.  Each qubit: X, Y, Z with probability p/3 each."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    w = (n + 63) // 64
    xs = torch.empty((shots, w), dtype=torch.int64, device=device)
    zs = torch.empty((shots, w), dtype=torch.int64, device=device)
    t1, t2, t3 = p / 3.0, 2 * p / 3.0, p
    for s0, s1 in _chunks(shots, n):
        u = torch.rand((s1 - s0, n), generator=g, device=device)
        is_y = (u >= t1) & (u < t2)
        xs[s0:s1] = _pack((u < t1) | is_y)
        zs[s0:s1] = _pack(((u >= t2) & (u < t3)) | is_y)
        del u, is_y
    return xs, zs
