"""Write tests/golden/outcomes_*.json: per-shot outcomes of the FP64 oracle
(and only the oracle) on large seeded workloads, for the statistical parity
tests (logical error rate, converged share and mean global iterations of the
GPU inside the oracle's 95 % intervals on the same shots).

Workloads (code-capacity noise as in Sec. IV-A of the paper; the decoder is
LEAD with BP locally and globally, Algorithm 1):
  * A5 code (n = 1080), i.i.d. bit flips, p = 0.02 and 0.05, 50 + 50 rounds;
  * PSL(2,7) code (n = 5376), depolarising noise, p = 0.01, 0.02, 0.03 and
    0.05, 64 + 64 rounds, X errors decoded with the Z checks and Z errors with
    the X checks, each with the marginal prior 2p/3.

Every point is 10^4 shots.  Per shot the file keeps: converged (global BP
reached H e = s), logical failure (not converged, or the residual e + e_hat
is a non-trivial logical), global iterations and the sum of local
iterations.  Arrays are stored zlib-compressed and base64-encoded.

With --perturbed the same shots are decoded once more by the oracle with
every computed value multiplied by 1 + eps*xi (eps = 2.4e-7, a few FP32 ulps;
xi uniform in [-1, 1) from the oracle's seeded stream, seed 1), and the
outcomes are added to each part under "perturbed": a second correct
implementation whose rounding differs, which calibrates how far two correct
decoders drift apart shot by shot where min-sum is ill-conditioned.

Usage: python tests/golden/make_outcomes.py [--procs P] [--only NAME ...] [--perturbed]
"""
from __future__ import annotations

import argparse
import base64
import json
import os
import sys
import time
import zlib
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from lead_inputs import standard, bitflip_packed, depolarizing_packed, channel_llr  # noqa: E402

SHOTS = 10000
SHARD = 250
PERTURB = 2.4e-7
PERTURB_SEED = 1

# name -> (code, noise, p, rounds, seed)
POINTS = {
    "M_bitflip_p002": ("M", "bitflip", 0.02, 50, 101),
    "M_bitflip_p005": ("M", "bitflip", 0.05, 50, 102),
    "L_depol_p001": ("L", "depol", 0.01, 64, 201),
    "L_depol_p002": ("L", "depol", 0.02, 64, 202),
    "L_depol_p003": ("L", "depol", 0.03, 64, 203),
    "L_depol_p005": ("L", "depol", 0.05, 64, 205),
}


def point_inputs(name, shots=SHOTS):
    """Seeded errors of a point: a list of (check type, packed errors) and
    the per-shot prior (float32 LLR)."""
    code, noise, p, T, seed = POINTS[name]
    spec = standard(code)
    n = spec.order * spec.delta ** 2 // 2
    if noise == "bitflip":
        e = bitflip_packed(shots, n, p, seed)
        parts = [(0, e)]
        lam = np.full(shots, float(channel_llr(p)), dtype=np.float32)
    else:
        xs, zs = depolarizing_packed(shots, n, p, seed)
        parts = [(0, xs), (1, zs)]
        lam = np.full(shots, float(channel_llr(2 * p / 3)), dtype=np.float32)
    return spec, parts, lam


def _shard(args):
    name, t, s0, s1, pert = args
    from oracle import oracle as O
    code, noise, p, T, seed = POINTS[name]
    # the draws are sequential per shot, so the first s1 shots of a smaller
    # draw are the first s1 shots of the full one
    spec, parts, lam = point_inputs(name, s1)
    e = dict(parts)[t][s0:s1]
    oc = O.OracleCode.from_spec(spec)
    s = oc.syndrome(e, t)
    kw = dict(perturb=PERTURB, perturb_seed=PERTURB_SEED) if pert else {}
    o = oc.decode(s, lam[s0:s1].astype(np.float64), t=t,
                  p=O.params(max_iter_local=T, max_iter_global=T, **kw))
    conv = o["stats"][:, 0] != 0
    fail = ~conv | oc.logical_failure(o["ehat"] ^ e, t)
    return name, t, s0, conv, fail, o["stats"][:, 1].copy(), o["stats"][:, 2].copy()


def enc(a: np.ndarray) -> str:
    return base64.b64encode(zlib.compress(np.ascontiguousarray(a).tobytes(), 9)).decode()


def dec(s: str, dtype) -> np.ndarray:
    return np.frombuffer(zlib.decompress(base64.b64decode(s)), dtype=dtype)


def path_of(name):
    return os.path.join(HERE, f"outcomes_{name}.json")


def load(name):
    """Outcomes of a point: dict with per-part arrays conv, fail (bool),
    iters_g (int), iters_l_sum (int)."""
    with open(path_of(name)) as f:
        d = json.load(f)
    for part in d["parts"]:
        for x in [part] + ([part["perturbed"]] if "perturbed" in part else []):
            x["conv"] = dec(x["conv"], np.uint8).astype(bool)
            x["fail"] = dec(x["fail"], np.uint8).astype(bool)
            x["iters_g"] = dec(x["iters_g"], np.uint8).astype(np.int64)
            x["iters_l_sum"] = dec(x["iters_l_sum"], np.uint16).astype(np.int64)
    return d


def _arrays(conv, fail, ig, il):
    assert ig.max() <= 255 and il.max() < 65536
    return dict(conv=enc(conv.astype(np.uint8)), fail=enc(fail.astype(np.uint8)), iters_g=enc(ig.astype(np.uint8)),
                iters_l_sum=enc(il.astype(np.uint16)),
                summary=dict(converged=float(conv.mean()), failure=float(fail.mean()), mean_iters_g=float(ig.mean())))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*")
    ap.add_argument("--perturbed", action="store_true")
    args = ap.parse_args()
    names = args.only or list(POINTS)
    jobs = []
    for name in names:
        nparts = 1 if POINTS[name][1] == "bitflip" else 2
        for t in range(nparts):
            for s0 in range(0, SHOTS, SHARD):
                jobs.append((name, t, s0, min(SHOTS, s0 + SHARD), args.perturbed))
    res = {}
    t0 = time.time()
    with ProcessPoolExecutor(args.procs) as ex:
        for k, r in enumerate(ex.map(_shard, jobs)):
            res[(r[0], r[1], r[2])] = r[3:]
            if (k + 1) % 20 == 0:
                print(f"{k + 1}/{len(jobs)} shards, {time.time() - t0:.0f} s", flush=True)
    for name in names:
        code, noise, p, T, seed = POINTS[name]
        nparts = 1 if noise == "bitflip" else 2
        if args.perturbed:
            with open(path_of(name)) as f:
                out = json.load(f)
            for t in range(nparts):
                cols = [res[(name, t, s0)] for s0 in range(0, SHOTS, SHARD)]
                arr = _arrays(*(np.concatenate([c[i] for c in cols]) for i in range(4)))
                arr.update(perturb=PERTURB, perturb_seed=PERTURB_SEED)
                out["parts"][t]["perturbed"] = arr
            with open(path_of(name), "w") as f:
                json.dump(out, f, indent=1)
            print(name, "perturbed", [pt["perturbed"]["summary"] for pt in out["parts"]], flush=True)
            continue
        parts = []
        for t in range(nparts):
            cols = [res[(name, t, s0)] for s0 in range(0, SHOTS, SHARD)]
            parts.append(dict(check_type=t, errors="X" if t == 0 else "Z",
                              **_arrays(*(np.concatenate([c[i] for c in cols]) for i in range(4)))))
        out = dict(point=name, code=code, noise=noise, p=p, max_iter_local=T, max_iter_global=T, seed=seed,
                   shots=SHOTS, ms_scale=0.75, alpha=1.0, prior="ln((1-q)/q) in float32, q = p (bit flips) "
                   "or 2p/3 (depolarising)", writer="tests/golden/make_outcomes.py (oracle only)", parts=parts)
        with open(path_of(name), "w") as f:
            json.dump(out, f, indent=1)
        print(name, [pt["summary"] for pt in parts], flush=True)


if __name__ == "__main__":
    main()
