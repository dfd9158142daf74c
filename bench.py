"""Benchmark: decoded shots/s of the LEAD decoder on one MI355X.

Workload (the configuration the headline metric is quoted on): the A_5 code
(order 60, Delta = 6, [6,3] local codes, n = 1080, m = 540 Z checks), i.i.d.
bit flips with p = 0.05, channel LLR ln(19) per shot, min-sum scale 0.75,
alpha = 1, at most 50 local and 50 global iterations, 10^5 shots per step.
One step = one full LEAD decode of a batch already resident in HBM: local BP
on all 60 vertex views of every shot, alpha-regularised aggregation, global
BP, and the outputs (packed e_hat, FP32 posterior LLRs, per-shot statistics)
written back to HBM.  Every step decodes a different batch.

Prints one JSON line.  See the design doc for the roofline and baseline
definitions.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P_FLIP = 0.05
ROUNDS = 50
SHOTS = 100_000
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: non-packed FP32/INT VALU lane-ops
VALU_PEAK_GOPS = 256 * 64 * 2.4
# Lane operations counted per edge update of min-sum (check update of one
# edge plus its share of the variable update); see the design doc.
OPS_PER_EDGE_UPDATE = 10
KERNEL_SRC = os.path.join(ROOT, "paper_2605_17796_amd", "csrc", "lead_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "decode_kernel_A5_p005_traffic.json")


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def algorithmic_bytes_per_shot(n: int, m: int) -> float:
    # syndrome in (m bits) + prior (4 B) + e_hat out (n bits) + L_post out
    # (4n B) + statistics out (5 x 4 B)
    return m / 8 + 4 + n / 8 + 4 * n + 20


def cpu_baseline(spec, shots_sample: int, seed: int, workers: int):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload, in independent worker processes."""
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        per = [shots_sample // workers + (1 if i < shots_sample % workers else 0) for i in range(workers)]
        jobs = [(spec.group, spec.delta, spec.kA, spec.kB, spec.seed, k, seed + i) for i, k in enumerate(per)]
        done = sum(pool.map(_oracle_worker, jobs))
    wall = time.time() - t0
    return done / wall, wall


def _oracle_worker(job):
    group, delta, kA, kB, cseed, shots, seed = job
    sys.path.insert(0, ROOT)
    from lead_inputs import sample_code, bitflip_packed, channel_llr
    from oracle import oracle as O
    spec = sample_code(group, delta, kA, kB, cseed)
    oc = O.OracleCode.from_spec(spec)
    e = bitflip_packed(shots, oc.n, P_FLIP, seed)
    s = oc.syndrome(e)
    oc.decode(s, np.full(shots, float(channel_llr(P_FLIP))),
              p=O.params(max_iter_local=ROUNDS, max_iter_global=ROUNDS))
    return shots


def copy_probe():
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")      # 1 GiB
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": x.numel() * 4, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shots", type=int, default=SHOTS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3200)
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the plain per-round-launch form timed for comparison (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); shots are independent, "
              "so a multi-GPU run would shard batches with nothing exchanged.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_17796_amd as P
    from lead_inputs import standard, bitflip_packed, channel_llr

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    spec = standard("M")
    code = P.Code.from_spec(spec)
    n, m = code.n, code.m()
    shots = args.shots
    dec = P.Decoder(code, max_shots=shots, max_iter_local=ROUNDS, max_iter_global=ROUNDS, ms_scale=0.75,
                    alpha=1.0)

    # A pool of distinct error batches, resident on the GPU: step i decodes
    # batch i mod pool.
    pool_batches = 4
    synd_pool = []
    for b in range(pool_batches):
        e = bitflip_packed(shots, n, P_FLIP, seed=1000 + b)
        synd_pool.append(dec.syndrome(torch.from_numpy(e.view(np.int64)).to(dev)))
    lam = torch.full((shots,), float(channel_llr(P_FLIP)), dtype=torch.float32, device=dev)
    out = dec.alloc_outputs(shots, dev)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        dec.decode(synd_pool[i % pool_batches], lam, out=out)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    stats_acc = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        dec.decode(synd_pool[i % pool_batches], lam, out=out)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    st = out["stats"].cpu().numpy()
    stats_acc.append(st)

    ms_per_step = wall * 1000.0 / args.steps
    value = shots / (wall / args.steps)
    k_ms = float(np.mean(kernel_ms))

    # edge updates actually performed in the last step (local: every view of
    # every shot runs its own count; global: every edge of the shot's graph)
    info = code.info
    eloc = info.eloc[0]
    edge_updates = float(st[:, 2].astype(np.float64).sum() * eloc +
                         st[:, 1].astype(np.float64).sum() * eloc * info.order)
    bytes_launch = algorithmic_bytes_per_shot(n, m) * shots
    hbm_gbs = bytes_launch / (k_ms * 1e-3) / 1e9
    valu_gops = OPS_PER_EDGE_UPDATE * edge_updates / (k_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_sha") == kernel_hash() and rec.get("shots") == shots:
            traffic = rec.get("hbm_bytes_per_launch")

    hbm_frac = hbm_gbs / HBM_PEAK_GBS
    valu_frac = valu_gops / VALU_PEAK_GOPS
    if hbm_frac >= valu_frac:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4), "traffic": traffic}
    else:
        roof = {"bound": "alu", "achieved": round(valu_gops / 1000, 3), "peak": round(VALU_PEAK_GOPS / 1000, 2),
                "unit": "TOP/s", "frac": round(valu_frac, 4), "traffic": traffic}

    plain = None
    if args.plain_steps > 0:
        dec.decode(synd_pool[0], lam, out=out, plain=True)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for i in range(args.plain_steps):
            dec.decode(synd_pool[i % pool_batches], lam, out=out, plain=True)
        torch.cuda.synchronize()
        pw = (time.perf_counter() - tp) / args.plain_steps
        plain = {"shots_per_s": round(shots / pw, 1), "ms_per_step": round(pw * 1000, 3),
                 "form": "lead_decode_plain: Phases 1-2 launch, one launch per global round with state in HBM "
                         "and a host-visible convergence count, finalize launch",
                 "fused_over_plain": round(value * pw / shots, 3)}

    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        sample = args.cpu_sample
        rate, cwall = cpu_baseline(spec, sample, seed=7, workers=workers)
        cpu = {"value": round(rate, 1), "unit": "decoded shots/s", "cores": workers, "kind": "oracle",
               "sample": f"{sample} shots of the same workload (A5 code, p=0.05, 50+50 rounds), FP64 oracle, "
                         f"{workers} worker processes, {cwall:.1f} s wall"}

    line = {
        "metric": "decoded shots/sec at n~1080, p=0.05",
        "value": round(value, 1),
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "LEAD-BP full decode, A5 code n=1080 (Delta=6, [6,3] local codes), "
                               "bit-flip p=0.05, <=50 local + <=50 global min-sum rounds, beta=0.75, alpha=1",
                   "shots_per_step": shots, "form": "fused single launch (lead_decode)"},
        "kernel_ms": round(k_ms, 3),
        "roofline": roof,
        "hbm_frac": round(hbm_frac, 4),
        "valu_frac": round(valu_frac, 4),
        "decode_stats": {"converged": round(float((st[:, 0] == 1).mean()), 4),
                         "mean_global_iters": round(float(st[:, 1].mean()), 2),
                         "mean_local_iters": round(float(st[:, 2].mean() / 60.0), 2)},
        "plain_form": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
