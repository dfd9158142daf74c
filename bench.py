"""Benchmark: decoded shots/s of the LEAD decoder on one MI355X.

Headline workload: the A_5 code (order 60, Delta = 6, [6,3] local codes,
n = 1080, m = 540 Z checks), i.i.d. bit flips with p = 0.05, channel LLR
ln(19) per shot, min-sum scale 0.75, alpha = 1, at most 50 local and 50
global iterations, 10^5 shots per step.  One step = one full LEAD decode of
a batch already resident in HBM (local BP on all 60 vertex views of every
shot, alpha-regularised aggregation, global BP, and e_hat, FP32 posterior
LLRs and per-shot statistics written back to HBM), replayed as a captured
graph with the autotuned schedule.  Every step decodes a different batch.

Reported beside it (same GPU, identical outputs): the plain per-round-launch
form on the same batches and the same compiled kernels, and the same decode
eager on one stream; a mixed-code batch (D6 / A5 / PSL(2,7) codes with
10^3 / 3*10^4 / 10^5 shots, p ~ U[0.02, 0.08] per shot) as one graph launch
vs plain per-code launches; the PSL(2,7) code under depolarising noise at
10^6 shots per p; the serving loop fed Poisson request streams (batch sizes
log-uniform in 1..4096) with p50/p99 latency per code; the dominant kernel's
roofline and the whole decode's HBM fraction; and the FP64 oracle on the host
cores.  Every reported shot is a distinct error draw (drawn on the GPU for
the throughput legs).

Prints one JSON line.
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
ROUNDS = {"T": 32, "M": 50, "L": 64}
SHOTS = 100_000
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: non-packed FP32/INT VALU lane-ops
VALU_PEAK_GOPS = 256 * 64 * 2.4
# Lane operations counted per edge update of min-sum (check update of one
# edge plus its share of the variable update).
OPS_PER_EDGE_UPDATE = 10
# Fixed-point exit of the decoders: local BP runs only.  Ending a run whose
# messages reproduce themselves changes no output; in Phase 1 it ends most
# of the views that run to the cap, in global BP few runs (the A5 headline:
# Phases 2-3 take about as long with the exit as without), and testing it
# there costs a comparison per message and round.
FIXED_POINT = 2
CSRC = os.path.join(ROOT, "paper_2605_17796_amd", "csrc")
# sources of the kernels compiled for the code (device code and its generator)
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("lead_spec.hpp", "lead_device.hpp", "lead_args.hpp", "lead_jit.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lead_spec_global_A5_p005_traffic.json")
COUNTER_FILE = os.path.join(ROOT, "profiles", "lead_spec_global_A5_p005_valu.json")
# schedule of the headline when the autotuner is skipped (--schedule overrides)
DEFAULT_SCHEDULE = {"specialized": 2, "local_chunk": 256}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_shot(n: int, m: int) -> float:
    # the decode's own I/O: syndrome in (m bits) + prior (4 B) + e_hat out
    # (n bits) + L_post out (4n B) + statistics out (32 B)
    return m / 8 + 4 + n / 8 + 4 * n + 32


def global_kernel_bytes_per_shot(n: int, m: int, order: int, d2: int) -> float:
    # Phases 2-3 kernel: local posteriors in (order * d2 * 4 B) and their
    # flags (order * 4 B), syndrome in, e_hat + L_post + statistics out
    return order * d2 * 4 + order * 4 + m / 8 + n / 8 + 4 * n + 32


def edge_updates(stats: np.ndarray, eloc: int, order: int):
    """Min-sum edge updates of a decode, (Phase 1, Phase 3): every local run
    updates the E_loc edges of its view once per iteration, every global
    iteration the order * E_loc edges of the global graph."""
    return (float(stats[:, 2].astype(np.float64).sum() * eloc),
            float(stats[:, 1].astype(np.float64).sum() * eloc * order))


# ---------------------------------------------------------------------------
# CPU baseline (FP64 oracle, test infrastructure)
# ---------------------------------------------------------------------------

def cpu_baseline(spec, shots_sample: int, seed: int, workers: int):
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        per = [shots_sample // workers + (1 if i < shots_sample % workers else 0) for i in range(workers)]
        jobs = [(spec.group, spec.delta, spec.kA, spec.kB, spec.seed, k, seed + i) for i, k in enumerate(per)]
        done = sum(pool.map(_oracle_worker, jobs))
    wall = time.time() - t0
    return done / wall, wall


def host_facts():
    """nproc, the CPU model name and the physical core count of this host."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None and core is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model, "physical_cores": len(cores) or None}


def cpu_latency(spec, shots: int, seed: int):
    """Median wall time of one oracle decode of one shot, in one process."""
    from lead_inputs import bitflip_packed, channel_llr
    from oracle import oracle as O
    oc = O.OracleCode.from_spec(spec)
    e = bitflip_packed(shots, oc.n, P_FLIP, seed)
    s = oc.syndrome(e)
    prm = O.params(max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"])
    lam = np.full(1, float(channel_llr(P_FLIP)))
    t = []
    for i in range(shots):
        t0 = time.perf_counter()
        oc.decode(s[i:i + 1], lam, p=prm)
        t.append(time.perf_counter() - t0)
    return float(np.median(t)) * 1e3


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
              p=O.params(max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"]))
    return shots


def copy_probe():
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")      # 1 GiB
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": x.numel() * 4, "launches": 3}), flush=True)


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def make_decoder(P, name, max_shots, t=0):
    from lead_inputs import standard
    code = P.Code.from_spec(standard(name))
    dec = P.Decoder(code, t=t, max_shots=max_shots, max_iter_local=ROUNDS[name], max_iter_global=ROUNDS[name],
                    fixed_point_stop=FIXED_POINT, ms_scale=0.75, alpha=1.0)
    return code, dec


def syndromes(torch, dec, n, shots, p, seed):
    """Device syndromes of `shots` distinct seeded bit-flip errors (p scalar
    or per shot), drawn on the GPU."""
    from lead_inputs.noise_device import bitflip_packed_device
    e = bitflip_packed_device(shots, n, p, seed)
    s = dec.syndrome(e)
    del e
    return s


def timed(torch, fn, reps):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(reps):
        ev[i][0].record(stream)
        fn(i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in ev]


def served_stream(P, decs, requests, offered_shots_per_s, seed, names=None):
    """Feed `requests` [(decoder index, synd, prior)] to a fresh server at
    Poisson arrival times for the offered load; returns throughput and
    latency percentiles."""
    server = P.Server(list(decs), mem_budget_bytes=8 << 30, max_batch_shots=8192, max_slots_per_decoder=4)
    rng = np.random.default_rng(seed)
    mean_shots = np.mean([r[1].shape[0] for r in requests])
    rate = offered_shots_per_s / mean_shots
    gaps = rng.exponential(1.0 / rate, size=len(requests))
    tickets = []
    due = time.perf_counter()
    for (k, synd, prior), gap in zip(requests, gaps):
        due += gap
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        tickets.append((k, synd.shape[0], server.submit(k, synd, prior)))
    lat, codes, first, last, shots = [], [], None, None, 0
    for k, n, t in tickets:
        server.wait(t)
        r = server.result(t, k, n)
        lat.append((r["done_ns"] - r["submit_ns"]) / 1e6)
        codes.append(k)
        first = r["submit_ns"] if first is None else min(first, r["submit_ns"])
        last = r["done_ns"] if last is None else max(last, r["done_ns"])
        shots += n
    st = server.stats()
    server.close()
    span = (last - first) / 1e9
    lat, codes = np.array(lat), np.array(codes)
    res = {"offered_shots_per_s": offered_shots_per_s, "requests": len(requests), "shots": shots,
           "shots_per_s": round(shots / span, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3), "launches": st["launches"], "slots": st["slots"]}
    if names is not None and len(names) > 1:
        res["per_code"] = {names[k]: {"requests": int((codes == k).sum()),
                                      "p50_ms": round(float(np.percentile(lat[codes == k], 50)), 3),
                                      "p99_ms": round(float(np.percentile(lat[codes == k], 99)), 3)}
                           for k in range(len(names)) if (codes == k).any()}
    return res


def request_mix(torch, decs_named, n_requests, seed, codes):
    """Requests with log-uniform batch sizes in 1..4096, codes uniform over
    `codes`, per-request p ~ U[0.02, 0.08]; host copies of syndromes and
    per-shot priors."""
    from lead_inputs import channel_llr
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(0, np.log(4097), size=n_requests))).astype(int)
    ks = rng.integers(0, len(codes), size=n_requests)
    ps = rng.uniform(0.02, 0.08, size=n_requests)
    pools = {}
    for k in range(len(codes)):
        code, dec = decs_named[codes[k]]
        sel = ks == k
        if not sel.any():
            continue
        pp = np.repeat(ps[sel], sizes[sel])
        s = syndromes(torch, dec, code.n, int(sizes[sel].sum()), pp, seed=seed * 7 + k)
        pools[k] = (s.cpu().numpy().view(np.uint64), channel_llr(pp))
    off = {k: 0 for k in pools}
    reqs = []
    for k, n in zip(ks, sizes):
        s, pr = pools[int(k)]
        o = off[int(k)]
        reqs.append((int(k), s[o:o + n], pr[o:o + n]))
        off[int(k)] = o + n
    return reqs


def osd_only():
    """LEAD followed by global OSD-0 and by the order-3 sweep, one decode
    each after a warm-up, on the A5 headline batch (rows of H in registers)
    and on PSL(2,7) X errors at depolarising p = 0.03 (matrix in device
    memory); prints the time and the shots OSD resolved."""
    import torch
    import paper_2605_17796_amd as P
    from lead_inputs import channel_llr, standard
    from lead_inputs.noise_device import depolarizing_packed_device
    torch.cuda.set_device(0)
    res = {}
    for name, shots in (("M", SHOTS), ("L", 20_000)):
        code = P.Code.from_spec(standard(name))
        for order in (0, 3):
            dec = P.Decoder(code, max_shots=shots, max_iter_local=ROUNDS[name], max_iter_global=ROUNDS[name],
                            fixed_point_stop=FIXED_POINT, global_post=1, osd_order=order)
            if name == "M":
                synd = syndromes(torch, dec, code.n, shots, P_FLIP, seed=1000)
                lam = torch.full((shots,), float(channel_llr(P_FLIP)), dtype=torch.float32, device="cuda")
            else:
                xs, _ = depolarizing_packed_device(shots, code.n, 0.03, seed=3000)
                synd = dec.syndrome(xs)
                lam = torch.full((shots,), float(channel_llr(0.02)), dtype=torch.float32, device="cuda")
            out = dec.alloc_outputs(shots)
            dec.decode(synd[:256], lam[:256], out={k: (v[:256] if v is not None else None) for k, v in out.items()})
            w, _ = timed(torch, lambda i: dec.decode(synd, lam, out=out), 1)
            st = out["stats"].cpu().numpy()
            res[f"{name}_order{order}"] = {"shots": shots, "ms": round(w * 1e3, 3),
                                           "resolved_by_osd": int((st[:, 0] == 2).sum()),
                                           "form": dec.get_schedule()["global_osd_form"]}
            del dec, out
    print(json.dumps({"osd_only": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shots", type=int, default=SHOTS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000)
    ap.add_argument("--large-shots", type=int, default=1_000_000,
                    help="shots per p of the PSL(2,7) depolarising leg")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-code batch leg")
    ap.add_argument("--no-served", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the sum-product / alpha sweep / depolarising legs")
    ap.add_argument("--no-baseline-decoder", action="store_true",
                    help="skip the global-BP-only (single-stage) comparison leg")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the eager pass used for the roofline, with --schedule (for profilers)")
    ap.add_argument("--schedule", type=str, default=None,
                    help="JSON schedule of the headline instead of the autotuner's choice")
    ap.add_argument("--code", choices=("M", "L"), default="M",
                    help="with --roofline-only: M = the A5 headline (p = 0.05, 50 + 50 rounds), L = the PSL(2,7) "
                         "code (p = 0.03, 64 + 64 rounds, 5*10^4 shots)")
    ap.add_argument("--check-type", type=int, choices=(0, 1), default=0,
                    help="with --roofline-only: the check type decoded (0: Z checks, 1: X checks)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates the HBM byte counters)")
    ap.add_argument("--osd-only", action="store_true",
                    help="only decodes with global OSD (OSD-0, then the order-3 sweep): A5 headline batch, and "
                         "PSL(2,7) depolarising p = 0.03 (X part, 2*10^4 shots), for profilers")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.osd_only:
        osd_only()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); shots are independent, "
              "so a multi-GPU run would shard batches with nothing exchanged.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_17796_amd as P
    from lead_inputs import channel_llr

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if (args.code != "M" or args.check_type != 0) and not args.roofline_only:
        raise SystemExit("--code and --check-type select the workload of --roofline-only")
    cname = args.code
    shots = args.shots if cname == "M" else min(args.shots, 50_000)
    pflip = P_FLIP if cname == "M" else 0.03
    code, dec = make_decoder(P, cname, shots, args.check_type)
    n, m = code.n, code.m(args.check_type)
    info = code.info

    pool_batches = 4
    synd_pool = [syndromes(torch, dec, n, shots, pflip, seed=1000 + b) for b in range(pool_batches)]
    lam = torch.full((shots,), float(channel_llr(pflip)), dtype=torch.float32, device="cuda")
    out = dec.alloc_outputs(shots)
    torch.cuda.synchronize()

    # ---- roofline pass: eager decodes with a schedule; HIP events on the
    #      decode stream around every Phase 1 and Phases 2-3 launch.  The
    #      fixed-point exit is off in this pass: a run it ends reports the cap
    #      as its iteration count, and the edge updates counted from the
    #      statistics must be ones the kernels execute
    rl_reps = 2 if args.roofline_only else 4

    def roofline_pass():
        dec.set_params(max_iter_local=ROUNDS[cname], max_iter_global=ROUNDS[cname], ms_scale=0.75, alpha=1.0,
                       fixed_point_stop=0)
        dec.decode(synd_pool[0], lam, out=out)
        torch.cuda.synchronize()
        dec.time_phases(True)
        eu = [0.0, 0.0]
        for i in range(rl_reps):
            dec.decode(synd_pool[i % pool_batches], lam, out=out)
            st = out["stats"].cpu().numpy()
            a, b = edge_updates(st, info.eloc[args.check_type], info.order)
            eu[0] += a
            eu[1] += b
        pt = dec.phase_times()
        dec.time_phases(False)
        dec.set_params(max_iter_local=ROUNDS[cname], max_iter_global=ROUNDS[cname], fixed_point_stop=FIXED_POINT,
                       ms_scale=0.75, alpha=1.0)
        return eu[0], eu[1], pt

    # ---- schedule of the headline: the autotuner's choice (or --schedule).
    #      The roofline pass runs before the autotuner's trial decodes, on
    #      the default schedule (the state of the profiled runs), and again
    #      on the autotuner's choice only where that differs
    if args.schedule is not None or args.roofline_only:
        best = dict(DEFAULT_SCHEDULE if args.schedule is None else json.loads(args.schedule))
        dec.set_schedule(**best)
        best = dec.get_schedule()
        eu_local, eu_global, pt = roofline_pass()
    else:
        dec.set_schedule(**DEFAULT_SCHEDULE)
        rl_sched = dec.get_schedule()
        eu_local, eu_global, pt = roofline_pass()
        best = dec.autotune(synd_pool[0], lam)
        if best != rl_sched:
            eu_local, eu_global, pt = roofline_pass()
    if pt["global_launches"] == 0:
        raise SystemExit(f"the schedule {best} does not run the work-queue form, which the roofline pass times")
    d2 = info.delta ** 2
    kern = {}
    for phase, eu, ms, nl in (("global", eu_global, pt["global_ms"], pt["global_launches"]),
                              ("local", eu_local, pt["local_ms"], pt["local_launches"])):
        gops = OPS_PER_EDGE_UPDATE * eu / (ms * 1e-3) / 1e9
        kern[phase] = {"achieved": gops / 1000, "frac": gops / VALU_PEAK_GOPS, "ms_per_launch": ms / nl,
                       "launches": nl, "ops_per_launch": OPS_PER_EDGE_UPDATE * eu / nl}
    shots_per_launch = rl_reps * shots / pt["global_launches"]
    g_bytes = global_kernel_bytes_per_shot(n, m, info.order, d2) * shots_per_launch
    hbm_gbs = g_bytes / (kern["global"]["ms_per_launch"] * 1e-3) / 1e9
    if args.roofline_only:
        print(json.dumps({"roofline_pass": kern, "schedule": best, "code": cname, "check_type": args.check_type,
                          "p": pflip, "shots": shots}),
              flush=True)
        return
    # (form 2 with the fixed-point exit off runs its variant without the test)
    gname = f"lead_spec_global_{best.get('specialized')}" + ("n" if best.get("specialized") == 2 else "")
    lname = f"lead_spec_local_{best.get('specialized')}0"
    traffic = traffic_local = None
    issued = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_sha") == kernel_hash() and rec.get("shots_per_launch") == shots_per_launch:
            traffic = rec.get("kernels", {}).get(gname, {}).get("hbm_bytes_per_launch")
            traffic_local = rec.get("kernels", {}).get(lname, {}).get("hbm_bytes_per_launch")
    if os.path.exists(COUNTER_FILE):
        rec = json.load(open(COUNTER_FILE))
        if rec.get("kernel_sha") == kernel_hash() and rec.get("shots_per_launch") == shots_per_launch:
            v = rec.get("kernels", {}).get(gname, {}).get("SQ_INSTS_VALU_per_launch")
            if v:
                # issued VALU lane-ops (64 per wave instruction) per launch
                # over the measured launch time
                issued = {"valu_insts_per_launch": v,
                          "achieved": round(v * 64 / (kern["global"]["ms_per_launch"] * 1e-3) / 1e12, 3),
                          "frac": round(v * 64 / (kern["global"]["ms_per_launch"] * 1e-3) / 1e9 / VALU_PEAK_GOPS, 4),
                          "per_counted_op": round(v * 64 / kern["global"]["ops_per_launch"], 3)}
    form = {1: "compressed check state",
            2: "one register per message, no fixed-point test"}.get(best.get("specialized"), "")
    roof = {"bound": "alu", "achieved": round(kern["global"]["achieved"], 3), "peak": round(VALU_PEAK_GOPS / 1000, 2),
            "unit": "TOP/s", "frac": round(kern["global"]["frac"], 4), "traffic": traffic,
            "kernel": f"{gname} (Phases 2-3 compiled for the A5 code, {form}; {shots_per_launch:.0f} shots per launch)",
            "kernel_ms": round(kern["global"]["ms_per_launch"], 3),
            "pass": "eager decodes of the headline batches with the fixed-point exit off, so that every edge "
                    "update counted from the statistics is executed",
            "achieved_is": "algorithmic lane operations (10 per min-sum edge update counted from the returned "
                           "statistics) per second of the kernel's HIP-event time",
            "algorithmic_ops_per_launch": round(kern["global"]["ops_per_launch"]),
            "issued_valu": issued,
            "kernel_hbm_bytes_per_launch": round(g_bytes),
            "kernel_hbm_gbs": round(hbm_gbs, 1), "kernel_hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 5),
            "phase1_kernel": {"kernel": f"lead_spec_local_{best.get('specialized')}0 (Phase 1 work queue)",
                              "kernel_ms": round(kern["local"]["ms_per_launch"], 3),
                              "achieved": round(kern["local"]["achieved"], 3),
                              "frac": round(kern["local"]["frac"], 4)}}

    # ---- headline: each batch captured as a graph, replayed
    graphs = [P.Batch([(dec, synd_pool[b], lam, out, P.LEAD_PRIOR_PER_SHOT)]).capture()
              for b in range(pool_batches)]
    for i in range(args.warmup):
        graphs[i % pool_batches].replay()
    wall, _ = timed(torch, lambda i: graphs[i % pool_batches].replay(), args.steps)
    st = out["stats"].cpu().numpy()
    ms_per_step = wall * 1000.0 / args.steps
    value = shots / (wall / args.steps)
    del graphs
    # the whole decode against the HBM roofline: the method's own bytes per
    # shot (syndrome, prior, L_post, e_hat, statistics) at the headline rate,
    # beside the bytes the counters saw for both kernels
    dec_bytes = algorithmic_bytes_per_shot(n, m)
    meas = None
    if traffic is not None and traffic_local is not None:
        meas = round((traffic + traffic_local) / shots_per_launch, 1)
    roof["decode_hbm"] = {
        "algorithmic_bytes_per_shot": round(dec_bytes, 1), "achieved_gbs": round(dec_bytes * value / 1e9, 1),
        "frac": round(dec_bytes * value / 1e9 / HBM_PEAK_GBS, 5),
        "counter_bytes_per_shot_both_kernels": meas,
        "excess": "the local posteriors (order x Delta^2 x 4 B = 8.6 KB per A5 shot) and view flags make a round "
                  "trip through HBM between the Phase 1 queue kernel and the Phases 2-3 kernel; the method's own "
                  "I/O is 4.5 KB per shot"}

    # ---- the same decode without batching: eager on one stream (same
    #      kernels, no graph), and the plain per-round-launch form on the
    #      same compiled kernels (one launch per global round, state in HBM,
    #      host-visible count of running shots); each warmed up once, then
    #      timed over plain_steps batches
    plain = None
    if args.plain_steps > 0:
        dec.decode(synd_pool[0], lam, out=out)
        ew, _ = timed(torch, lambda i: dec.decode(synd_pool[i % pool_batches], lam, out=out), args.plain_steps)
        ew /= args.plain_steps
        dec.decode(synd_pool[0], lam, out=out, plain=True)
        pw, _ = timed(torch, lambda i: dec.decode(synd_pool[i % pool_batches], lam, out=out, plain=True),
                      args.plain_steps)
        pw /= args.plain_steps
        # the precompiled per-round kernels (runtime masks, sums in LDS)
        dec.set_schedule(**{**best, "specialized": 0, "fused": 0})
        dec.decode(synd_pool[0], lam, out=out, plain=True)
        qw, _ = timed(torch, lambda i: dec.decode(synd_pool[i % pool_batches], lam, out=out, plain=True),
                      args.plain_steps)
        qw /= args.plain_steps
        dec.set_schedule(**best)
        plain = {"shots_per_s": round(shots / pw, 1), "ms_per_step": round(pw * 1000, 3),
                 "form": "lead_decode_plain on the kernels compiled for the code: Phase 1 launch, one launch of the "
                         "compiled round kernel per global round with sums and check state in HBM and a host-visible "
                         "count of running shots, a last launch for shots at the cap",
                 "batched_over_plain": round(value * pw / shots, 3),
                 "eager_one_stream": {"shots_per_s": round(shots / ew, 1), "ms_per_step": round(ew * 1000, 3),
                                      "batched_over_eager": round(value * ew / shots, 3),
                                      "form": "lead_decode eager on one stream, no graph (same kernels)"},
                 "precompiled_plain": {"shots_per_s": round(shots / qw, 1), "ms_per_step": round(qw * 1000, 3),
                                       "batched_over_plain": round(value * qw / shots, 3),
                                       "form": "lead_decode_plain on the precompiled kernels (runtime masks, "
                                               "variable sums in LDS, one launch per round)"},
                 "steps": args.plain_steps, "warmup": 1}

    # ---- the single-stage baseline: global BP alone with the channel priors
    #      on the same batches (stage GLOBAL)
    base_leg = None
    if not args.no_baseline_decoder:
        gdec = P.Decoder(code, max_shots=shots, max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"],
                         fixed_point_stop=FIXED_POINT, ms_scale=0.75, alpha=1.0, stage=2)
        gout = gdec.alloc_outputs(shots)
        gdec.decode(synd_pool[0], lam, out=gout)
        gw, _ = timed(torch, lambda i: gdec.decode(synd_pool[i % pool_batches], lam, out=gout), 2)
        gst = gout["stats"].cpu().numpy()     # batch 1 of the pool
        dec.decode(synd_pool[1], lam, out=out)
        lst = out["stats"].cpu().numpy()
        r_over_m = info.r[0] / m
        base_leg = {
            "global_bp_only_shots_per_s": round(2 * shots / gw, 1),
            "global_bp_only": {"converged": round(float(gst[:, 0].mean()), 4),
                               "mean_iterations": round(float(gst[:, 1].mean()), 2)},
            "lead": {"converged": round(float(lst[:, 0].mean()), 4),
                     "mean_iterations_I": round(float((lst[:, 1] + lst[:, 2] / info.order * r_over_m).mean()), 2),
                     "mean_global_iterations": round(float(lst[:, 1].mean()), 2)},
            "note": "same 10^5 syndromes; I = I_g + mean local iterations x r/m (the paper's iteration measure)"}

    # ---- variants on the same GPU: sum-product BP on the headline batches;
    #      alpha sweep at p = 0.02; PSL(2,7) under depolarising noise
    variants = None
    if not args.no_variants:
        variants = {}
        sdec = P.Decoder(code, max_shots=shots, max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"],
                         fixed_point_stop=FIXED_POINT, alpha=1.0, bp=1)
        sout = sdec.alloc_outputs(shots)
        sdec.decode(synd_pool[0], lam, out=sout)
        sw, _ = timed(torch, lambda i: sdec.decode(synd_pool[i % pool_batches], lam, out=sout), 2)
        sst = sout["stats"].cpu().numpy()
        variants["sum_product_A5_p005"] = {"shots_per_s": round(2 * shots / sw, 1),
                                          "converged": round(float(sst[:, 0].mean()), 4),
                                          "mean_global_iters": round(float(sst[:, 1].mean()), 2)}
        del sdec, sout
        odec = P.Decoder(code, max_shots=shots, max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"],
                         fixed_point_stop=FIXED_POINT, ms_scale=0.75, alpha=1.0, local_post=1)
        oout = odec.alloc_outputs(shots)
        odec.decode(synd_pool[0], lam, out=oout)
        ow, _ = timed(torch, lambda i: odec.decode(synd_pool[i % pool_batches], lam, out=oout), 2)
        ost = oout["stats"].cpu().numpy()
        variants["local_osd0_A5_p005"] = {"shots_per_s": round(2 * shots / ow, 1),
                                         "converged": round(float(ost[:, 0].mean()), 4),
                                         "mean_global_iters": round(float(ost[:, 1].mean()), 2),
                                         "osd_views_per_shot": round(float(ost[:, 7].mean()), 2)}
        del odec, oout
        # OSD-0 on H_t after global BP: LEAD with it, and BP-OSD-0 on H_t alone
        for key, kw in (("global_osd0_A5_p005", {}), ("bp_osd0_A5_p005", {"stage": P.LEAD_STAGE_GLOBAL}),
                        ("global_osd_cs3_A5_p005", {"osd_order": 3}),
                        ("bp_osd_cs3_A5_p005", {"stage": P.LEAD_STAGE_GLOBAL, "osd_order": 3}),
                        ("local_and_global_osd_cs3_A5_p005", {"local_post": 1, "osd_order": 3})):
            gd2 = P.Decoder(code, max_shots=shots, max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"],
                            fixed_point_stop=FIXED_POINT, ms_scale=0.75, alpha=1.0, global_post=1, **kw)
            go2 = gd2.alloc_outputs(shots)
            gd2.decode(synd_pool[0], lam, out=go2)
            w2, _ = timed(torch, lambda i: gd2.decode(synd_pool[i % pool_batches], lam, out=go2), 2)
            st2 = go2["stats"].cpu().numpy()
            variants[key] = {"shots_per_s": round(2 * shots / w2, 1),
                             "converged_by_bp": round(float((st2[:, 0] == 1).mean()), 4),
                             "resolved_by_osd": round(float((st2[:, 0] == 2).mean()), 4),
                             "mean_global_iters": round(float(st2[:, 1].mean()), 2)}
            del gd2, go2
        s02 = syndromes(torch, dec, n, shots, 0.02, seed=1500)
        lam02 = torch.full((shots,), float(channel_llr(0.02)), dtype=torch.float32, device="cuda")
        sweep = []
        for alpha in (1.0, 0.5, 0.1, 0.01):
            dec.set_params(max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"], fixed_point_stop=FIXED_POINT,
                           ms_scale=0.75, alpha=alpha)
            dec.decode(s02, lam02, out=out)
            aw, _ = timed(torch, lambda i: dec.decode(s02, lam02, out=out), 1)
            ast = out["stats"].cpu().numpy()
            sweep.append({"alpha": alpha, "shots_per_s": round(shots / aw, 1),
                          "converged": round(float(ast[:, 0].mean()), 4),
                          "mean_global_iters": round(float(ast[:, 1].mean()), 2)})
        dec.set_params(max_iter_local=ROUNDS["M"], max_iter_global=ROUNDS["M"], fixed_point_stop=FIXED_POINT,
                       ms_scale=0.75, alpha=1.0)
        variants["alpha_sweep_A5_p002"] = sweep
        # A5 at the four bit-flip rates of the mid-code workload (10^5 shots each)
        sweep_p = []
        for pi, pp in enumerate((0.02, 0.04, 0.06, 0.08)):
            sp_ = syndromes(torch, dec, n, shots, pp, seed=1600 + pi)
            lp_ = torch.full((shots,), float(channel_llr(pp)), dtype=torch.float32, device="cuda")
            dec.decode(sp_, lp_, out=out)
            pw_, _ = timed(torch, lambda i: dec.decode(sp_, lp_, out=out), 1)
            pst = out["stats"].cpu().numpy()
            sweep_p.append({"p": pp, "shots_per_s": round(shots / pw_, 1), "converged": round(float(pst[:, 0].mean()), 4),
                            "mean_global_iters": round(float(pst[:, 1].mean()), 2)})
            del sp_, lp_
        variants["p_sweep_A5"] = sweep_p
        # PSL(2,7) under depolarising noise (the large-code workload: 10^6
        # distinct shots per p): X errors decoded with the Z checks and Z
        # errors with the X checks, independently, prior 2p/3
        from lead_inputs.noise_device import depolarizing_packed_device
        lshots = args.large_shots
        lcode = P.Code.from_spec(__import__("lead_inputs").standard("L"))
        ldecs = [P.Decoder(lcode, t=t, max_shots=lshots, max_iter_local=ROUNDS["L"], max_iter_global=ROUNDS["L"],
                           fixed_point_stop=FIXED_POINT) for t in (0, 1)]
        lo_ = ldecs[0].alloc_outputs(lshots, post=False)
        dep = []
        for pi, pdep in enumerate((0.01, 0.02, 0.03, 0.04, 0.05)):
            xs, zs = depolarizing_packed_device(lshots, lcode.n, pdep, seed=2500 + pi)
            lam_d = torch.full((lshots,), float(channel_llr(2 * pdep / 3)), dtype=torch.float32, device="cuda")
            parts, ltime = {}, 0.0
            for t in (0, 1):
                ld = ldecs[t]
                ls = ld.syndrome(xs if t == 0 else zs)
                if pi == 0:
                    ld.decode(ls[:32768], lam_d[:32768], out={k: (v[:32768] if v is not None else None)
                                                             for k, v in lo_.items()})
                lw, _ = timed(torch, lambda i: ld.decode(ls, lam_d, out=lo_), 1)
                ltime += lw
                lst = lo_["stats"].cpu().numpy()
                parts["XZ"[t] + "_errors"] = {"converged": round(float((lst[:, 0] == 1).mean()), 4),
                                              "mean_global_iters": round(float(lst[:, 1].mean()), 2),
                                              "shots_per_s": round(lshots / lw, 1)}
                del ls
            del xs, zs
            dep.append({"p": pdep, "shots": lshots, "distinct_error_draws": lshots,
                        "shots_per_s_both_parts": round(lshots / ltime, 1), **parts})
        del ldecs, lo_
        variants["PSL27_depolarising"] = dep

    # ---- mixed-code batch (D6 / A5 / PSL(2,7)): one graph launch vs plain
    mixed = None
    decs_named = {"M": (code, dec)}
    if not args.no_mixed:
        from lead_inputs import uniform_p
        sizes = {"T": 1000, "M": 30000, "L": 100000}
        entries, plain_items = [], []
        for i, name in enumerate(("T", "M", "L")):
            c2, d2 = make_decoder(P, name, sizes[name]) if name != "M" else (code, dec)
            decs_named[name] = (c2, d2)
            ps = uniform_p(sizes[name], 0.02, 0.08, seed=2000 + i)
            s = syndromes(torch, d2, c2.n, sizes[name], ps, seed=2000 + i)
            pr = torch.from_numpy(channel_llr(ps)).cuda()
            o = d2.alloc_outputs(sizes[name])
            if name != "M":
                d2.autotune(s, pr)
                sc = d2.get_schedule()
                if sc["specialized"] == 0 or sc["fused"]:
                    # every leg of this comparison runs the kernels compiled
                    # for the code (the fused batch needs them)
                    d2.set_schedule(**{**sc, "specialized": 2, "fused": 0})
            entries.append((d2, s, pr, o, P.LEAD_PRIOR_PER_SHOT))
            plain_items.append((d2, s, pr, o))
        batch = P.Batch(entries).capture()
        batch.replay()
        bw, _ = timed(torch, lambda i: batch.replay(), 3)
        bw /= 3
        # the same requests fused: one persistent Phase 1 launch and one
        # Phases 2-3 launch for the three codes, replayed as a graph
        fused = P.FusedBatch(entries)
        fused.launch()
        fw, _ = timed(torch, lambda i: fused.launch(), 3)
        fw /= 3
        del fused
        for d2, s, pr, o in plain_items:   # warm-up: per-round state allocated here
            d2.decode(s, pr, out=o, plain=True)
        pw2, _ = timed(torch, lambda i: [d2.decode(s, pr, out=o, plain=True) for d2, s, pr, o in plain_items], 2)
        pw2 /= 2
        ew2, _ = timed(torch, lambda i: [d2.decode(s, pr, out=o) for d2, s, pr, o in plain_items], 2)
        ew2 /= 2
        total = sum(sizes.values())
        mixed = {"shots": sizes, "batched_graph_shots_per_s": round(total / bw, 1),
                 "fused_graph_shots_per_s": round(total / fw, 1),
                 "plain_per_code_shots_per_s": round(total / pw2, 1), "batched_over_plain": round(pw2 / bw, 3),
                 "fused_over_plain": round(pw2 / fw, 3),
                 "eager_per_code_one_stream_shots_per_s": round(total / ew2, 1),
                 "batched_over_eager": round(ew2 / bw, 3), "fused_over_eager": round(ew2 / fw, 3),
                 "form": "batched: one captured graph of the three codes' launch sequences on forked library "
                         "streams; fused: one persistent Phase 1 launch draining the three codes' work queues in "
                         "turn and one Phases 2-3 grid over all three, captured as a graph; plain = "
                         "lead_decode_plain per code in turn (same compiled kernels)"}
        del batch

    # ---- serving loop: Poisson streams of host requests (copy-in, decode,
    #      copy-out per request; latency from submit to completion)
    served = None
    if not args.no_served:
        served = {}
        reqs_m = request_mix(torch, decs_named, 10000, seed=31, codes=["M"])
        # A5 alone: offered loads up to and past the saturation point
        served["A5_only"] = [served_stream(P, [dec], reqs_m, load, seed=41) for load in (1e6, 4e6, 8e6, 1.6e7)]
        sat = [r for r in served["A5_only"] if r["shots_per_s"] < 0.95 * r["offered_shots_per_s"]]
        served["A5_saturation_shots_per_s"] = max(r["shots_per_s"] for r in served["A5_only"]) if sat else None
        # the same requests served without batching: one request at a time,
        # copy-in, plain decode, copy-out
        t0 = time.perf_counter()
        pshots = 0
        for k, s, pr in reqs_m[:200]:
            o = dec.decode(torch.from_numpy(s.view(np.int64)).cuda(), torch.from_numpy(pr).cuda(), plain=True)
            o["ehat"].cpu()
            pshots += s.shape[0]
        served["A5_plain_one_request_at_a_time_shots_per_s"] = round(pshots / (time.perf_counter() - t0), 1)
        if not args.no_mixed:
            decs_x = [decs_named[c][1] for c in ("T", "M", "L")]
            served["mixed_3_codes"] = []
            for j, (load, nreq) in enumerate(((1e5, 2000), (1e6, 4000))):
                reqs_x = request_mix(torch, decs_named, nreq, seed=32 + j, codes=["T", "M", "L"])
                served["mixed_3_codes"].append(served_stream(P, decs_x, reqs_x, load, seed=42 + j,
                                                             names=["D6", "A5", "PSL27"]))

    cpu = None
    if not args.no_cpu_baseline:
        from lead_inputs import standard
        # one process per core of the host's share for one GPU (16 on these
        # boxes, whatever nproc shows: the CPUs are shared between GPUs)
        workers = max(1, min(16, os.cpu_count() or 1))
        rate, cwall = cpu_baseline(standard("M"), args.cpu_sample, seed=7, workers=workers)
        lat_ms = cpu_latency(standard("M"), 200, seed=8)
        cpu = {"value": round(rate, 1), "unit": "decoded shots/s", "cores": workers, "kind": "oracle",
               "sample": f"{args.cpu_sample} shots of the headline workload (A5 code, p=0.05, 50+50 rounds), "
                         f"FP64 oracle (plain C, -O2, single-threaded), {workers} worker processes over shot shards, "
                         f"{cwall:.1f} s wall including process start",
               "host": host_facts(),
               "single_process_median_ms_per_shot": round(lat_ms, 3),
               "note": "16 worker processes = the host CPU share of one GPU on this machine"}

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
                   "shots_per_step": shots,
                   "form": "batched: captured graph of lead_decode (kernels compiled for the code), "
                           + ("schedule from --schedule" if args.schedule else "autotuned schedule"),
                   "fixed_point_exit": {0: "off", 1: "local and global BP runs",
                                        2: "local BP runs (outputs as without it)"}[FIXED_POINT],
                   "schedule": best},
        "roofline": roof,
        "decode_stats": {"converged": round(float((st[:, 0] == 1).mean()), 4),
                         "mean_global_iters": round(float(st[:, 1].mean()), 2),
                         "mean_local_iters": round(float(st[:, 2].mean() / info.order), 2)},
        "plain_form": plain,
        "single_stage_baseline": base_leg,
        "variants": variants,
        "mixed_batch": mixed,
        "served": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
