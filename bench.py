#!/usr/bin/env python3
"""Benchmark of HERS encrypted search on one MI355X.

Metric: encrypted scores per second (gallery items x probes per second), with
p50/p99 probe latency.  One step is one query through the whole per-query path
on data resident in HBM: encrypt the probe (one ciphertext per dimension),
search every gallery block (fused multiply-accumulate over d, exact t/q
rescale, one relinearization per block), decrypt and decode the scores.  The
one-time enrollment (key generation, gallery encoding, encryption and lift)
runs before the timed region and is reported on its own.

Printed: one JSON line with the metric, the roofline of the multiply-accumulate
kernel (k_mac; durations from HIP events on its launch stream), and the oracle
timed on a bounded sample on the host cores as the CPU baseline.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

WORKLOADS = {
    # the configuration the metric is quoted on: single probe, 2^20 items, d = 64
    "single": dict(desc="single probe vs 1,048,576-item gallery, d=64, n=4096, q=3x36-bit primes, t=1,032,193",
                   n=4096, qbits=(36, 36, 36), t_bits=20, w_bits=0, d=64, m=1 << 20),
    # largest single-GPU instance: 10^8 items, d = 32
    "large": dict(desc="single probe vs 100,000,000-item gallery, d=32, n=4096, q=3x36-bit primes, t=1,032,193",
                  n=4096, qbits=(36, 36, 36), t_bits=20, w_bits=0, d=32, m=100_000_000),
}

KEY_SEED, GALLERY_SEED, PROBE_SEED, FEATURE_SEED, QUERY_SEED = 201, 301, 401, 1000, 2000


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("kernels.hip", "hers_common.h", "ntt.h"):
        with open(os.path.join(ROOT, "paper_2003_12197_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per k_mac launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "k_mac_%s_pmc.txt" % workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"TRAFFIC_BYTES_PER_LAUNCH=(\d+)", text)
    s = re.search(r"KERNEL_SOURCE_DIGEST=(\w+)", text)
    if not m or not s or s.group(1) != kernel_source_digest():
        return None
    return int(m.group(1))


def cpu_baseline(cfg, P_block0, qv, m):
    """The oracle on one gallery block: probe encryption once plus one block's
    search and decryption, scaled to the whole gallery (blocks are independent)."""
    from oracle import fv, hers
    op = fv.Params(n=cfg["n"], qbits=cfg["qbits"], t_bits=cfg["t_bits"], w_bits=cfg["w_bits"])
    n = cfg["n"]
    sk, pk, rlk = fv.keygen(op, KEY_SEED)
    og = hers.encrypt_gallery_block(op, pk, P_block0, 0, GALLERY_SEED)
    t0 = time.perf_counter()
    oq = hers.encrypt_probe(op, pk, qv, PROBE_SEED)
    t1 = time.perf_counter()
    S = hers.search_block(op, rlk, oq, og)
    scores = hers.decrypt_scores(op, sk, {0: S}, n)
    t2 = time.perf_counter()
    assert np.array_equal(scores, hers.plaintext_scores(P_block0, qv))
    M = (m + n - 1) // n
    t_probe, t_block = t1 - t0, t2 - t1
    total = t_probe + M * t_block
    return {"value": m / total, "unit": "scores/s", "cores": 1, "kind": "oracle",
            "sample": "one %d-item block of the gallery (d=%d): probe encryption %.1f s once, block search + "
                      "decryption %.1f s, scaled to %d blocks" % (n, cfg["d"], t_probe, t_block, M)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_12197_amd import hers_gpu, synth

    cfg = WORKLOADS[args.workload]
    n, d, m = cfg["n"], cfg["d"], cfg["m"]
    dev = torch.device("cuda", 0)
    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = hers_gpu.Context(n=n, qbits=cfg["qbits"], t_bits=cfg["t_bits"], w_bits=cfg["w_bits"], d_max=d)
    M = ctx.blocks(m)
    print("workload %s: %d items x d=%d, %d blocks, K=%d base primes" % (args.workload, m, d, M, ctx.K),
          file=sys.stderr, flush=True)

    # ---- enrollment (untimed by the metric; reported separately)
    t0 = time.perf_counter()
    sk, pk, rlk = ctx.keygen(KEY_SEED)
    gallery = ctx.new_gallery(m, d)
    chunk = max(1, min(M, (1 << 30) // (d * n * 4)))      # features of up to 1 GiB per chunk
    ws = ctx.workspace(hers_gpu.OP_ENCRYPT_GALLERY, chunk * n, d)
    P_block0 = None
    enc_ms = 0.0
    for b0 in range(0, M, chunk):
        nb = min(chunk, M - b0)
        feats = synth.gallery_features(FEATURE_SEED, n, d, m, block0=b0, nblocks=nb)
        if b0 == 0:
            P_block0 = feats[:, :n].copy()
        ft = torch.from_numpy(feats).to(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.encrypt_gallery(ft, m, GALLERY_SEED, block0=b0, nblocks=nb, gallery=gallery, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        enc_ms += e0.elapsed_time(e1)
        del ft
    del ws
    setup_s = time.perf_counter() - t0
    print("enrolled in %.1f s (GPU encryption %.1f ms)" % (setup_s, enc_ms), file=sys.stderr, flush=True)

    qv, mate = synth.probe_for(QUERY_SEED, FEATURE_SEED, n, d, m)
    query = torch.from_numpy(qv).to(dev)
    probe = torch.empty(int(ctx.lib.hers_probe_words(ctx.handle, d)), dtype=torch.int32, device=dev)
    scores = ctx.new_scores(m)
    out = torch.empty(m, dtype=torch.int32, device=dev)
    ws_p = ctx.workspace(hers_gpu.OP_ENCRYPT_PROBE, 0, d)
    ws_s = ctx.workspace(hers_gpu.OP_SEARCH, m, d)
    ws_d = ctx.workspace(hers_gpu.OP_DECRYPT, m, 1)

    ctx.encrypt_probe(query, PROBE_SEED, probe=probe, workspace=ws_p)
    mac_variant = ctx.autotune(gallery, m, d, probe, reps=3, workspace=ws_s)
    print("autotuned k_mac schedule: %d" % mac_variant, file=sys.stderr, flush=True)

    def step(seed):
        ctx.encrypt_probe(query, seed, probe=probe, workspace=ws_p)
        ctx.search(gallery, m, d, probe, scores=scores, workspace=ws_s)
        ctx.decrypt_scores(sk, scores, m, out=out, workspace=ws_d)

    for w in range(args.warmup):
        step(PROBE_SEED + w)
    torch.cuda.synchronize()

    # ---- timed region
    ctx.profile_enable(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    evs[0].record()
    for s in range(args.steps):
        step(PROBE_SEED)
        evs[s + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = [evs[s].elapsed_time(evs[s + 1]) for s in range(args.steps)]
    total_ms = evs[0].elapsed_time(evs[-1])
    stages = {st: ctx.profile_read(st) for st in ("mac", "intt_acc", "rescale", "relin", "encrypt", "lift",
                                                 "ntt_fwd", "sk_ntt", "dec_mul", "dec_decode")}
    ctx.profile_enable(False)

    # ---- correctness of the last step (outside the timed region)
    got = out.cpu().numpy()
    if args.workload == "single":
        P = synth.gallery_features(FEATURE_SEED, n, d, m)
        ok = bool(np.array_equal(got, P.T.astype(np.int64) @ qv.astype(np.int64)))
        del P
    else:
        ok = bool(np.array_equal(got[:n], P_block0.T.astype(np.int64) @ qv.astype(np.int64)))
    top = int(np.argmax(got))

    # ---- roofline of k_mac: algorithmic bytes = gallery search form + probe + accumulators
    K = ctx.K
    mac_ms, mac_n = stages["mac"]
    gallery_bytes = M * K * d * 2 * n * 4
    probe_bytes = K * d * 2 * n * 4
    acc_bytes = M * 3 * K * n * 4
    launches_per_step = mac_n / args.steps
    bytes_per_launch = (gallery_bytes + acc_bytes) / launches_per_step + probe_bytes
    mac_avg_ms = mac_ms / mac_n
    achieved = bytes_per_launch / (mac_avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)

    value = m * args.steps / (total_ms * 1e-3)
    lat = np.array(step_ms)
    result = {
        "metric": "encrypted scores/sec (gallery items x probes per s); p50/p99 probe latency",
        "value": value,
        "unit": "scores/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "items": m, "dims": d, "probes_per_step": 1, "blocks": M,
                   "ring_degree": n, "q_primes_bits": list(cfg["qbits"]), "t": int(ctx.t),
                   "base_primes": K, "step": "encrypt probe + search all blocks + decrypt scores",
                   "mac_schedule": mac_variant},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "search_only_scores_per_s": m / (sum(stages[s][0] for s in ("mac", "intt_acc", "rescale", "relin"))
                                         / args.steps * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "k_mac", "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": mac_avg_ms},
        "enrollment": {"gpu_encrypt_ms": enc_ms, "items_per_s": m / (enc_ms * 1e-3), "wall_s": setup_s},
        "check": {"scores_equal_PTq": ok, "argmax": top, "mate": mate},
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        print("cpu baseline: oracle on one block ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(cfg, P_block0, qv, m)
    print(json.dumps(result), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
