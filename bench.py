#!/usr/bin/env python3
"""Quartics height-classified per second at p = 7 on one MI355X.

Workload (named in config.workload): the p = 7 batch of 65,536 seeded
quartics of uneven structure from workloads.config_p7_batch (seed 0): half
diagonal a x1^4 + b x2^4 + c x3^4 + d x4^4 plus 1-8 random cross terms, half
dense, nonzero values uniform in {1..6}.  One step is one qfs_height call over
the whole batch with the inputs already in HBM: Fedder's test for every
surface, then Delta_1 on int8 matrix cores and the theta loop for the
surfaces that fail it.

Printed: one JSON line with the throughput, the roofline of the dominant
kernel (the Delta_1 + theta kernel, timed live with hipEvents on its stream),
the CPU oracle on a bounded sample of the same workload, and the plain
per-surface GPU kernels on a sample.
"""
import argparse
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "quartics height-classified/sec at p=7 (batched int8-MFMA vs plain), bit-exact"
INT8_PEAK_TOPS = 5000.0  # MI355X dense int8 matrix peak, 5.0 POP/s

# HBM traffic of the deep kernel on the p7_batch65536 workload from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
# scaled by what the same counter read for a 512 MiB device-to-device copy
# (FETCH x 1.9998, WRITE x 1.0).  Valid only for the kernel sources they were
# taken on; any change to those sources reports null until re-measured.
TRAFFIC_SOURCES = ("qfs_batched.hip", "qfs_device.h", "qfs_common.h", "qfs_internal.h")
TRAFFIC = {
    "workload": "p7_batch65536",
    "sources_sha256": "d4b61a1b179fdc5afe27734e924d5d1b3949eb405e6ed3c75b993bc097dd9327",
    "fetch_kib": 311307806.4375, "fetch_scale": 524288.0 / 262170.625,
    "write_kib": 66872266.375, "write_scale": 1.0,
    "profile": "profiles/k_deep7_p7_batch65536_counters.md",
}


def measured_traffic(workload):
    """Calibrated HBM bytes per deep-kernel launch, or None if stale or for another workload."""
    import hashlib
    if workload != TRAFFIC["workload"]:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_12428_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sources_sha256"]:
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"])


def delta1_macs(p):
    """Useful multiply-adds of the chain g~^(k+1) = g~^k * g~, k = 1..p-1 (dense schoolbook counts)."""
    d = 4 * (p - 1)
    return sum(comb(d * k + 3, 3) * comb(d + 3, 3) for k in range(1, p))


def theta_macs(p, h, bound=10):
    """theta work of one deep surface with height h: (tests) x len_g + (full maps) x len_g^2."""
    lg = comb(4 * p - 1, 3)
    if h == 0:
        tests, full = bound - 1, bound - 2
    else:
        tests, full = h - 1, h - 2
    return tests * lg + max(full, 0) * lg * lg


WORKLOADS = {
    "p7_batch65536": "p=7, 65536 seeded quartics (half diagonal plus 1-8 cross terms, half dense; values uniform 1..6)",
    "p5_batch8192": "p=5, 8192 seeded quartics (Bernoulli support of density 0.1/0.3/0.6/1.0; values uniform 1..4)",
    "mixed4096": "4096 seeded quartics, p uniform over 3/5/7/11, Bernoulli support of density U[0.1,1], values 1..p-1",
    "p7_single": "p=7: Fermat, the p=7 rows of the paper's height table and 16 seeded Bernoulli(0.5) quartics",
    "p5_single": "p=5: one seeded dense quartic and the Fermat quartic",
}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="p7_batch65536")
    ap.add_argument("--cpu-sample", type=int, default=384)
    ap.add_argument("--cpu-sample-single", type=int, default=48)
    ap.add_argument("--plain-sample", type=int, default=48)
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before the timed region, copy this many MiB device-to-device once: a plain copy "
                         "kernel of known size whose memory counters scale the profiler's byte counts")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the height pipeline has no cross-GPU step and this build runs on a "
              "single MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2502_12428_amd as qfs
    import workloads

    F, P = workloads.CONFIGS[args.workload]()
    B = F.shape[0]
    p = int(P.max())
    f = torch.from_numpy(F).cuda()
    pt = torch.from_numpy(P).cuda()
    ws = qfs.Workspace()
    print("bench: workload %s, batch %d, warmup %d, steps %d" % (args.workload, B, args.warmup, args.steps),
          file=sys.stderr, flush=True)

    if args.calibrate_copy_mb > 0:
        src = torch.ones(args.calibrate_copy_mb << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cold_ms = None
    for i in range(args.warmup):
        t0 = time.perf_counter()
        h = qfs.height(f, pt, max_p=p, workspace=ws)
        if i == 0:  # the cold first call: one-time kernel set-up and first touch of the workspace
            torch.cuda.synchronize()
            cold_ms = 1e3 * (time.perf_counter() - t0)
    torch.cuda.synchronize()
    qfs.profile_collect()
    qfs.profile(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        h = qfs.height(f, pt, max_p=p, workspace=ws)
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    qfs.profile(False)
    stage_ms, calls = qfs.profile_collect()
    elapsed = t1 - t0
    step_ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    heights = h.cpu().numpy()

    parity = "unchecked"
    gold = os.path.join(ROOT, "tests", "golden", "heights_%s.npz" % args.workload)
    if os.path.exists(gold):
        parity = bool(np.array_equal(np.load(gold)["heights"].astype(np.int32), heights))

    # the dominant deep kernel (the prime whose deep launch takes longest)
    per_call = {k: v / max(calls, 1) for k, v in stage_ms.items()}
    pd = max((q for q in (3, 5, 7, 11) if (P == q).any()), key=lambda q: per_call["deep_p%d" % q])
    deep_ms = per_call["deep_p%d" % pd]
    is_deep = (heights == 0) | (heights >= 2)
    deep = heights[is_deep & (P == pd)]
    n_deep = int(deep.size)
    useful = n_deep * delta1_macs(pd) + sum(theta_macs(pd, int(x)) for x in deep)
    achieved = 2.0 * useful / (deep_ms * 1e-3) / 1e12 if deep_ms > 0 else 0.0
    executed = 2.0 * n_deep * qfs.mfma_per_surface(pd) * 16384 / (deep_ms * 1e-3) / 1e12 if deep_ms > 0 else 0.0
    per_prime = {}
    for q in (3, 5, 7, 11):
        n_q = int((P == q).sum())
        if n_q:
            t_q = per_call["deep_p%d" % q] + per_call["stage1"] * n_q / B + per_call["plan"] / 4
            per_prime[str(q)] = {"surfaces": n_q, "deep_surfaces": int((is_deep & (P == q)).sum()),
                                 "deep_kernel_ms": per_call["deep_p%d" % q],
                                 "quartics_per_s": n_q / (t_q * 1e-3) if t_q > 0 else None}
    traffic = measured_traffic(args.workload)
    print("bench: %.1f ms/step, stages %s, deep surfaces %d" % (1e3 * elapsed / args.steps,
          {k: round(v, 3) for k, v in per_call.items()}, n_deep), file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": B * args.steps / elapsed,
        "unit": "quartics/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "ms_per_step_median": step_ms[len(step_ms) // 2] if step_ms else None,
        "cold_first_call_ms": cold_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "%s: %s, bound 10" % (args.workload, WORKLOADS.get(args.workload, "")),
                   "p": sorted(int(q) for q in np.unique(P)), "batch": B, "bound": 10},
        "parity_vs_oracle": parity,
        "roofline": {
            "bound": "mfma",
            "kernel": "k_deep<%d> (Delta_1 chain on v_mfma_i32_16x16x64_i8 + theta)" % pd,
            "achieved": achieved,
            "peak": INT8_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved / INT8_PEAK_TOPS,
            "traffic": traffic,
            "traffic_unit": "bytes/launch",
            "traffic_gbps": traffic / (deep_ms * 1e-3) / 1e9 if traffic and deep_ms > 0 else None,
            "traffic_profile": TRAFFIC["profile"] if traffic else None,
            "kernel_ms_per_launch": deep_ms,
            "useful_ops_per_launch": 2.0 * useful,
            "deep_surfaces_per_launch": n_deep,
            "executed_mfma_tops": executed,
            "executed_mfma_frac": executed / INT8_PEAK_TOPS,
        },
        "stage_ms_per_step": per_call,
        "per_prime": per_prime,
    }

    if not args.no_baselines:
        # plain per-surface GPU kernels on the first surfaces of the dominant prime
        idx = np.nonzero(P == pd)[0][:args.plain_sample]
        n = int(idx.size)
        fs = f[torch.from_numpy(idx).cuda()].contiguous()
        hp = qfs.height_plain(fs, pd)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        hp = qfs.height_plain(fs, pd)
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        out["plain_baseline"] = {
            "value": n / (tp1 - tp0), "unit": "quartics/s", "kind": "plain per-surface VALU kernels",
            "sample": "first %d p=%d surfaces of %s" % (n, pd, args.workload),
            "agrees_with_batched": bool(np.array_equal(hp.cpu().numpy(), heights[idx])),
        }
        # batched rate of the same prime: the whole job for one-prime workloads, the per-prime rate otherwise
        batched = out["value"] if len(per_prime) == 1 else per_prime[str(pd)]["quartics_per_s"]
        out["speedup_vs_plain"] = batched / out["plain_baseline"]["value"]
        # CPU oracle on a bounded sample: the host's share of cores, then one core
        from oracle import fast
        n = min(args.cpu_sample, B)
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        tc0 = time.perf_counter()
        hc = fast.heights(F[:n], P[:n], threads=threads)
        tc1 = time.perf_counter()
        n1 = min(args.cpu_sample_single, B)
        ts0 = time.perf_counter()
        hs = fast.heights(F[:n1], P[:n1], threads=1)
        ts1 = time.perf_counter()
        out["cpu_baseline"] = {
            "value": n / (tc1 - tc0), "unit": "quartics/s", "cores": threads, "kind": "oracle",
            "sample": "first %d surfaces of %s, C oracle (oracle/qfs_oracle.c) on a thread pool" % (n, args.workload),
            "agrees_with_gpu": bool(np.array_equal(hc, heights[:n]) and np.array_equal(hs, heights[:n1])),
            "single_core": {"value": n1 / (ts1 - ts0), "unit": "quartics/s",
                            "sample": "first %d surfaces of %s" % (n1, args.workload)},
            "cpu_model": cpu_model(),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
