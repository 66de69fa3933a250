"""Throughput of exact epipolar-guided matching (retrieve + match) on one MI355X.

Workload (the at-scale configuration): image pairs of 6048x4032 px, f = 3400
px, 20000 keypoints per image (70% true matches, 30% outliers), 128-d FP32
unit descriptors, sideways motion (epipole far outside the image) and
forward motion (epipole at the image centre), each at eps = 1, 2 and 4 px.
One step processes the six (motion, eps) pairs: 120000 image-1 queries, each
retrieving its exact candidate set and selecting its best match.  Inputs are
synthetic (seeded), resident in HBM before the timed region.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is keypoint queries/s of the batched path;
`plain_gpu` is the same work through the plain path (one pipeline per pair,
host-synchronised CSR sizing, gather-based matching).
"""

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "keypoint queries/s (retrieve+match), exact candidate sets, vs plain GPU path"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4000,
                    help="queries per pair in the oracle sample")
    ap.add_argument("--algo", default="auto")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 2 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


KERNEL = "k_match_window_f32"
KERNEL_SRC = os.path.join(ROOT, "paper_2603_18401_amd", "csrc", "match_window.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_window_traffic.md")


def source_hash(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith(("source_sha256:", "traffic_bytes_per_launch:")))
    if vals.get("source_sha256", "").strip() != source_hash(KERNEL_SRC):
        return None
    try:
        return int(vals["traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def make_workload():
    import synth
    pairs, eps_list = [], []
    for motion in ("sideways", "forward"):
        base = synth.cfg1_pair(motion)
        for eps in (1.0, 2.0, 4.0):
            pairs.append(base)
            eps_list.append(eps)
    return pairs, eps_list


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}): the "
              "matching path has no multi-GPU form in this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2603_18401_amd as E

    dev = torch.device("cuda:0")
    pairs, eps_list = make_workload()
    P = len(pairs)
    m = np.array([p.m for p in pairs])
    n = np.array([p.n for p in pairs])
    kp1 = np.concatenate([p.kp1 for p in pairs])
    kp2 = np.concatenate([p.kp2 for p in pairs])
    eps2 = np.concatenate([np.full(p.n, e, np.float32) for p, e in zip(pairs, eps_list)])
    d1 = np.concatenate([p.desc1 for p in pairs])
    d2 = np.concatenate([p.desc2 for p in pairs])
    N1, N2 = int(m.sum()), int(n.sum())
    g = {k: torch.from_numpy(v).to(dev) for k, v in
         dict(kp1=kp1, kp2=kp2, eps2=eps2, d1=d1, d2=d2).items()}
    specs = [E.PairSpec(p.F, p.W, p.H, p.m, p.n) for p in pairs]
    stream = torch.cuda.current_stream(dev)

    # ---- batched path: one build/query/match over the six pairs
    idx0 = E.Index(specs, g["kp2"], eps2=g["eps2"])
    ws = idx0.workspace
    offs, cols = idx0.query(g["kp1"])
    nnz = int(offs[-1].item())
    cap = nnz
    row_offsets = torch.empty(N1 + 1, dtype=torch.int64, device=dev)
    col_indices = torch.empty(cap, dtype=torch.int32, device=dev)
    best = torch.empty(N1, dtype=torch.int32, device=dev)
    bd = torch.empty(N1, dtype=torch.float32, device=dev)
    sd = torch.empty(N1, dtype=torch.float32, device=dev)
    idx0.close()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]

    def step(ev=None):
        idx = E.Index(specs, g["kp2"], eps2=g["eps2"], workspace=ws)
        if ev:
            ev[0].record(stream)
        idx.query(g["kp1"], row_offsets=row_offsets, col_indices=col_indices, sync=False)
        if ev:
            ev[1].record(stream)
        idx.match(row_offsets, col_indices, g["d1"], g["d2"], dtype="f32", algo=args.algo,
                  out=(best, bd, sd))
        if ev:
            ev[2].record(stream)
        idx.close()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    qps = N1 * args.steps / elapsed
    query_ms = [e[0].elapsed_time(e[1]) for e in evs]
    match_ms = [e[1].elapsed_time(e[2]) for e in evs]
    assert int(row_offsets[-1].item()) == nnz

    # ---- plain path: one pipeline per pair, sized through the host
    plain = None
    if not args.no_plain:
        per = []
        for p_i in range(P):
            sl1 = slice(int(m[:p_i].sum()), int(m[:p_i + 1].sum()))
            sl2 = slice(int(n[:p_i].sum()), int(n[:p_i + 1].sum()))
            per.append(dict(spec=[specs[p_i]], kp1=g["kp1"][sl1].contiguous(),
                            kp2=g["kp2"][sl2].contiguous(), d1=g["d1"][sl1].contiguous(),
                            d2=g["d2"][sl2].contiguous(), eps=eps_list[p_i]))

        def plain_step():
            for q in per:
                idx = E.Index(q["spec"], q["kp2"], eps=q["eps"])
                o, c = idx.query(q["kp1"])
                idx.match(o, c, q["d1"], q["d2"], dtype="f32", algo="plain")
                idx.close()

        for _ in range(max(1, args.warmup)):
            plain_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ksteps = max(1, args.steps // 2)
        for _ in range(ksteps):
            plain_step()
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
        plain = {"value": N1 * ksteps / pel, "unit": "queries/s",
                 "ms_per_step": 1e3 * pel / ksteps, "steps": ksteps}

    # ---- roofline of the dominant kernel (descriptor matching)
    match_avg_ms = float(np.mean(match_ms))
    b_desc = 512
    match_bytes = N1 * (b_desc + 16 + 12) + nnz * 4 + N2 * b_desc
    achieved = match_bytes / (match_avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": KERNEL if args.algo == "auto" else args.algo,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if args.algo == "auto" else None,
                "avg_launch_ms": round(match_avg_ms, 5),
                "algorithmic_bytes_per_launch": int(match_bytes),
                "kernel_source_sha256": source_hash(KERNEL_SRC)}

    if args.calibrate_copy:
        src = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # the machine's CPU share, not the host's core count
        threads = min(16, len(os.sched_getaffinity(0)))
        s = args.cpu_sample
        t0 = time.perf_counter()
        done = 0
        for p_i, p in enumerate(pairs):
            ro, rc, _ = oracle.candidates(p.F, p.kp1[:s], p.kp2, eps_list[p_i], nthreads=threads)
            oracle.match(p.desc1[:s], p.desc2, ro, rc, nthreads=threads)
            done += min(s, p.m)
        cel = time.perf_counter() - t0
        cpu = {"value": round(done / cel, 1), "unit": "queries/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {s} queries of each of the {P} pairs against all 20000 "
                         f"keypoints ({done} queries, brute-force FP64 candidates + FP32 "
                         f"matching, {cel:.1f} s)",
               "cpu": platform.processor() or platform.machine()}

    out = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "6048x4032 pairs, 20000 keypoints/image, sideways+forward "
                               "motion x eps {1,2,4} px (6 pairs, 120000 queries per step), "
                               "FP32 descriptors",
                   "queries_per_step": N1, "candidates_per_step": nnz,
                   "kbar": round(nnz / N1, 2), "algo": args.algo,
                   "query_ms_avg": round(float(np.mean(query_ms)), 4),
                   "match_ms_avg": round(match_avg_ms, 4)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_gpu": plain,
    }
    if plain:
        out["speedup_vs_plain"] = round(qps / plain["value"], 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
