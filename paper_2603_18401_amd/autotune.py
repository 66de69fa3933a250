"""Autotuner for the work distribution and tile shape of the angle-tile
kernels.

A batch of image pairs of uneven sizes can run its stabbing and matching
tiles one workgroup per tile, or as persistent launches of a few workgroups
per compute unit that take tiles from a device queue, in angle order or
longest first; the stabbing pass stages 256, 512 or 1024 window records in
LDS per round (Sched).  Which is fastest depends on the batch's shape and the
device, and every form gives the same results, so the choice is measured:
each candidate is recorded as a HIP graph of the whole batch (Batch) and
replayed a few times; the fastest is kept.

Results are cached in a JSON file keyed by the device architecture, the HIP
runtime version, the library version and the shape class of the batch
(descriptor type and the powers of two of the pair and keypoint counts).
The cache file is EPM_TUNE_CACHE if set, else ~/.cache/epm/tune.json.
"""

import json
import math
import os
import time

from . import Batch, Sched, load_library

__all__ = ["candidates", "shape_key", "tune", "cache_path"]


def cache_path():
    return os.environ.get("EPM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "epm", "tune.json"))


def _pow2(x):
    return 1 << max(0, int(math.floor(math.log2(max(int(x), 1)))))


def shape_key(torch, device, specs, dtype):
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    lib = load_library().epm_version().decode()
    n1 = sum(s.m for s in specs)
    n2 = sum(s.n for s in specs)
    return (f"{arch}|hip {torch.version.hip}|{lib}|{dtype}|pairs {_pow2(len(specs))}"
            f"|n1 {_pow2(n1)}|n2 {_pow2(n2)}")


STAB_CHUNKS = (256, 512, 1024)


def candidates(num_cus):
    """One workgroup per tile, and persistent launches of 1-3 (stabbing) and
    1-2 (matching: its LDS allows two per CU) workgroups per compute unit, in
    angle order and longest first; each with 256, 512 and 1024 window records
    per round of the stabbing pass."""
    out = []
    for ch in STAB_CHUNKS:
        out.append(Sched(0, 0, 0, ch))
        for s in (1, 2, 3):
            for m in (1, 2):
                for lpt in (0, 1):
                    out.append(Sched(s * num_cus, m * num_cus, lpt, ch))
    return out


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_batch(torch, b, steps, warmup):
    for _ in range(warmup):
        b.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def tune(specs, kp1, kp2, desc1, desc2, capacity, *, dtype="f32", eps2=None, eps=0.0,
         scale1=None, scale2=None, desc1_f32=None, desc2_f32=None, ratio=0.0,
         cache=None, use_cache=True, steps=5, warmup=2, sched_list=None, log=None):
    """Returns (best Sched, info).  info holds the key, every candidate's time
    (seconds per replay) and whether the result came from the cache.

    Every candidate's outputs are compared with the first one's, bit for bit
    (they must agree whatever the schedule); a mismatch raises."""
    import torch
    dev = kp2.device
    path = cache if cache is not None else cache_path()
    key = shape_key(torch, dev, specs, dtype)
    if use_cache:
        hit = _load(path).get(key)
        if hit is not None:
            return Sched.from_dict(hit["sched"]), {"key": key, "cached": True, **hit}
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    cand = sched_list if sched_list is not None else candidates(cus)
    ws = torch.empty(0, dtype=torch.uint8, device=dev)
    times, ref = [], None
    for sc in cand:
        b = Batch(specs, kp1, kp2, desc1, desc2, capacity, eps2=eps2, eps=eps, dtype=dtype,
                  scale1=scale1, scale2=scale2, desc1_f32=desc1_f32, desc2_f32=desc2_f32,
                  ratio=ratio, sched=sc, workspace=ws if ws.numel() else None)
        ws = b.workspace
        t = _time_batch(torch, b, steps, warmup)
        outs = [x.clone() for x in b.outputs()]
        if ref is None:
            ref = outs
        else:
            for a, r in zip(outs, ref):
                if not torch.equal(a, r):
                    raise RuntimeError(f"schedule {sc} changed the results")
        times.append(t)
        if log:
            log(f"autotune {sc}: {t * 1e3:.3f} ms")
        b.close()
        del b
    best = min(range(len(cand)), key=lambda i: times[i])
    entry = {"sched": cand[best].as_dict(), "seconds": times[best],
             "candidates": [[c.as_dict(), t] for c, t in zip(cand, times)]}
    data = _load(path)
    data[key] = entry
    _store(path, data)
    return cand[best], {"key": key, "cached": False, **entry}
