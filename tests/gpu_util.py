"""Helpers for the GPU tests: run the library on synthetic pairs and fetch
the results as NumPy arrays."""

import numpy as np


def torch_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def specs_of(pairs):
    import paper_2603_18401_amd as E
    return [E.PairSpec(p.F, p.W, p.H, p.m, p.n) for p in pairs]


def run_candidates(pairs, eps, eps2=None, kp1=None, kp2=None):
    """Builds one index over `pairs` and queries it; returns (offs, cols, idx)."""
    import paper_2603_18401_amd as E
    torch = torch_gpu()
    if kp1 is None:
        kp1 = np.concatenate([p.kp1 for p in pairs]) if pairs else np.zeros((0, 2), np.float32)
    if kp2 is None:
        kp2 = np.concatenate([p.kp2 for p in pairs]) if pairs else np.zeros((0, 2), np.float32)
    dev = torch.device("cuda:0")
    k1 = torch.from_numpy(np.ascontiguousarray(kp1, np.float32).reshape(-1, 2)).to(dev)
    k2 = torch.from_numpy(np.ascontiguousarray(kp2, np.float32).reshape(-1, 2)).to(dev)
    e2 = None if eps2 is None else torch.from_numpy(np.ascontiguousarray(eps2, np.float32)).to(dev)
    idx = E.Index(specs_of(pairs), k2, eps2=e2, eps=eps)
    offs, cols = idx.query(k1)
    torch.cuda.synchronize()
    return offs.cpu().numpy(), cols.cpu().numpy(), idx


def oracle_batch(pairs, eps, eps2=None, kp1=None, kp2=None):
    import oracle
    m = [p.m for p in pairs]
    n = [p.n for p in pairs]
    qb = np.concatenate([[0], np.cumsum(m)[:-1]]).astype(np.int64)
    kb = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    if kp1 is None:
        kp1 = np.concatenate([p.kp1 for p in pairs])
    if kp2 is None:
        kp2 = np.concatenate([p.kp2 for p in pairs])
    e = eps if eps2 is None else eps2
    return oracle.candidates_batch([p.F for p in pairs], kp1, kp2, e, qb, m, kb, n)


def assert_csr_equal(got, ref, what=""):
    go, gc = got
    ro, rc = ref
    assert go.shape == ro.shape, what
    if not np.array_equal(go, ro):
        bad = np.where(go != ro)[0]
        raise AssertionError(f"{what}: row_offsets differ at {bad[:10]} (of {len(bad)})")
    if not np.array_equal(gc, rc):
        bad = np.where(gc != rc)[0]
        raise AssertionError(f"{what}: col_indices differ at {bad[:10]} (of {len(bad)})")


def fp8_rows(d):
    """E4M3FN codes and scales of FP32 rows (synth's encoder) with an upper
    bound on |x - code * scale| per row, in FP64 from the E4M3FN definition
    and rounded up to float32: the rounding-error input of the fused FP8 pass."""
    import synth
    codes, scale = synth.f32_to_fp8_e4m3(d)
    deq = synth.fp8_e4m3_to_f32(codes).astype(np.float64) * scale.astype(np.float64)[:, None]
    err = np.sqrt(((d.astype(np.float64) - deq) ** 2).sum(axis=1)) * (1.0 + 1e-6)
    err32 = err.astype(np.float32)
    err32 = np.where(err32.astype(np.float64) < err, np.nextafter(err32, np.float32(np.inf)),
                     err32).astype(np.float32)
    return codes, scale, err32
