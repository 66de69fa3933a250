"""Learned per-keypoint tolerance: binding and training loop.

The candidate test takes one tolerance per image-2 keypoint (Eq. 3-4), and the
paper names predicting it from keypoint attributes as future work (Sec. 6).
Here a 6 -> 64 -> 64 -> 1 ReLU network (include/epm.h, epm_eps_*) predicts
eps_j = clamp(softplus(z), 0.5, 8) px from (scale, response, orientation,
normalised position, distance to the epipole).  It is trained on point-line
residuals of matches the method itself accepts at a generous fixed
tolerance, with a pinball loss at a high quantile, so that eps_j covers the
residual of a true match with that probability; a fixed scalar tolerance
stays the fallback.

Every arithmetic step runs in the library's HIP kernels: features, BF16
inference, FP32 forward/backward with deterministic reductions, Adam, and the
FP64 residuals.  This module marshals arguments and draws the minibatch
order (host RNG, passed to the kernels as indices).
"""


import numpy as np

from . import Index, _check, _dptr, _pair_array, _stream, _torch, load_library

__all__ = ["NPARAM", "features", "infer", "residual_targets", "Trainer"]

NPARAM = 4673


def _workspace(torch, lib, device, num_pairs):
    n = lib.epm_eps_workspace_bytes(int(num_pairs))
    return torch.empty(n, dtype=torch.uint8, device=device)


def features(specs, kp2, attrs, stream=None):
    """[N2, 6] float32 features of the image-2 keypoints of a batch of pairs.
    attrs: [N2, 3] float32 (scale px, response, orientation rad)."""
    torch = _torch()
    lib = load_library()
    pairs, _, n2 = _pair_array(specs)
    if tuple(kp2.shape) != (n2, 2) or tuple(attrs.shape) != (n2, 3):
        raise ValueError("kp2 must be [N2, 2] and attrs [N2, 3]")
    out = torch.empty((n2, 6), dtype=torch.float32, device=kp2.device)
    ws = _workspace(torch, lib, kp2.device, len(specs))
    st = lib.epm_eps_features(pairs, len(specs), _dptr(kp2.contiguous()),
                              _dptr(attrs.contiguous()), _dptr(out), _dptr(ws), ws.numel(),
                              _stream(torch, kp2.device, stream))
    _check(st, "epm_eps_features")
    return out


def infer(feat, params, stream=None):
    """eps2 [N] float32 from features [N, 6] (BF16 weights, FP32 arithmetic)."""
    torch = _torch()
    lib = load_library()
    eps = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
    st = lib.epm_eps_infer(_dptr(feat.contiguous()), feat.shape[0], _dptr(params), _dptr(eps),
                           _stream(torch, feat.device, stream))
    _check(st, "epm_eps_infer")
    return eps


def residual_targets(specs, kp1, kp2, desc1, desc2, eps=8.0, ratio=0.8, stream=None):
    """The method's own matches at a fixed tolerance and Lowe ratio: per query
    the point-line residual of its accepted match (or -1) and the global
    image-2 row of that match (or -1)."""
    torch = _torch()
    lib = load_library()
    idx = Index(specs, kp2, eps=eps, stream=stream)
    offs, cols = idx.query(kp1)
    best, _, _ = idx.match(offs, cols, desc1, desc2, dtype="f32", ratio=ratio)
    res = torch.empty(idx.n1, dtype=torch.float32, device=kp1.device)
    fidx = torch.empty(idx.n1, dtype=torch.int64, device=kp1.device)
    st = lib.epm_match_residuals(idx.handle, _dptr(kp1), _dptr(kp2), _dptr(best), _dptr(res),
                                 _dptr(fidx), _stream(torch, kp1.device, stream))
    _check(st, "epm_match_residuals")
    torch.cuda.current_stream(kp1.device).synchronize()
    idx.close()
    return res, fidx


class Trainer:
    """FP32 parameters with Adam moments on the device."""

    def __init__(self, params, device, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                 q=0.99, stream=None):
        torch = _torch()
        self.torch = torch
        self.lib = load_library()
        self.device = device
        p = torch.as_tensor(np.asarray(params, np.float32)).to(device)
        if p.numel() != NPARAM:
            raise ValueError(f"expected {NPARAM} parameters")
        self.params = p.contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad_buf = torch.zeros_like(self.params)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws = _workspace(torch, self.lib, device, 0)
        self.lr, self.beta1, self.beta2, self.adam_eps, self.q = lr, beta1, beta2, adam_eps, q
        self.t = 0
        self.stream = stream

    def _s(self):
        return _stream(self.torch, self.device, self.stream)

    def grad(self, feat, target, sample_idx, feat_index=None):
        """(grad [NPARAM], loss [1]) of the mean pinball loss over the listed
        samples (device tensors, written into this trainer's buffers)."""
        st = self.lib.epm_eps_grad(_dptr(feat), int(feat.shape[0]), _dptr(feat_index),
                                   _dptr(target), int(target.numel()), _dptr(sample_idx),
                                   int(sample_idx.numel()), float(self.q),
                                   _dptr(self.params), _dptr(self.grad_buf),
                                   _dptr(self.loss_buf), _dptr(self.ws), self.ws.numel(),
                                   self._s())
        _check(st, "epm_eps_grad")
        return self.grad_buf, self.loss_buf

    def adam(self):
        self.t += 1
        st = self.lib.epm_eps_adam(_dptr(self.params), _dptr(self.m), _dptr(self.v),
                                   _dptr(self.grad_buf), self.t, float(self.lr),
                                   float(self.beta1), float(self.beta2), float(self.adam_eps),
                                   self._s())
        _check(st, "epm_eps_adam")

    def step(self, feat, target, sample_idx, feat_index=None):
        self.grad(feat, target, sample_idx, feat_index)
        self.adam()
        return self.loss_buf

    def fit(self, feat, target, epochs, batch=65536, seed=0, log=None):
        """Epochs over all samples (rows of feat / target) in shuffled
        minibatches; returns the mean loss of every epoch."""
        torch = self.torch
        n = int(target.numel())
        rng = np.random.default_rng(seed)
        history = []
        for ep in range(epochs):
            order = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(self.device)
            tot = torch.zeros(1, dtype=torch.float32, device=self.device)
            nb = 0
            for b0 in range(0, n, batch):
                sl = order[b0:b0 + batch]
                tot += self.step(feat, target, sl)
                nb += 1
            history.append(float(tot.item()) / max(nb, 1))
            if log:
                log(f"epoch {ep}: pinball loss {history[-1]:.5f}")
        return history

    def params_numpy(self):
        return self.params.detach().cpu().numpy().copy()
