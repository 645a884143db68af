"""Training driver of the learned precision selector.

Labels come from the method itself (mpchol_selector_labels: per-tile
residuals measured at each class, greedy lowering under the backward-error
budget, verified by a factorization); features from mpchol_selector_features;
training runs the library's forward/backward/Adam kernels
(mpchol_mlp_train_step).  This module only orchestrates those calls and
stores the weights.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import mpchol as M

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.json")


def he_uniform_init(seed: int = 3) -> np.ndarray:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases."""
    import synth

    u = synth.uniform01(seed, M.MLP_NPARAM) * 2.0 - 1.0
    p = np.zeros(M.MLP_NPARAM, dtype=np.float64)
    layers = [(0, 64 * 8, 8), (64 * 8 + 64, 64 * 64, 64), (64 * 8 + 64 + 64 * 64 + 64, 4 * 64, 64)]
    for off, cnt, fan_in in layers:
        p[off:off + cnt] = u[off:off + cnt] * np.sqrt(6.0 / fan_in)
    return p.astype(np.float32)


def label_matrix(L, tile, rho, seed, eps, nugget=1e-8, band=1, lo16=M.LO16_F16, device=0, label_eps=None, rates=None):
    """(features [m x 8], labels [m], verified backward error) of the off-band
    tiles of one synthetic matrix; labels for the budget of `label_eps`
    (default eps), features relative to `eps`; rates: the per-class update
    rates the greedy lowering weighs time with (default: the library's)."""
    import synth

    sigma, x = synth.workload(L, seed)
    n = L * L
    nt = (n + tile - 1) // tile
    h = M.mpchol_create(n, tile, device=device, lo16=lo16, band=band)
    try:
        M.mpchol_set_generator(h, sigma, x, rho, nugget)
        labels, berr = M.mpchol_selector_labels(h, eps if label_eps is None else label_eps, nt, rates)
        feats = M.mpchol_selector_features(h, eps, nt)
    finally:
        M.mpchol_destroy(h)
    idx = [(I, J) for J in range(nt) for I in range(J + band + 1, nt)]
    X = np.array([feats[I + J * nt] for I, J in idx], dtype=np.float32).reshape(-1, 8)
    y = np.array([labels[I, J] for I, J in idx], dtype=np.int32)
    return X, y, berr


def class_weights(y) -> np.ndarray:
    """Inverse-frequency weights (mean 1 over present classes), clipped to
    [0.25, 8]; absent classes get 0."""
    cnt = np.bincount(y, minlength=4).astype(np.float64)
    present = cnt > 0
    w = np.zeros(4)
    w[present] = np.clip(cnt.sum() / cnt[present] / present.sum(), 0.25, 8.0)
    return w


def train(X, y, steps=600, lr=3e-3, alpha=2.0, seed=3, device=0, log_every=0, state=None, return_state=False):
    """Full-batch Adam on the GPU kernels; returns (params, losses), or with
    return_state (params, losses, state).  state = (params, m1, m2, step), the
    trainer's parameters, Adam moments and step count: passed back in, it
    continues the same run bit for bit (the bias corrections use the step)."""
    import torch

    m = M.mpchol_mlp_create(device)
    try:
        if state is None:
            M.mpchol_mlp_set_params(m, he_uniform_init(seed))
            s0 = 0
        else:
            M.mpchol_mlp_set_state(m, *state)
            s0 = int(state[3])
        Xt = torch.tensor(np.ascontiguousarray(X, dtype=np.float32), device=f"cuda:{device}")
        yt = torch.tensor(np.ascontiguousarray(y, dtype=np.int32), device=f"cuda:{device}")
        cw = class_weights(y)
        losses = []
        for s in range(steps):
            want = log_every and (s % log_every == 0 or s == steps - 1)
            l = M.mpchol_mlp_train_step(m, Xt, yt, cw, alpha, lr, want_loss=bool(want))
            if want:
                losses.append((s0 + s, l))
        st = M.mpchol_mlp_get_state(m)
    finally:
        M.mpchol_mlp_destroy(m)
    return (st[0], losses, st) if return_state else (st[0], losses)


def predict(params, X, device=0):
    import torch

    m = M.mpchol_mlp_create(device)
    try:
        M.mpchol_mlp_set_params(m, params)
        Xt = torch.tensor(np.ascontiguousarray(X, dtype=np.float32), device=f"cuda:{device}")
        cls = torch.zeros(X.shape[0], dtype=torch.int32, device=f"cuda:{device}")
        M.mpchol_mlp_predict(m, Xt, cls=cls)
        torch.cuda.synchronize()
        return cls.cpu().numpy()
    finally:
        M.mpchol_mlp_destroy(m)


def save(params, path=WEIGHTS, meta=None, state=None):
    """Weights (and, with state = (params, m1, m2, step) from train, the Adam
    moments and step, for a checkpoint that resumes training) as JSON; float32
    values round-trip exactly."""
    d = {"nparam": int(M.MLP_NPARAM), "params": [float(v) for v in params], "meta": meta or {}}
    if state is not None:
        d["adam"] = {"m1": [float(v) for v in state[1]], "m2": [float(v) for v in state[2]], "step": int(state[3])}
    with open(path, "w") as f:
        json.dump(d, f)


def load_checkpoint(path):
    """(params, m1, m2, step) from a file written by save(..., state=...)."""
    with open(path) as f:
        d = json.load(f)
    if "adam" not in d:
        raise ValueError(f"{path} holds weights only, no optimizer state")
    arrs = [np.array(v, dtype=np.float32) for v in (d["params"], d["adam"]["m1"], d["adam"]["m2"])]
    if any(a.size != M.MLP_NPARAM for a in arrs):
        raise ValueError(f"{path}: expected {M.MLP_NPARAM} values per array")
    return arrs[0], arrs[1], arrs[2], int(d["adam"]["step"])


def load(path=WEIGHTS) -> np.ndarray:
    with open(path) as f:
        d = json.load(f)
    p = np.array(d["params"], dtype=np.float32)
    assert p.size == M.MLP_NPARAM
    return p
