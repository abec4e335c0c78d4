"""FP64 reference of the learned weight proposer (not part of the paper: it
stands in front of the weight update of Alg. 1).

Network: x = [t; phi] (threshold point and instance features) ->
Linear -> ReLU -> Linear -> ReLU -> Linear -> ReLU -> Linear -> softmax, so the
output is a weight vector (non-negative, summing to 1, as Alg. 1 requires of
w).  Loss: cross-entropy between the target weight vector w* and the softmax
output, averaged over the batch; its gradient with respect to the logits is
(softmax - w*) / B.  Optimiser: Adam (Kingma and Ba, 2015) with bias
correction.

Parameters are a list [(W1, b1), ..., (W4, b4)] with W_l of shape
[fan_out, fan_in] (y = x W^T + b).  ``act_round`` (e.g. ``to_bf16``) mirrors a
storage precision: it is applied to the input and to every hidden activation.
"""
from __future__ import annotations

import numpy as np


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def softmax(z: np.ndarray) -> np.ndarray:
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def forward(params, X, act_round=None):
    """Returns (probabilities [B, out], cache)."""
    rnd = act_round or (lambda v: v)
    h = rnd(np.asarray(X, dtype=np.float64))
    acts = [h]
    n = len(params)
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        if l < n - 1:
            h = rnd(np.maximum(z, 0.0))
            acts.append(h)
        else:
            logits = z
    return softmax(logits), (acts, logits)


def loss(P: np.ndarray, T: np.ndarray) -> float:
    """Mean cross-entropy -sum_k T_k log P_k."""
    return float(-(T * np.log(np.maximum(P, 1e-300))).sum(axis=1).mean())


def backward(params, cache, P, T, grad_round=None):
    """Gradients [(dW1, db1), ...] of the mean cross-entropy.

    ``grad_round`` (e.g. ``to_bf16``) mirrors a storage precision of the
    back-propagated gradient: the gradient at each layer's output is rounded
    before it enters that layer's weight, bias and input gradients."""
    rnd = grad_round or (lambda v: v)
    acts, _ = cache
    B = P.shape[0]
    g = (P - T) / B                      # d loss / d logits
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        h = acts[l]
        g = rnd(g)
        grads[l] = (g.T @ h, g.sum(axis=0))
        if l > 0:
            g = (g @ W) * (acts[l] > 0)
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; ``state`` = {"t": int, "m": [...], "v": [...]}."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        for k, (p, g) in enumerate(((W, gW), (b, gb))):
            m = state["m"][l][k]
            v = state["v"][l][k]
            m *= b1
            m += (1 - b1) * g
            v *= b2
            v += (1 - b2) * g * g
            mhat = m / (1 - b1 ** t)
            vhat = v / (1 - b2 ** t)
            p -= lr * mhat / (np.sqrt(vhat) + eps)
    return params


def init_params(rng: np.random.Generator, sizes=(62, 256, 256, 256, 30)):
    """He-uniform weights, zero biases."""
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / fi)
        params.append((rng.uniform(-lim, lim, size=(fo, fi)), np.zeros(fo)))
    return params
