"""Pins of the FP64 proposer reference: central finite differences of the
loss, softmax normalisation, the closed-form logit gradient, the first Adam
step and bfloat16 rounding.  CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _small(rng):
    params = mlp.init_params(rng, sizes=(7, 9, 8, 6, 5))
    params = [(W, rng.normal(scale=0.1, size=b.shape)) for W, b in params]
    X = rng.normal(size=(4, 7))
    T = rng.dirichlet(np.ones(5), size=4)
    return params, X, T


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    params, X, T = _small(rng)
    P, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, P, T)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss(mlp.forward(params, X)[0], T)
                flat[idx] = old - h
                lm = mlp.loss(mlp.forward(params, X)[0], T)
                flat[idx] = old
                assert g.reshape(-1)[idx] == pytest.approx((lp - lm) / (2 * h), abs=1e-7)


def test_softmax_and_logit_gradient():
    rng = np.random.default_rng(1)
    z = rng.normal(size=(3, 5)) * 10
    p = mlp.softmax(z)
    assert np.allclose(p.sum(1), 1.0) and (p > 0).all()
    T = rng.dirichlet(np.ones(5), size=3)
    # d/dz of mean CE = (softmax - T)/B, checked by differences in z
    h = 1e-6
    for i in range(3):
        for k in range(5):
            zp, zm = z.copy(), z.copy()
            zp[i, k] += h
            zm[i, k] -= h
            num = (mlp.loss(mlp.softmax(zp), T) - mlp.loss(mlp.softmax(zm), T)) / (2 * h)
            assert num == pytest.approx((p[i, k] - T[i, k]) / 3, abs=1e-7)


def test_first_adam_step_is_signed_lr():
    W = np.array([[1.0, -2.0]])
    b = np.array([0.5])
    g = [(np.array([[3.0, -0.25]]), np.array([1e-3]))]
    mlp.adam_step([(W, b)], g, {}, lr=0.01, eps=1e-12)
    assert np.allclose(W, [[0.99, -1.99]]) and np.allclose(b, [0.49])


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -3.14159, 0.0])
    r = mlp.to_bf16(x)
    # bfloat16 keeps 7 fraction bits: the spacing at 1 is 2^-7
    assert r[0] == 1.0
    assert r[1] == 1.0                      # exactly half-way: ties to the even 1.0
    assert r[2] == 1.0                      # a quarter spacing rounds down
    assert r[3] == 1.0 + 2 ** -7            # three quarters rounds up
    assert abs(r[4] + 3.140625) < 1e-12 and r[5] == 0.0
