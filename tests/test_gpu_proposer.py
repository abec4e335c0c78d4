"""The learned weight proposer's kernels (BF16 MFMA forward and backward, FP32
softmax / cross-entropy, Adam) against the FP64 oracle MLP.

The oracle is given the same storage precisions as the device: BF16 copies of
the weights, BF16 inputs and activations, BF16 back-propagated gradients,
FP32 biases.  What remains is FP32 accumulation order and the odd BF16
rounding that lands on the other side of a tie; the bounds below are stated
per element from the magnitudes of the operands.
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

N_IN, D = 62, 30
U_BF16 = 2.0 ** -8       # unit roundoff of BF16


@pytest.fixture(scope="module")
def ctx():
    from paper_2305_04397_amd import morap
    c = morap.Context(0)
    yield c
    c.close()


def _unflatten(flat, n_in=N_IN, d=D):
    sizes = (n_in, 256, 256, 256, d)
    out, o = [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + fo * fi].reshape(fo, fi).astype(np.float64)
        o += fo * fi
        b = flat[o:o + fo].astype(np.float64)
        o += fo
        out.append((W, b))
    assert o == flat.size
    return out


def _device_view(params):
    """What the device computes with: BF16 weights, FP32 biases."""
    return [(mlp.to_bf16(W), b) for W, b in params]


def _inputs(rng, n):
    t = np.concatenate([rng.uniform(-60, 0, (n, 10)), rng.uniform(0, 1, (n, 20))], 1)
    phi = np.concatenate([rng.uniform(-60, 0, (n, 10)), rng.uniform(0, 1, (n, 20)), rng.uniform(0, 3, (n, 2))], 1)
    return np.concatenate([t, phi], 1).astype(np.float32)


def _targets(rng, n):
    return rng.dirichlet(np.full(D, 0.3), size=n).astype(np.float32)


def test_forward_matches_oracle(ctx):
    ctx.proposer_init(N_IN, D, seed=3)
    assert ctx.proposer_params().size == 62 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 30 + 30
    rng = np.random.default_rng(0)
    X = _inputs(rng, 333)                      # ragged: not a multiple of 16 rows
    P = ctx.proposer_infer(X, D)
    params = _device_view(_unflatten(ctx.proposer_params()))
    Po, _ = mlp.forward(params, X, act_round=mlp.to_bf16)
    assert np.allclose(P.sum(1), 1.0, atol=1e-5)
    err = np.abs(P - Po)
    assert err.max() <= 5e-3 and err.mean() <= 2e-4, (err.max(), err.mean())


def test_gradients_match_oracle(ctx):
    ctx.proposer_init(N_IN, D, seed=4)
    rng = np.random.default_rng(1)
    n = 200
    X, T = _inputs(rng, n), _targets(rng, n)
    loss, g = ctx.proposer_step(X, T, apply=False)
    params = _device_view(_unflatten(ctx.proposer_params()))
    Po, cache = mlp.forward(params, X, act_round=mlp.to_bf16)
    assert loss == pytest.approx(mlp.loss(Po, T), rel=2e-3)
    go = mlp.backward(params, cache, Po, T, grad_round=mlp.to_bf16)
    gg = _unflatten(g)
    acts, _ = cache
    # per-element bound: a few BF16 units of sum_r |G[r, i]| |H[r, k]|, with
    # |G| recomputed from the oracle's own back-propagated gradients
    B = n
    gl = np.abs((Po - T) / B)
    for l in range(3, -1, -1):
        W = params[l][0]
        bound_w = 8 * U_BF16 * (gl.T @ np.abs(acts[l])) + 1e-12
        bound_b = 8 * U_BF16 * gl.sum(0) + 1e-12
        assert (np.abs(gg[l][0] - go[l][0]) <= bound_w).all(), (l, np.abs(gg[l][0] - go[l][0]).max())
        assert (np.abs(gg[l][1] - go[l][1]) <= bound_b).all(), (l, np.abs(gg[l][1] - go[l][1]).max())
        # in aggregate the two agree to the BF16 level (a dropped term or a
        # transposed operand would not)
        rel = np.linalg.norm(gg[l][0] - go[l][0]) / np.linalg.norm(go[l][0])
        assert rel <= 2e-2, (l, rel)
        if l:
            gl = (gl @ np.abs(W)) * (acts[l] > 0)


def test_adam_step_matches_oracle(ctx):
    ctx.proposer_init(N_IN, D, seed=5)
    rng = np.random.default_rng(2)
    X, T = _inputs(rng, 64), _targets(rng, 64)
    p0 = ctx.proposer_params().astype(np.float64)
    _, g = ctx.proposer_step(X, T, apply=False)
    _, g_now = ctx.proposer_step(X, T, apply=True, lr=1e-3)
    assert np.array_equal(g_now, g)     # same batch and parameters: same gradients
    p1 = ctx.proposer_params().astype(np.float64)
    params = [(W.copy(), b.copy()) for W, b in _unflatten(p0)]
    state = {}
    mlp.adam_step(params, _unflatten(g_now.astype(np.float64)), state, lr=1e-3)
    ref = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])
    # the first step moves a parameter with gradient g by lr g / (|g| + eps);
    # the device rounds the update and the parameter to FP32
    assert np.abs(p1 - ref).max() <= 2e-7 * np.abs(ref).max() + 1e-9
    # a second step from the new parameters (bias correction at t = 2)
    _, g2 = ctx.proposer_step(X, T, apply=True, lr=1e-3)
    p2 = ctx.proposer_params().astype(np.float64)
    params = [(W.copy(), b.copy()) for W, b in _unflatten(p1)]
    state["m"] = [(m[0].copy(), m[1].copy()) for m in state["m"]]
    mlp.adam_step(params, _unflatten(g2.astype(np.float64)), state, lr=1e-3)
    ref2 = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])
    assert np.abs(p2 - ref2).max() <= 4e-7 * np.abs(ref2).max() + 1e-8


def test_training_learns_a_fixed_map_and_roundtrips(ctx, tmp_path):
    ctx.proposer_init(N_IN, D, seed=6)
    rng = np.random.default_rng(3)
    n = 4096
    X = _inputs(rng, n)
    A = rng.normal(0, 0.05, (D, N_IN))
    Z = X.astype(np.float64) @ A.T
    T = np.exp(Z - Z.max(1, keepdims=True))
    T = (T / T.sum(1, keepdims=True)).astype(np.float32)
    ent = float(-(T * np.log(T)).sum(1).mean())      # the loss floor
    ctx.proposer_set_input_norm(X.mean(0), X.std(0) + 1e-3)
    losses = ctx.proposer_train(X, T, batch=512, epochs=30, lr=2e-3, seed=1)
    assert losses[-1] < losses[0]
    assert losses[-1] - ent < 0.25 * (losses[0] - ent), (losses[0], losses[-1], ent)
    P = ctx.proposer_infer(X[:50], D)
    path = str(tmp_path / "prop.bin")
    ctx.proposer_save(path)
    ctx.proposer_init(N_IN, D, seed=99)
    ctx.proposer_load(path)
    assert np.array_equal(ctx.proposer_infer(X[:50], D), P)


def test_bad_inputs(ctx):
    from paper_2305_04397_amd import morap
    ctx.proposer_init(N_IN, D, seed=7)
    rng = np.random.default_rng(4)
    X = _inputs(rng, 4)
    bad_T = np.full((4, D), 0.5, np.float32)          # rows do not sum to 1
    with pytest.raises(morap.MorapError) as e:
        ctx.proposer_step(X, bad_T)
    assert e.value.code == morap.E_INVALID
    X[0, 0] = np.nan
    with pytest.raises(morap.MorapError):
        ctx.proposer_infer(X, D)
