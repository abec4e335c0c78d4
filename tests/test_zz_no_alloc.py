"""The allocation-free proposer inference (morap_proposer_infer_noalloc)
against morap_proposer_infer: the same kernels on the same inputs, so the
outputs are bit-identical; two calls in a row, the second smaller, share the
fixed device scratch.  Device buffers come from the HIP runtime the library
itself loaded (ctypes); the test allocates them, the entry point does not."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def morap():
    from paper_2305_04397_amd import morap as m
    return m


@pytest.fixture(scope="module")
def hip(morap):
    h = ctypes.CDLL("libamdhip64.so")
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipFree.argtypes = [ctypes.c_void_p]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return h


H2D, D2H = 1, 2


def _dev(hip, nbytes):
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), nbytes) == 0
    return p.value


@pytest.mark.parametrize("n_in,d", [(62, 30), (182, 150)])
def test_noalloc_inference_equals_inference(morap, hip, n_in, d):
    rng = np.random.default_rng(n_in)
    with morap.Context(0) as ctx:
        ctx.proposer_init(n_in, d, seed=11)
        ctx.proposer_set_input_norm(rng.normal(size=n_in).astype(np.float32),
                                    rng.uniform(0.5, 2.0, size=n_in).astype(np.float32))
        for n in (1000, 37):           # the second call is smaller: stale scratch rows must not leak in
            X = rng.normal(size=(n, n_in)).astype(np.float32)
            ref = ctx.proposer_infer(X, d)
            dx, dw = _dev(hip, X.nbytes), _dev(hip, n * d * 4)
            try:
                assert hip.hipMemcpy(dx, X.ctypes.data, X.nbytes, H2D) == 0
                ctx.proposer_infer_noalloc(dx, n, dw)
                assert hip.hipDeviceSynchronize() == 0
                out = np.zeros((n, d), np.float32)
                assert hip.hipMemcpy(out.ctypes.data, dw, out.nbytes, D2H) == 0
            finally:
                hip.hipFree(dx)
                hip.hipFree(dw)
            assert np.array_equal(out, ref), (n, np.abs(out - ref).max())
            assert np.allclose(out.sum(axis=1), 1.0, atol=1e-5)


def test_noalloc_inference_rejects_too_many_rows(morap, hip):
    with morap.Context(0) as ctx:
        ctx.proposer_init(62, 30, seed=1)
        with pytest.raises(morap.MorapError) as e:
            ctx.proposer_infer_noalloc(1, 4713, 1)   # beyond the scratch; nothing is enqueued
        assert e.value.code == -6 and "4712 rows" in str(e.value)
        with pytest.raises(morap.MorapError):
            ctx.proposer_infer_noalloc(0, 10, 0)      # NULL device pointers
