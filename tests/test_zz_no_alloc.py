"""The allocation-free gradient entry point (psc_mlp_grad_static): the same results as
psc_mlp_grad on consecutive calls (the second smaller than the first, so stale scratch beyond it
must not leak in), sizes past its fixed scratch rejected, and two models sharing one GPU's array."""
import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import mlp as omlp
from gpu_helpers import normwise

pytestmark = pytest.mark.gpu

F = psc.PSC_FEATURES


def _data(seed, n):
    g = np.random.default_rng(seed)
    x = g.normal(0.0, 1.0, size=(n, F)).astype(np.float32)
    t = (0.7 * x[:, 1] - 0.4 * x[:, 2] * x[:, 5] + np.cos(x[:, 9])).astype(np.float32)
    return x, t


def _model(seed):
    m = psc.psc_mlp_create(0)
    p = workloads.mlp_init(seed, F)
    psc.psc_mlp_set_params(m, psc.mlp_flatten(p))
    return m, p


def _check(m, p, x, t):
    g_s, l_s = psc.psc_mlp_grad_static(m, x, t)
    g_a, l_a = psc.psc_mlp_grad(m, x, t)
    # same kernels, same summation order: the gradient is bit-identical
    np.testing.assert_array_equal(g_s, g_a)
    assert abs(l_s - l_a) <= 1e-12 * abs(l_a)
    # and both agree with the float64 oracle
    y0, cache = omlp.forward(p, x)
    g0 = omlp.backward(p, cache, y0, t)
    assert l_s == pytest.approx(omlp.loss(y0, t), rel=1e-5)
    gg = psc.mlp_unflatten(g_s)
    for k in omlp.NAMES:
        assert normwise(gg[k], g0[k].reshape(gg[k].shape)) < 1e-4, k


def test_two_calls_second_smaller():
    print("no-alloc grad: n=4096 then n=100", flush=True)
    m, p = _model(11)
    try:
        x1, t1 = _data(1, psc.PSC_MLP_STATIC_MAX)
        _check(m, p, x1, t1)
        x2, t2 = _data(2, 100)
        _check(m, p, x2, t2)
    finally:
        psc.psc_mlp_destroy(m)


def test_sizes_past_the_scratch_are_rejected():
    print("no-alloc grad: size limits", flush=True)
    m, _ = _model(12)
    try:
        x, t = _data(3, psc.PSC_MLP_STATIC_MAX + 1)
        with pytest.raises(psc.PscError) as e:
            psc.psc_mlp_grad_static(m, x, t)
        assert e.value.status == psc.PSC_ERR_ARG
        with pytest.raises(psc.PscError) as e:
            psc.psc_mlp_grad_static(m, x[:0], t[:0])
        assert e.value.status == psc.PSC_ERR_ARG
        # the rejection left the entry point usable
        x2, t2 = _data(4, 1)
        g, _ = psc.psc_mlp_grad_static(m, x2, t2)
        np.testing.assert_array_equal(g, psc.psc_mlp_grad(m, x2, t2)[0])
    finally:
        psc.psc_mlp_destroy(m)


def test_two_models_share_the_array():
    print("no-alloc grad: two models, alternating calls", flush=True)
    a, pa = _model(13)
    b, pb = _model(14)
    try:
        xa, ta = _data(5, 777)
        xb, tb = _data(6, 333)
        for _ in range(2):
            _check(a, pa, xa, ta)
            _check(b, pb, xb, tb)
    finally:
        psc.psc_mlp_destroy(a)
        psc.psc_mlp_destroy(b)
