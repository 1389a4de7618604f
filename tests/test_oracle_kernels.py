"""Pins of the oracle's kernels against closed forms, brute force and library routines."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import kernels as K
from oracle.bf16 import round_bf16, round_f32
from oracle import dag


def test_gemm_matches_triple_loop():
    g = np.random.default_rng(1)
    for (m, k, n) in [(1, 1, 1), (3, 5, 2), (7, 4, 9), (0, 3, 2)]:
        a = g.standard_normal((m, k))
        b = g.standard_normal((k, n))
        ref = np.array(K.gemm_loops(a.tolist(), b.tolist(), 0.5)).reshape(m, n)
        np.testing.assert_allclose(K.gemm(a, b, 0.5), ref, rtol=1e-13, atol=1e-13)


def test_gemm_identity_and_transpose_rule():
    g = np.random.default_rng(2)
    a = g.standard_normal((6, 6))
    b = g.standard_normal((6, 4))
    np.testing.assert_array_equal(K.gemm(np.eye(6), b), b)
    lhs = K.transpose(K.gemm(a, b))
    rhs = K.gemm(K.transpose(b), K.transpose(a))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13)
    with pytest.raises(ValueError):
        K.gemm(a, g.standard_normal((5, 2)))


def test_transpose_hand_example_and_involution():
    a = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    np.testing.assert_array_equal(K.transpose(a), [[1.0, 4.0], [2.0, 5.0], [3.0, 6.0]])
    np.testing.assert_array_equal(K.transpose(K.transpose(a)), a)


def test_softmax_hand_examples():
    y = K.softmax(np.array([[0.0, math.log(2.0)], [5.0, 5.0]]))
    np.testing.assert_allclose(y, [[1 / 3, 2 / 3], [0.5, 0.5]], rtol=1e-15)
    y = K.softmax(np.zeros((3, 7)))
    np.testing.assert_allclose(y, np.full((3, 7), 1 / 7), rtol=1e-15)
    # one dominant entry gives a one-hot row (e^-1000 underflows to 0)
    x = np.zeros((1, 5))
    x[0, 3] = 1000.0
    np.testing.assert_array_equal(K.softmax(x), [[0, 0, 0, 1, 0]])
    # very negative rows do not underflow to 0/0
    np.testing.assert_allclose(K.softmax(np.full((1, 4), -1e4)), np.full((1, 4), 0.25))


def test_softmax_rows_sum_to_one_and_shift_invariance():
    g = np.random.default_rng(3)
    x = g.standard_normal((17, 33)) * 4
    y = K.softmax(x)
    np.testing.assert_allclose(y.sum(axis=1), 1.0, rtol=1e-14)
    assert (y > 0).all()
    np.testing.assert_allclose(K.softmax(x + 123.25), y, rtol=1e-12)
    # a row permutation of the columns permutes the outputs
    p = g.permutation(33)
    np.testing.assert_allclose(K.softmax(x[:, p]), y[:, p], rtol=1e-14)


def test_add_hand_example():
    np.testing.assert_array_equal(K.add(np.array([[1.0, -2.0]]), np.array([[0.5, 2.0]])),
                                  [[1.5, 0.0]])


def test_round_bf16_matches_torch_conversion():
    g = np.random.default_rng(4)
    x = np.concatenate([
        g.standard_normal(50000).astype(np.float32),
        (g.standard_normal(20000) * 1e-30).astype(np.float32),
        (g.standard_normal(20000) * 1e30).astype(np.float32),
        np.float32([0.0, -0.0, 1.0, 65504.0, 3.0e38, -3.0e38, 1e-40, 1e-45, -1e-42]),
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = round_bf16(x.astype(np.float64))
    np.testing.assert_array_equal(got, ref)


def test_round_bf16_ties_to_even():
    one = 1.0
    assert round_bf16(np.array([one + 2.0 ** -8]))[0] == 1.0            # tie, even is 1.0
    assert round_bf16(np.array([one + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie up to even
    assert round_bf16(np.array([one + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    assert np.isinf(round_bf16(np.array([3.4e38]))[0])


def test_round_f32_matches_numpy_cast():
    g = np.random.default_rng(5)
    x = np.concatenate([g.standard_normal(50000), g.standard_normal(1000) * 1e-40,
                        g.standard_normal(1000) * 1e38, [0.0, 2.0 ** -149, 2.0 ** -150]])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(round_f32(x), ref)


# --- fork-join DAG (Fig. 1 shape) ------------------------------------------------------------

def _run(spec, inputs, **kw):
    return dag.run_dag(spec, inputs, **kw)


def test_forkjoin_closed_forms_ternary():
    n = 32
    spec = workloads.forkjoin_spec(n)
    inp = workloads.forkjoin_inputs(0, n, ternary=True)
    a0, b0, b1, b2 = (inp[k].astype(np.float64) for k in ("A0", "B0", "B1", "B2"))
    st = _run(spec, inp)
    # integers below 2^24: exact in any summation order
    assert np.array_equal(st["C3"], np.round(st["C3"]))
    # A0 = I  =>  C0 = B0
    inp2 = dict(inp, A0=np.eye(n, dtype=np.float32))
    np.testing.assert_array_equal(_run(spec, inp2)["C0"], b0)
    # B1 = B2 = I  =>  C3 = 2 A0 B0
    inp3 = dict(inp, B1=np.eye(n, dtype=np.float32), B2=np.eye(n, dtype=np.float32))
    c0 = [[sum(a0[i, t] * b0[t, j] for t in range(n)) for j in range(n)] for i in range(n)]
    np.testing.assert_array_equal(_run(spec, inp3)["C3"], 2 * np.array(c0))
    # B2 = -B1  =>  C3 = 0
    inp4 = dict(inp, B2=-inp["B1"])
    np.testing.assert_array_equal(_run(spec, inp4)["C3"], np.zeros((n, n)))


def test_forkjoin_distributive_invariant():
    n = 48
    spec = workloads.forkjoin_spec(n)
    inp = workloads.forkjoin_inputs(1, n)
    st = _run(spec, inp)
    a0, b0, b1, b2 = (inp[k].astype(np.float64) for k in ("A0", "B0", "B1", "B2"))
    other = (a0 @ b0) @ (b1 + b2)
    np.testing.assert_allclose(st["C3"], other, rtol=1e-12, atol=1e-12)
