"""The DAG's data-parallel kernels in float64, each the plain definition (test infrastructure).

Sec. V builds each attention head from GEMM, transpose and softmax kernels (the matrix product
of the GEMM kernel of Sec. IV-A: C (M x N) from A (M x K) and B (K x N)); Sec. II's example adds
the element-wise vector add.  Every function takes and returns float64 arrays and never mutates
its arguments.
"""
import numpy as np


def gemm(a: np.ndarray, b: np.ndarray, alpha: float = 1.0) -> np.ndarray:
    """C = alpha * A * B (Sec. IV-A's matmul kernel; alpha carries the 1/sqrt(dh) score scale).

    The matrix product is numpy's float64 matmul, used as a library primitive.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim != 2 or b.ndim != 2 or a.shape[1] != b.shape[0]:
        raise ValueError(f"gemm shape mismatch {a.shape} x {b.shape}")
    return float(alpha) * (a @ b)


def transpose(a: np.ndarray) -> np.ndarray:
    """B[j, i] = A[i, j] (the transpose kernel producing K^T in Sec. V)."""
    return np.array(np.asarray(a, dtype=np.float64).T, copy=True)


def softmax(x: np.ndarray) -> np.ndarray:
    """Row-wise normalised exponential of Sec. V: y[i, j] = exp(x[i, j]) / sum_j exp(x[i, j]).

    Computed as exp(x - m_i) / sum_j exp(x[i, j] - m_i) with m_i the row maximum, which is the
    same value in exact arithmetic and avoids overflow.  An empty row stays empty.
    """
    x = np.asarray(x, dtype=np.float64)
    if x.shape[1] == 0:
        return x.copy()
    m = x.max(axis=1, keepdims=True)
    e = np.exp(x - m)
    return e / e.sum(axis=1, keepdims=True)


def add(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """C = A + B element-wise (the vadd kernel of Sec. II)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError(f"add shape mismatch {a.shape} vs {b.shape}")
    return a + b


def gemm_loops(a, b, alpha=1.0):
    """Triple-loop matrix product in pure Python, for tiny inputs only (a brute-force pin)."""
    m, k = len(a), len(a[0]) if len(a) else 0
    n = len(b[0]) if len(b) else 0
    out = [[0.0] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = 0.0
            for t in range(k):
                s += float(a[i][t]) * float(b[t][j])
            out[i][j] = float(alpha) * s
    return out
