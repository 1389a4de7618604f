"""Executes a DAG spec on the CPU in float64, one kernel at a time (test infrastructure).

Sec. III models an application as G = <(K, B), (E_I, E_O, E)>: kernels K read input buffers and
write output buffers, and an edge of E makes a producer's output the consumer's input.  A valid
schedule dispatches the kernels in a topological order of these edges (Def. 5).  Fine- and
coarse-grained schedules only reorder independent kernels, so every valid schedule computes the
result of this plain sequential execution.

``run_dag`` takes a spec from ``workloads`` (buffers, kernels, edges) and a dict of host input
arrays (root buffer name -> float32 array), executes the kernels in a topological order (by
default Kahn's algorithm taking the smallest kernel index first) and returns the storage of every
root buffer.  Views are windows of their root's storage; unwritten storage holds NaN so a read
of data nobody produced is visible.

Modes
  exact    (default) every value is float64; the float32 host inputs are widened exactly.
  emulate  values are rounded to their buffer's storage dtype (bf16 or f32) wherever the GPU
           path stores them: host inputs before use, and each kernel's outputs.  Arithmetic
           inside a kernel stays float64.
"""
from __future__ import annotations

import heapq
import itertools

import numpy as np

from . import kernels as K
from .bf16 import round_to


def _buffers(spec):
    return {b["name"]: b for b in spec["buffers"]}


def resolve(spec, name):
    """(root name, row offset, col offset, rows, cols) of a buffer or view."""
    by = _buffers(spec)
    b = by[name]
    rows, cols = b["rows"], b["cols"]
    r0 = c0 = 0
    while b["view_of"] is not None:
        r0 += b["row_off"]
        c0 += b["col_off"]
        b = by[b["view_of"]]
    return b["name"], r0, c0, rows, cols


def predecessors(spec):
    """Kernel index -> set of kernel indices that feed it through an edge of E."""
    pred = {i: set() for i in range(len(spec["kernels"]))}
    for (s, _, t, _) in spec["edges"]:
        pred[t].add(s)
    return pred


def topological_order(spec):
    """Kahn's algorithm, smallest ready kernel index first; raises on a cycle."""
    n = len(spec["kernels"])
    pred = predecessors(spec)
    succ = {i: set() for i in range(n)}
    for t, ps in pred.items():
        for s in ps:
            succ[s].add(t)
    indeg = {i: len(pred[i]) for i in range(n)}
    ready = [i for i in range(n) if indeg[i] == 0]
    heapq.heapify(ready)
    order = []
    while ready:
        k = heapq.heappop(ready)
        order.append(k)
        for s in sorted(succ[k]):
            indeg[s] -= 1
            if indeg[s] == 0:
                heapq.heappush(ready, s)
    if len(order) != n:
        raise ValueError("the DAG has a cycle")
    return order


def is_topological(spec, order):
    pos = {k: i for i, k in enumerate(order)}
    if sorted(order) != list(range(len(spec["kernels"]))):
        return False
    return all(pos[s] < pos[t] for (s, _, t, _) in spec["edges"])


def all_topological_orders(spec, limit=100000):
    """Every topological order of the kernels (for invariance tests on tiny DAGs)."""
    n = len(spec["kernels"])
    pred = predecessors(spec)
    out = []

    def rec(done, order):
        if len(out) >= limit:
            return
        if len(order) == n:
            out.append(list(order))
            return
        for k in range(n):
            if k not in done and pred[k] <= done:
                done.add(k)
                order.append(k)
                rec(done, order)
                order.pop()
                done.remove(k)

    rec(set(), [])
    return out


def run_dag(spec, inputs, order=None, emulate=False):
    """Execute ``spec`` on ``inputs``; returns {root buffer name: float64 array}."""
    by = _buffers(spec)
    store = {}
    for b in spec["buffers"]:
        if b["view_of"] is None:
            store[b["name"]] = np.full((b["rows"], b["cols"]), np.nan, dtype=np.float64)
    for name, arr in inputs.items():
        root, r0, c0, rows, cols = resolve(spec, name)
        a = np.asarray(arr, dtype=np.float64)
        if a.shape != (rows, cols):
            raise ValueError(f"input {name}: shape {a.shape} != {(rows, cols)}")
        if emulate:
            a = round_to(a, by[name]["dtype"])
        store[root][r0:r0 + rows, c0:c0 + cols] = a

    def read(name):
        root, r0, c0, rows, cols = resolve(spec, name)
        return store[root][r0:r0 + rows, c0:c0 + cols].copy()

    def write(name, val):
        root, r0, c0, rows, cols = resolve(spec, name)
        if val.shape != (rows, cols):
            raise ValueError(f"output {name}: shape {val.shape} != {(rows, cols)}")
        if emulate:
            val = round_to(val, by[name]["dtype"])
        store[root][r0:r0 + rows, c0:c0 + cols] = val

    if order is None:
        order = topological_order(spec)
    elif not is_topological(spec, order):
        raise ValueError("order is not a topological order of the DAG")
    for ki in order:
        k = spec["kernels"][ki]
        ins = [read(b) for b in k["inputs"]]
        kind = k["kind"]
        if kind == "gemm":
            out = K.gemm(ins[0], ins[1], k.get("alpha", 1.0))
        elif kind == "transpose":
            out = K.transpose(ins[0])
        elif kind == "softmax":
            out = K.softmax(ins[0])
        elif kind == "add":
            out = K.add(ins[0], ins[1])
        else:
            raise ValueError(f"unknown kernel kind {kind!r}")
        write(k["outputs"][0], out)
    return store


def read_buffer(spec, store, name):
    """The window of ``store`` that buffer ``name`` (root or view) denotes."""
    root, r0, c0, rows, cols = resolve(spec, name)
    return store[root][r0:r0 + rows, c0:c0 + cols]


def count_orders(spec):
    """Number of topological orders (brute force; tiny DAGs only)."""
    n = len(spec["kernels"])
    pred = predecessors(spec)
    return sum(1 for p in itertools.permutations(range(n))
               if all(set(pred[k]) <= set(p[:i]) for i, k in enumerate(p)))
