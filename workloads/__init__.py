"""Seeded synthetic inputs and DAG specifications for the attention and fork-join workloads.

This module is shared by the CPU oracle (``oracle/``) and by the HIP path's tests and benchmark.
It holds no arithmetic of the method: it only draws random numbers and writes down DAG
*structure* (which kernels exist, which buffers they read and write, and which producer output
feeds which consumer input), in the shape of the paper's specification file (Sec. IV-A: kernels
with ids and names, buffers with type and size, edges ``k_i,b_r -> k_j,b_s``).

A DAG spec is a plain dict::

    {"buffers": [{"name", "dtype" ("f32"|"bf16"), "rows", "cols",
                  "view_of" (None|name), "row_off", "col_off"}],
     "kernels": [{"name", "kind" ("gemm"|"transpose"|"softmax"|"add"),
                  "inputs": [names], "outputs": [names], "alpha": float}],
     "edges":   [(src_kernel_index, src_buffer, dst_kernel_index, dst_buffer)],
     "component": [task-component id per kernel]}

Kernel semantics (defined by the oracle, computed by the HIP path): ``gemm`` C = alpha*A*B with
A (M x K), B (K x N) row-major; ``transpose`` B = A^T; ``softmax`` row-wise normalised exponential;
``add`` C = A + B.  A buffer with ``view_of`` is a rectangular window of its parent's storage.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) and are returned as float32 arrays.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng", "forkjoin_spec", "forkjoin_inputs", "mha_spec", "mha_inputs",
    "batch_lengths", "batch_spec", "batch_inputs", "random_dag_spec", "random_dag_inputs",
    "host_inputs_of", "host_outputs_of", "spec_flops", "mlp_init",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _buf(name, dtype, rows, cols, view_of=None, row_off=0, col_off=0):
    return {"name": name, "dtype": dtype, "rows": int(rows), "cols": int(cols),
            "view_of": view_of, "row_off": int(row_off), "col_off": int(col_off)}


def _ker(name, kind, inputs, outputs, alpha=1.0):
    return {"name": name, "kind": kind, "inputs": list(inputs), "outputs": list(outputs),
            "alpha": float(alpha)}


# ----------------------------------------------------------------------------------------------
# Fork-join DAG (the four-kernel example of Fig. 1: k0 feeds k1 and k2, which join in k3)
# ----------------------------------------------------------------------------------------------

def forkjoin_spec(n: int = 256, dtype: str = "f32", c0_dtype: str | None = None) -> dict:
    """k0: C0 = A0*B0; k1: C1 = C0*B1; k2: C2 = C0*B2 (k1, k2 independent); k3: C3 = C1 + C2.

    ``dtype`` is the dtype of the host inputs A0, B0, B1, B2; ``c0_dtype`` that of C0 (defaults
    to ``dtype``); C1, C2, C3 are always f32.
    """
    c0_dtype = c0_dtype or dtype
    bufs = [_buf(b, dtype, n, n) for b in ("A0", "B0", "B1", "B2")]
    bufs += [_buf("C0", c0_dtype, n, n)] + [_buf(b, "f32", n, n) for b in ("C1", "C2", "C3")]
    kers = [
        _ker("k0", "gemm", ["A0", "B0"], ["C0"]),
        _ker("k1", "gemm", ["C0", "B1"], ["C1"]),
        _ker("k2", "gemm", ["C0", "B2"], ["C2"]),
        _ker("k3", "add", ["C1", "C2"], ["C3"]),
    ]
    edges = [(0, "C0", 1, "C0"), (0, "C0", 2, "C0"), (1, "C1", 3, "C1"), (2, "C2", 3, "C2")]
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": [0, 0, 0, 0]}


def forkjoin_inputs(seed: int, n: int = 256, ternary: bool = False) -> dict:
    """A0, B0, B1, B2 drawn in that order: U[-1, 1) float32, or integers {-1, 0, 1}."""
    g = rng(seed)
    out = {}
    for name in ("A0", "B0", "B1", "B2"):
        if ternary:
            out[name] = g.integers(-1, 2, size=(n, n)).astype(np.float32)
        else:
            out[name] = g.uniform(-1.0, 1.0, size=(n, n)).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------------
# Multi-head attention inference DAG (Sec. V, the per-head chain of the transformer layer)
# ----------------------------------------------------------------------------------------------

def mha_spec(n: int, d: int, heads: int, layers: int = 1, gemm_dtype: str = "f32",
             prefix: str = "", x_name: str | None = None, weight_prefix: str | None = None,
             final_dtype: str = "f32") -> dict:
    """One or more stacked attention layers as a DAG of gemm/transpose/softmax kernels.

    Per layer l and head h (head dim dh = d/heads, columns [h*dh, (h+1)*dh) of the weights):
      q: Q = X*Wq_h,  k: K = X*Wk_h,  v: V = X*Wv_h      (three independent GEMMs)
      kt: Kt = K^T                                       (transpose)
      s: S = (1/sqrt(dh)) * Q*Kt                         (GEMM, FP32 output)
      p: P = softmax(S)                                  (row softmax)
      o: O_h = P*V, written into columns [h*dh, (h+1)*dh) of Ocat
    join: Y = Ocat*Wo; Y of layer l is X of layer l+1.

    ``gemm_dtype`` is the storage dtype of X, the weights and every GEMM operand (Q, K, V, Kt, P,
    Ocat, intermediate Y); S is always f32; the last layer's Y has ``final_dtype``.
    ``prefix`` namespaces instance-private buffers and kernels; ``weight_prefix`` (default
    ``prefix``) namespaces the weight buffers, so several instances can share one weight set.
    """
    assert d % heads == 0
    dh = d // heads
    wp = prefix if weight_prefix is None else weight_prefix
    alpha = 1.0 / math.sqrt(dh)
    gd = gemm_dtype
    bufs, kers, edges, comp = [], [], [], []
    names = set()

    def add_buf(*a, **k):
        b = _buf(*a, **k)
        if b["name"] not in names:
            names.add(b["name"])
            bufs.append(b)

    x = x_name or f"{prefix}X"
    add_buf(x, gd, n, d)
    prev_y_kernel = None
    for l in range(layers):
        for w in ("Wq", "Wk", "Wv", "Wo"):
            add_buf(f"{wp}{w}{l}", gd, d, d)
        ocat = f"{prefix}Ocat{l}"
        add_buf(ocat, gd, n, d)
        o_kernels = []
        for h in range(heads):
            t = f"{prefix}L{l}H{h}"
            for w in ("Wq", "Wk", "Wv"):
                add_buf(f"{wp}{w}{l}_h{h}", gd, d, dh, view_of=f"{wp}{w}{l}", col_off=h * dh)
            for b in ("Q", "K", "V"):
                add_buf(f"{t}_{b}", gd, n, dh)
            add_buf(f"{t}_Kt", gd, dh, n)
            add_buf(f"{t}_S", "f32", n, n)
            add_buf(f"{t}_P", gd, n, n)
            add_buf(f"{t}_O", gd, n, dh, view_of=ocat, col_off=h * dh)
            base = len(kers)
            kq, kk, kv, kkt, ks, kp, ko = range(base, base + 7)
            kers += [
                _ker(f"{t}_q", "gemm", [x, f"{wp}Wq{l}_h{h}"], [f"{t}_Q"]),
                _ker(f"{t}_k", "gemm", [x, f"{wp}Wk{l}_h{h}"], [f"{t}_K"]),
                _ker(f"{t}_v", "gemm", [x, f"{wp}Wv{l}_h{h}"], [f"{t}_V"]),
                _ker(f"{t}_kt", "transpose", [f"{t}_K"], [f"{t}_Kt"]),
                _ker(f"{t}_s", "gemm", [f"{t}_Q", f"{t}_Kt"], [f"{t}_S"], alpha=alpha),
                _ker(f"{t}_p", "softmax", [f"{t}_S"], [f"{t}_P"]),
                _ker(f"{t}_o", "gemm", [f"{t}_P", f"{t}_V"], [f"{t}_O"]),
            ]
            comp += [h] * 7
            if prev_y_kernel is not None:
                for kid in (kq, kk, kv):
                    edges.append((prev_y_kernel, x, kid, x))
            edges += [
                (kk, f"{t}_K", kkt, f"{t}_K"),
                (kq, f"{t}_Q", ks, f"{t}_Q"),
                (kkt, f"{t}_Kt", ks, f"{t}_Kt"),
                (ks, f"{t}_S", kp, f"{t}_S"),
                (kp, f"{t}_P", ko, f"{t}_P"),
                (kv, f"{t}_V", ko, f"{t}_V"),
            ]
            o_kernels.append((ko, f"{t}_O"))
        y = f"{prefix}Y{l}"
        add_buf(y, gd if l < layers - 1 else final_dtype, n, d)
        ky = len(kers)
        kers.append(_ker(f"{prefix}L{l}_y", "gemm", [ocat, f"{wp}Wo{l}"], [y]))
        comp.append(heads)
        for ko, oname in o_kernels:
            edges.append((ko, oname, ky, ocat))
        prev_y_kernel = ky
        x = y
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": comp}


def mha_inputs(seed: int, n: int, d: int, layers: int = 1, prefix: str = "",
               weights: bool = True, weight_prefix: str | None = None) -> dict:
    """X ~ N(0, 1) (n x d), then per layer Wq, Wk, Wv, Wo ~ N(0, 1/d) (d x d), in that order."""
    g = rng(seed)
    wp = prefix if weight_prefix is None else weight_prefix
    out = {f"{prefix}X": g.standard_normal((n, d)).astype(np.float32)}
    if weights:
        s = 1.0 / math.sqrt(d)
        for l in range(layers):
            for w in ("Wq", "Wk", "Wv", "Wo"):
                out[f"{wp}{w}{l}"] = (g.standard_normal((d, d)) * s).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------------
# Batched serving: many attention-DAG instances of uneven sequence length sharing one weight set
# ----------------------------------------------------------------------------------------------

def batch_lengths(seed: int, count: int = 64, lo: int = 64, hi: int = 2048) -> list[int]:
    """n_i = round(exp(U(ln lo, ln hi))), clamped to [lo, hi] (log-uniform lengths)."""
    g = rng(seed)
    u = g.uniform(math.log(lo), math.log(hi), size=count)
    return [int(min(hi, max(lo, round(math.exp(v))))) for v in u]


def batch_spec(lengths, d: int = 512, heads: int = 8, layers: int = 6,
               gemm_dtype: str = "bf16") -> dict:
    """One DAG holding every instance (disconnected components) over one shared weight set."""
    bufs, kers, edges, comp = [], [], [], []
    seen = set()
    for i, n in enumerate(lengths):
        sp = mha_spec(n, d, heads, layers, gemm_dtype, prefix=f"i{i}_", weight_prefix="")
        base = len(kers)
        for b in sp["buffers"]:
            if b["name"] not in seen:
                seen.add(b["name"])
                bufs.append(b)
        kers += sp["kernels"]
        edges += [(s + base, sb, t + base, tb) for (s, sb, t, tb) in sp["edges"]]
        comp += [i] * len(sp["kernels"])
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": comp}


def batch_inputs(seed: int, lengths, d: int = 512, layers: int = 6) -> dict:
    """Shared weights first (per layer Wq, Wk, Wv, Wo ~ N(0, 1/d)), then X_i ~ N(0, 1) per instance."""
    g = rng(seed)
    s = 1.0 / math.sqrt(d)
    out = {}
    for l in range(layers):
        for w in ("Wq", "Wk", "Wv", "Wo"):
            out[f"{w}{l}"] = (g.standard_normal((d, d)) * s).astype(np.float32)
    for i, n in enumerate(lengths):
        out[f"i{i}_X"] = g.standard_normal((n, d)).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------------
# Random layered DAGs (timing corpus for the cost model)
# ----------------------------------------------------------------------------------------------

def random_dag_spec(seed: int, n_nodes: tuple = (50, 500), width: tuple = (1, 16),
                    dim: tuple = (64, 4096), dtype: str | None = None) -> dict:
    """A layered DAG of gemm / softmax / transpose / add nodes with consistent shapes.

    Node kinds are drawn with probabilities gemm 1/2, softmax, transpose, add 1/6 each.  Every
    node in a layer after the first takes a primary input from a node of an earlier layer; a GEMM
    takes its B operand (K x N, N ~ U[dim]) from the host, an add takes a second earlier node of
    the same shape when one exists and otherwise a host buffer.  First-layer nodes read host
    buffers of shape U[dim] x U[dim].  ``dtype`` None draws f32 or bf16 per DAG.
    """
    g = rng(seed)
    total = int(g.integers(n_nodes[0], n_nodes[1] + 1))
    dt = dtype or ("f32" if g.integers(0, 2) == 0 else "bf16")
    bufs, kers, edges = [], [], []
    outputs = []          # (kernel index, buffer name, rows, cols)
    layer_of = []
    host_count = 0

    def host(rows, cols):
        nonlocal host_count
        name = f"h{host_count}"
        host_count += 1
        bufs.append(_buf(name, dt, rows, cols))
        return name

    def dimv():
        return int(g.integers(dim[0], dim[1] + 1))

    layer = 0
    while len(kers) < total:
        w = int(g.integers(width[0], width[1] + 1))
        w = min(w, total - len(kers))
        earlier = list(range(len(outputs)))
        for _ in range(w):
            kid = len(kers)
            r = g.random()
            kind = "gemm" if r < 0.5 else ("softmax" if r < 4 / 6 else ("transpose" if r < 5 / 6 else "add"))
            out_name = f"t{kid}"
            if layer == 0 or not earlier:
                rows, cols = dimv(), dimv()
                a_name, a_src = host(rows, cols), None
            else:
                a_src = earlier[int(g.integers(0, len(earlier)))]
                _, a_name, rows, cols = outputs[a_src]
            ins = [a_name]
            srcs = [(a_src, a_name)]
            alpha = 1.0
            if kind == "gemm":
                nn = dimv()
                ins.append(host(cols, nn))
                srcs.append((None, None))
                orows, ocols = rows, nn
            elif kind == "transpose":
                orows, ocols = cols, rows
            elif kind == "softmax":
                orows, ocols = rows, cols
            else:
                same = [e for e in earlier if outputs[e][2] == rows and outputs[e][3] == cols and e != a_src]
                if same and layer > 0:
                    b_src = same[int(g.integers(0, len(same)))]
                    ins.append(outputs[b_src][1])
                    srcs.append((b_src, outputs[b_src][1]))
                else:
                    ins.append(host(rows, cols))
                    srcs.append((None, None))
                orows, ocols = rows, cols
            out_dtype = "f32" if kind == "softmax" and dt == "f32" else dt
            bufs.append(_buf(out_name, out_dtype, orows, ocols))
            kers.append(_ker(f"n{kid}", kind, ins, [out_name], alpha))
            for s, bname in srcs:
                if s is not None:
                    edges.append((outputs[s][0], bname, kid, bname))
            outputs.append((kid, out_name, orows, ocols))
            layer_of.append(layer)
        layer += 1
    # de-duplicate edges (an add may read the same producer twice)
    seen, uniq = set(), []
    for e in edges:
        if e not in seen:
            seen.add(e)
            uniq.append(e)
    return {"buffers": bufs, "kernels": kers, "edges": uniq, "component": [0] * len(kers),
            "dtype": dt, "layer": layer_of}


def random_dag_inputs(seed: int, spec: dict) -> dict:
    """Every host buffer of ``spec`` ~ U[-1, 1) float32, drawn in buffer order.

    A host buffer used as a GEMM B operand (K x N) is drawn from U[-r, r) with r = sqrt(3/K)
    (variance 1/K), so chains of GEMMs keep their magnitude instead of growing without bound.
    """
    g = rng(seed + 7919)
    b_operand = {k["inputs"][1] for k in spec["kernels"] if k["kind"] == "gemm"}
    out = {}
    for name in host_inputs_of(spec):
        b = next(x for x in spec["buffers"] if x["name"] == name)
        r = math.sqrt(3.0 / b["rows"]) if name in b_operand else 1.0
        out[name] = g.uniform(-r, r, size=(b["rows"], b["cols"])).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------------
# Structural helpers (no arithmetic)
# ----------------------------------------------------------------------------------------------

def _root(spec, name):
    by = {b["name"]: b for b in spec["buffers"]}
    b = by[name]
    while b["view_of"] is not None:
        b = by[b["view_of"]]
    return b["name"]


def host_inputs_of(spec: dict) -> list[str]:
    """Root buffers of the isolated writes: inputs that no edge feeds (Sec. III, isolated copy)."""
    fed = {(t, tb) for (_, _, t, tb) in spec["edges"]}
    seen, out = set(), []
    for ki, k in enumerate(spec["kernels"]):
        for b in k["inputs"]:
            if (ki, b) not in fed:
                r = _root(spec, b)
                if r not in seen:
                    seen.add(r)
                    out.append(r)
    return out


def host_outputs_of(spec: dict) -> list[str]:
    """Buffers of the isolated reads: outputs that feed no edge."""
    src = {(s, sb) for (s, sb, _, _) in spec["edges"]}
    out = []
    for ki, k in enumerate(spec["kernels"]):
        for b in k["outputs"]:
            if (ki, b) not in src and b not in out:
                out.append(b)
    return out


def spec_flops(spec: dict) -> float:
    """Algorithmic multiply-add count x 2 of the GEMM nodes (2*M*N*K each)."""
    by = {b["name"]: b for b in spec["buffers"]}
    f = 0.0
    for k in spec["kernels"]:
        if k["kind"] == "gemm":
            a, b = by[k["inputs"][0]], by[k["inputs"][1]]
            f += 2.0 * a["rows"] * a["cols"] * b["cols"]
    return f


def mlp_init(seed: int, n_features: int, hidden: int = 64) -> dict:
    """Initial cost-model weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias,
    drawn in the order W1, b1, W2, b2, W3, b3 (float32)."""
    g = rng(seed)
    shapes = [("W1", (hidden, n_features), n_features), ("b1", (hidden,), n_features),
              ("W2", (hidden, hidden), hidden), ("b2", (hidden,), hidden),
              ("W3", (1, hidden), hidden), ("b3", (1,), hidden)]
    out = {}
    for name, shape, fan_in in shapes:
        r = 1.0 / math.sqrt(fan_in)
        out[name] = g.uniform(-r, r, size=shape).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------------
# The paper's own head DAG as a specification file (Sec. V with the JSON form of Sec. IV-A)
# ----------------------------------------------------------------------------------------------

def paper_heads_json(heads: int, dtype: str = "float", queues: int = 4) -> str:
    """JSON text of the transformer layer as the paper draws it (Sec. V): per head h, with X and
    every per-head weight beta x beta (symbol ``n``),
      0: Q = X*WQ_h   1: K = X*WK_h   2: V = X*WV_h      (matmul)
      3: Kt = K^T                                          (transpose)
      4: A = Q*Kt                                          (matmul, no scaling)
      5: B = softmax(A)                                    (softmax)
      6: C = B*V                                           (matmul)
      7: Z_h = C*W_h, written into columns [h*n, (h+1)*n) of Z, the concatenation (matmul)
    Kernel ids 8h..8h+7, one task component per head, ``queues`` GPU command queues.  Inputs
    are the buffers named X, WQ<h>, WK<h>, WV<h>, W<h>; the output is Z (n x heads*n)."""
    import json as _json
    t = dtype

    def mm(kid, ins, out, m, nn, k):
        return {"id": kid, "name": "matmul", "dev": "gpu", "workDimension": 2, "globalWorkSize": [m, nn, 1],
                "inputBuffers": [dict(b, pos=i) for i, b in enumerate(ins)],
                "outputBuffers": [dict(out, pos=2)],
                "varArguments": [{"type": "int", "pos": 3, "value": m}, {"type": "int", "pos": 4, "value": nn},
                                 {"type": "int", "pos": 5, "value": k}]}

    kernels, edges, tc = [], [], []
    for h in range(heads):
        b = 8 * h
        sq = {"type": t, "size": "n*n"}
        kernels += [
            mm(b + 0, [dict(sq, name="X"), dict(sq, name=f"WQ{h}")], sq, "n", "n", "n"),
            mm(b + 1, [dict(sq, name="X"), dict(sq, name=f"WK{h}")], sq, "n", "n", "n"),
            mm(b + 2, [dict(sq, name="X"), dict(sq, name=f"WV{h}")], sq, "n", "n", "n"),
            {"id": b + 3, "name": "transpose", "dev": "gpu", "workDimension": 2, "globalWorkSize": ["n", "n", 1],
             "inputBuffers": [dict(sq, pos=0)], "outputBuffers": [dict(sq, pos=1)],
             "varArguments": [{"type": "int", "pos": 2, "value": "n"}, {"type": "int", "pos": 3, "value": "n"}]},
            mm(b + 4, [sq, sq], dict(sq, type="float"), "n", "n", "n"),
            {"id": b + 5, "name": "softmax", "dev": "gpu", "workDimension": 1, "globalWorkSize": ["n", 1, 1],
             "inputBuffers": [{"type": "float", "size": "n*n", "pos": 0}], "outputBuffers": [dict(sq, pos=1)],
             "varArguments": [{"type": "int", "pos": 2, "value": "n"}, {"type": "int", "pos": 3, "value": "n"}]},
            mm(b + 6, [sq, sq], sq, "n", "n", "n"),
            mm(b + 7, [sq, dict(sq, name=f"W{h}")],
               {"type": "float", "size": "n*n", "name": f"Z{h}", "view_of": "Z", "row_off": 0,
                "col_off": f"{h}*n"}, "n", "n", "n"),
        ]
        edges += [f"{b + 0},2 -> {b + 4},0", f"{b + 1},2 -> {b + 3},0", f"{b + 3},1 -> {b + 4},1",
                  f"{b + 4},2 -> {b + 5},0", f"{b + 5},1 -> {b + 6},0", f"{b + 2},2 -> {b + 6},1",
                  f"{b + 6},2 -> {b + 7},0"]
        tc.append(list(range(b, b + 8)))
    doc = {"symbols": {"n": 256},
           "buffers": [{"name": "Z", "type": "float", "rows": "n", "cols": f"{heads}*n"}],
           "kernels": kernels, "edges": edges, "tc": tc, "cq": {"gpu": queues}}
    return _json.dumps(doc, indent=1)


def paper_heads_inputs(seed: int, heads: int, n: int) -> dict:
    """X ~ N(0, 1) (n x n), then per head WQ, WK, WV, W ~ N(0, 1/n) (n x n), in that order."""
    g = rng(seed)
    out = {"X": g.standard_normal((n, n)).astype(np.float32)}
    s = 1.0 / math.sqrt(n)
    for h in range(heads):
        for w in ("WQ", "WK", "WV", "W"):
            out[f"{w}{h}"] = (g.standard_normal((n, n)) * s).astype(np.float32)
    return out


# ----------------------------------------------------------------------------------------------
# Attention with the add-tree join: Y = sum_h O_h * Wo[h*dh:(h+1)*dh, :]
# ----------------------------------------------------------------------------------------------

def mha_addtree_spec(n: int, d: int, heads: int, gemm_dtype: str = "f32") -> dict:
    """One attention layer whose join is a sum of per-head projections instead of one projection
    of the concatenated heads: head h's output O_h (n x dh) times the row window h of Wo
    (dh x d) gives a partial P_h (n x d, f32); the partials are summed pairwise, in a balanced
    binary tree of add kernels, into Y (f32).  Heads and their partial projections are one task
    component each; the adds are one more.  Inputs as ``mha_inputs`` with layers = 1."""
    assert d % heads == 0
    dh = d // heads
    gd = gemm_dtype
    alpha = 1.0 / math.sqrt(dh)
    bufs = [_buf("X", gd, n, d)] + [_buf(f"{w}0", gd, d, d) for w in ("Wq", "Wk", "Wv", "Wo")]
    kers, edges, comp = [], [], []
    level = []   # (kernel index, buffer name) of each partial
    for h in range(heads):
        t = f"L0H{h}"
        for w in ("Wq", "Wk", "Wv"):
            bufs.append(_buf(f"{w}0_h{h}", gd, d, dh, view_of=f"{w}0", col_off=h * dh))
        bufs.append(_buf(f"Wo0_r{h}", gd, dh, d, view_of="Wo0", row_off=h * dh))
        for b in ("Q", "K", "V", "O"):
            bufs.append(_buf(f"{t}_{b}", gd, n, dh))
        bufs += [_buf(f"{t}_Kt", gd, dh, n), _buf(f"{t}_S", "f32", n, n), _buf(f"{t}_P", gd, n, n),
                 _buf(f"{t}_Y", "f32", n, d)]
        kq, kk, kv, kkt, ks, kp, ko, ky = range(len(kers), len(kers) + 8)
        kers += [
            _ker(f"{t}_q", "gemm", ["X", f"Wq0_h{h}"], [f"{t}_Q"]),
            _ker(f"{t}_k", "gemm", ["X", f"Wk0_h{h}"], [f"{t}_K"]),
            _ker(f"{t}_v", "gemm", ["X", f"Wv0_h{h}"], [f"{t}_V"]),
            _ker(f"{t}_kt", "transpose", [f"{t}_K"], [f"{t}_Kt"]),
            _ker(f"{t}_s", "gemm", [f"{t}_Q", f"{t}_Kt"], [f"{t}_S"], alpha=alpha),
            _ker(f"{t}_p", "softmax", [f"{t}_S"], [f"{t}_P"]),
            _ker(f"{t}_o", "gemm", [f"{t}_P", f"{t}_V"], [f"{t}_O"]),
            _ker(f"{t}_y", "gemm", [f"{t}_O", f"Wo0_r{h}"], [f"{t}_Y"]),
        ]
        comp += [h] * 8
        edges += [(kk, f"{t}_K", kkt, f"{t}_K"), (kq, f"{t}_Q", ks, f"{t}_Q"), (kkt, f"{t}_Kt", ks, f"{t}_Kt"),
                  (ks, f"{t}_S", kp, f"{t}_S"), (kp, f"{t}_P", ko, f"{t}_P"), (kv, f"{t}_V", ko, f"{t}_V"),
                  (ko, f"{t}_O", ky, f"{t}_O")]
        level.append((ky, f"{t}_Y"))
    depth = 0
    while len(level) > 1:
        nxt = []
        for i in range(0, len(level) - 1, 2):
            (ka, a), (kb, b) = level[i], level[i + 1]
            out = "Y0" if len(level) == 2 else f"sum{depth}_{i // 2}"
            bufs.append(_buf(out, "f32", n, d))
            kid = len(kers)
            kers.append(_ker(f"add{depth}_{i // 2}", "add", [a, b], [out]))
            comp.append(heads)
            edges += [(ka, a, kid, a), (kb, b, kid, b)]
            nxt.append((kid, out))
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
        depth += 1
    if heads == 1:   # no add: the single partial is the output
        bufs[-1]["name"] = "Y0"
        kers[-1]["outputs"] = ["Y0"]
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": comp}


# ----------------------------------------------------------------------------------------------
# Back-to-back inferences: several attention instances in one schedule, sharing one weight set
# ----------------------------------------------------------------------------------------------

def pipeline_spec(count: int, n: int, d: int, heads: int, layers: int = 1, gemm_dtype: str = "f32") -> dict:
    """``count`` independent inferences of the attention DAG over the same weights, instance i
    its own X<i>/Y<i> and kernels ("i<i>_" prefix), one task component per instance and head
    (so a clustering mapper spreads each instance's heads); with copy streams the upload of
    inference i+1 and the read-back of inference i overlap compute of its neighbours."""
    bufs, kers, edges, comp = [], [], [], []
    seen = set()
    for i in range(count):
        s = mha_spec(n, d, heads, layers, gemm_dtype=gemm_dtype, prefix=f"i{i}_", weight_prefix="")
        off = len(kers)
        for b in s["buffers"]:
            if b["name"] not in seen:
                seen.add(b["name"])
                bufs.append(b)
        kers += s["kernels"]
        edges += [(a + off, x, c + off, y) for a, x, c, y in s["edges"]]
        comp += [i * (heads + 1) + c for c in s["component"]]
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": comp}


def pipeline_inputs(seed: int, count: int, n: int, d: int, layers: int = 1) -> dict:
    """The shared weights as ``mha_inputs(seed, ...)`` draws them, then X<i> ~ N(0, 1) per
    instance from ``default_rng(seed + 1 + i)``."""
    out = {k: v for k, v in mha_inputs(seed, n, d, layers).items() if k != "X"}
    for i in range(count):
        out[f"i{i}_X"] = rng(seed + 1 + i).standard_normal((n, d)).astype(np.float32)
    return out
