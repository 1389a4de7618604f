"""Shared helpers of the GPU parity tests: one-kernel specs, error measures, oracle runs."""
import numpy as np

import workloads
from oracle import dag as odag


def one_kernel_spec(kind, shapes, dtypes, alpha=1.0, tile=0):
    """Spec of a single kernel; shapes/dtypes list the inputs then the output."""
    names = ["A", "B"][: len(shapes) - 1] + ["C"]
    bufs = [{"name": n, "dtype": d, "rows": r, "cols": c, "view_of": None, "row_off": 0, "col_off": 0}
            for n, (r, c), d in zip(names, shapes, dtypes)]
    ker = {"name": "k", "kind": kind, "inputs": names[:-1], "outputs": ["C"], "alpha": alpha, "tile": tile}
    return {"buffers": bufs, "kernels": [ker], "edges": [], "component": [0]}


def normwise(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def oracle_outputs(spec, inputs, emulate=False):
    st = odag.run_dag(spec, inputs, emulate=emulate)
    return {n: odag.read_buffer(spec, st, n) for n in workloads.host_outputs_of(spec)}


def uniform(seed, shape, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(np.float32)
