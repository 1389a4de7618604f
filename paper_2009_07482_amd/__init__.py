"""Python binding of libpsc (include/psc.h): a fine-grained DAG executor for MI355X (gfx950).

The functions below carry the C names and only marshal arguments (names to bytes, numpy/torch
buffers to pointers, exported structs to dicts); every step of scheduling and execution runs in
the native library.  Importing the package loads ``libpsc.so`` from this directory and raises
ImportError if it is missing -- there is no fallback implementation.  Build it with
``python paper_2009_07482_amd/build.py``.

Workload specs from ``workloads`` (the JSON-like DAG descriptions) are lowered onto the C ABI by
``build_dag``; ``run_spec`` runs one with host inputs and returns host outputs.

Host staging memory comes from the library (psc_host_alloc, page-locked), and this package
never initialises torch's GPU runtime: torch ships its own HIP runtime, and a second initialised
runtime in one process cannot see the GPU.  torch is used here only for CPU dtype casts.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2009_07482_amd/build.py`")
_lib = C.CDLL(LIB_PATH)

# --- constants (psc.h) ------------------------------------------------------------------------
PSC_OK = 0
STATUS = {0: "PSC_OK", -1: "PSC_ERR_ARG", -2: "PSC_ERR_NAME", -3: "PSC_ERR_SHAPE", -4: "PSC_ERR_CYCLE",
          -5: "PSC_ERR_RACE", -6: "PSC_ERR_STATE", -7: "PSC_ERR_HIP", -8: "PSC_ERR_OOM",
          -9: "PSC_ERR_UNSUPPORTED", -10: "PSC_ERR_TIMEOUT", -11: "PSC_ERR_IO"}
(PSC_ERR_ARG, PSC_ERR_NAME, PSC_ERR_SHAPE, PSC_ERR_CYCLE, PSC_ERR_RACE, PSC_ERR_STATE, PSC_ERR_HIP, PSC_ERR_OOM,
 PSC_ERR_UNSUPPORTED, PSC_ERR_TIMEOUT, PSC_ERR_IO) = range(-1, -12, -1)
PSC_F32, PSC_BF16 = 0, 1
DTYPES = {"f32": PSC_F32, "bf16": PSC_BF16}
PSC_GEMM, PSC_TRANSPOSE, PSC_SOFTMAX, PSC_ADD = 0, 1, 2, 3
KINDS = {"gemm": PSC_GEMM, "transpose": PSC_TRANSPOSE, "softmax": PSC_SOFTMAX, "add": PSC_ADD}
PSC_COARSE, PSC_FINE, PSC_DEVICE, PSC_EAGER, PSC_HEFT = 0, 1, 2, 3, 4
POLICIES = {"coarse": PSC_COARSE, "fine": PSC_FINE, "device": PSC_DEVICE, "eager": PSC_EAGER, "heft": PSC_HEFT}
PSC_MAP_RR, PSC_MAP_EFT, PSC_MAP_COMPONENT = 0, 1, 2
MAPPERS = {"rr": PSC_MAP_RR, "eft": PSC_MAP_EFT, "component": PSC_MAP_COMPONENT}
PSC_OP_H2D, PSC_OP_KERNEL, PSC_OP_D2H = 0, 1, 2
PSC_DISPATCH_HIP, PSC_DISPATCH_AQL = 0, 1
DISPATCH = {"hip": PSC_DISPATCH_HIP, "aql": PSC_DISPATCH_AQL}
OP_TYPES = {0: "h2d", 1: "kernel", 2: "d2h"}
PSC_FRONT, PSC_END, PSC_IN = 1, 2, 4


class PscError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


# --- structs ------------------------------------------------------------------------------------
class psc_kernel_params(C.Structure):
    _fields_ = [("alpha", C.c_float), ("alpha_set", C.c_int32), ("tile", C.c_int32),
                ("reserved", C.c_int32)]


class psc_sched_opts(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("mapper", C.c_int32), ("copy_stream", C.c_int32),
                ("use_graph", C.c_int32), ("record_ops", C.c_int32), ("device", C.c_int32),
                ("cost", C.c_void_p), ("host_threads", C.c_int32), ("mark_components", C.c_int32),
                ("fault_inject_op", C.c_int32), ("timeout_ms", C.c_int32), ("dispatch", C.c_int32),
                ("out_of_order", C.c_int32), ("copy_roots", C.c_int32), ("exec_per_cu", C.c_int32)]


class psc_op(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("id", "type", "kernel", "buffer", "stream", "pos",
                                          "host_order", "n_waits", "wait_off")]


class psc_host_io(C.Structure):
    _fields_ = [("name", C.c_char_p), ("host_ptr", C.c_void_p), ("bytes", C.c_size_t)]


class psc_run_stats(C.Structure):
    _fields_ = [("makespan_ms", C.c_double), ("host_enqueue_ms", C.c_double)] + [
        (n, C.c_int32) for n in ("n_ops", "n_kernels", "n_h2d", "n_d2h", "n_waits", "n_streams",
                                 "graph", "aql_packets")]


class psc_op_time(C.Structure):
    _fields_ = [("op", C.c_int32), ("stream", C.c_int32), ("start_us", C.c_float),
                ("end_us", C.c_float)]


class psc_spec_info(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_kernels", "n_buffers", "n_edges", "n_components", "gpu_queues")] + \
               [("reserved", C.c_int32 * 3)]


class psc_mlp_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("shuffle_seed", C.c_uint64),
                ("reserved", C.c_int32 * 4)]


PSC_FEATURES = 12
PSC_MLP_PARAMS = 5057
PSC_MLP_STATIC_MAX = 4096

_P = C.c_void_p
_I = C.c_int32
_I64 = C.c_int64
_S = C.c_char_p
_SIGS = {
    "psc_dag_create": [C.POINTER(_P)],
    "psc_dag_destroy": [_P],
    "psc_add_buffer": [_P, _S, _I, _I64, _I64, _S, _I64, _I64],
    "psc_add_kernel": [_P, _S, _I, C.POINTER(_S), _I, C.POINTER(_S), _I,
                       C.POINTER(psc_kernel_params), C.POINTER(_I)],
    "psc_add_edge": [_P, _I, _S, _I, _S],
    "psc_set_component": [_P, _I, _I],
    "psc_bind_device": [_P, _S, _P, C.c_size_t],
    "psc_dag_info": [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)],
    "psc_dag_from_json": [_S, C.POINTER(_S), C.POINTER(_I64), _I, C.POINTER(_P), C.POINTER(psc_spec_info)],
    "psc_buffer_desc": [_P, _I, C.c_char_p, _I, C.POINTER(_I), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I),
                        C.POINTER(_I64), C.POINTER(_I64)],
    "psc_kernel_desc": [_P, _I, C.c_char_p, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I), C.POINTER(_I),
                        C.POINTER(C.c_float), C.POINTER(_I)],
    "psc_edge_desc": [_P, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)],
    "psc_buffer_id": [_P, _S, C.POINTER(_I)],
    "psc_dag_classify": [_P, _I, C.POINTER(_I), C.POINTER(_I)],
    "psc_schedule": [_P, _I, C.POINTER(psc_sched_opts), C.POINTER(_P)],
    "psc_schedule_batch": [C.POINTER(_P), _I, _I, C.POINTER(psc_sched_opts), C.POINTER(_P)],
    "psc_sched_export": [_P, C.POINTER(psc_op), _I, C.POINTER(_I), C.POINTER(_I), _I,
                         C.POINTER(_I)],
    "psc_sched_streams": [_P, C.POINTER(_I)],
    "psc_sched_prepare": [_P],
    "psc_run": [_P, C.POINTER(psc_host_io), _I, C.POINTER(psc_run_stats)],
    "psc_sched_op_times": [_P, C.POINTER(psc_op_time), _I, C.POINTER(_I)],
    "psc_sched_device_ptr": [_P, _S, C.POINTER(_P), C.POINTER(_I64)],
    "psc_sched_queue_order": [_P, C.POINTER(_I)],
    "psc_sched_read": [_P, C.c_char_p, C.c_void_p, C.c_size_t],
    "psc_kernel_time": [_P, _I, _I, C.POINTER(C.c_float)],
    "psc_sched_destroy": [_P],
    "psc_host_alloc": [C.c_size_t, C.POINTER(_P)],
    "psc_host_free": [_P],
    "psc_device_sync": [_I],
    "psc_sched_dispatch_trace": [_P, _I, _I, C.c_uint32, C.POINTER(_I), _I, C.POINTER(_I)],
    "psc_gemm_tile_count": [C.POINTER(_I)],
    "psc_tile_cache_set": [_I, _I, _I, _I, _I, _I],
    "psc_tile_cache_get": [_I, _I, _I, _I, _I, C.POINTER(_I)],
    "psc_tile_cache_clear": [C.POINTER(_I)],
    "psc_tile_cache_key": [_I, C.c_char_p, _I],
    "psc_tile_cache_save": [C.c_char_p, C.c_char_p],
    "psc_tile_cache_load": [C.c_char_p, C.c_char_p, C.POINTER(_I)],
    "psc_mlp_save": [_P, C.c_char_p],
    "psc_mlp_load": [_P, C.c_char_p],
    "psc_mlp_file_check": [C.c_char_p, C.POINTER(_I64)],
    "psc_autotune_gemm": [_I, _I, _I, _I, _I, _I, _I, C.POINTER(_I), C.POINTER(C.c_float),
                          C.POINTER(C.c_float), _I],
    "psc_autotune_dag": [_P, _I, _I, C.POINTER(_I)],
    "psc_sched_kernel_tile": [_P, _I, C.POINTER(_I)],
    "psc_sched_executor_info": [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(C.c_uint32)],
    "psc_mlp_create": [_I, C.POINTER(_P)],
    "psc_mlp_destroy": [_P],
    "psc_mlp_set_params": [_P, C.c_void_p, _I64],
    "psc_mlp_get_params": [_P, C.c_void_p, _I64],
    "psc_mlp_set_norm": [_P, C.c_void_p, C.c_void_p],
    "psc_mlp_predict": [_P, C.c_void_p, _I64, C.c_void_p],
    "psc_mlp_grad": [_P, C.c_void_p, C.c_void_p, _I64, C.c_void_p, C.POINTER(C.c_double)],
    "psc_mlp_grad_static": [_P, C.c_void_p, C.c_void_p, _I64, C.c_void_p, C.POINTER(C.c_double)],
    "psc_mlp_train": [_P, C.c_void_p, C.c_void_p, _I64, C.POINTER(psc_mlp_train_opts), C.c_void_p],
    "psc_cost_predict": [_P, C.c_void_p, _I64, C.c_void_p],
    "psc_kernel_features": [_P, _I, _I, C.c_void_p],
    "psc_device_info": [_I, C.c_char_p, _I, C.c_char_p, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I64)],
    "psc_sched_device_tasks": [_P, _I, C.c_void_p, _I, C.POINTER(_I), C.c_void_p],
    "psc_sched_component_times": [_P, C.c_void_p, _I, C.POINTER(_I)],
    "psc_sched_aql_check": [_P, C.POINTER(_I), C.c_char_p, _I],
    "psc_sched_samples": [_P, C.c_void_p, C.c_void_p, _I, C.POINTER(_I)],
    "psc_autotune_dag_in_schedule": [_P, _I, C.POINTER(psc_sched_opts), _I, _I, _I, C.POINTER(_I)],
    "psc_autotune_schedule": [_P, _I, C.POINTER(psc_sched_opts), _I, _I, C.POINTER(_I),
                              C.POINTER(C.c_float)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int32
_lib.psc_last_error.argtypes = []
_lib.psc_last_error.restype = C.c_char_p
_lib.psc_abi_version.argtypes = []
_lib.psc_abi_version.restype = C.c_int32

EXPORTED = sorted(list(_SIGS) + ["psc_last_error", "psc_abi_version"])


def _check(status):
    if status != PSC_OK:
        raise PscError(status, _lib.psc_last_error().decode())


def _b(s):
    return None if s is None else s.encode()


# --- thin wrappers with the C names --------------------------------------------------------------
def psc_abi_version():
    return _lib.psc_abi_version()


def psc_last_error():
    return _lib.psc_last_error().decode()


def psc_dag_create():
    h = _P()
    _check(_lib.psc_dag_create(C.byref(h)))
    return h


def psc_dag_destroy(dag):
    _check(_lib.psc_dag_destroy(dag))


def psc_add_buffer(dag, name, dtype, rows, cols, view_of=None, row_off=0, col_off=0):
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    _check(_lib.psc_add_buffer(dag, _b(name), dt, int(rows), int(cols), _b(view_of), int(row_off),
                               int(col_off)))


def psc_add_kernel(dag, name, kind, inputs, outputs, alpha=None, tile=0):
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    ins = (_S * len(inputs))(*[_b(x) for x in inputs])
    outs = (_S * len(outputs))(*[_b(x) for x in outputs])
    p = psc_kernel_params(float(1.0 if alpha is None else alpha), 1, int(tile), 0)
    kid = _I()
    _check(_lib.psc_add_kernel(dag, _b(name), k, ins, len(inputs), outs, len(outputs), C.byref(p),
                               C.byref(kid)))
    return kid.value


def psc_add_edge(dag, src_kernel, src_output, dst_kernel, dst_input):
    _check(_lib.psc_add_edge(dag, int(src_kernel), _b(src_output), int(dst_kernel), _b(dst_input)))


def psc_set_component(dag, kernel, component):
    _check(_lib.psc_set_component(dag, int(kernel), int(component)))


def psc_bind_device(dag, name, dptr, nbytes):
    _check(_lib.psc_bind_device(dag, _b(name), C.c_void_p(int(dptr)), int(nbytes)))


def psc_dag_info(dag):
    a, b, c = _I(), _I(), _I()
    _check(_lib.psc_dag_info(dag, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def psc_dag_from_json(text, symbols=None):
    """The specification file (JSON text) as a new DAG; returns (dag, info dict)."""
    symbols = dict(symbols or {})
    names = (_S * max(1, len(symbols)))(*[_b(k) for k in symbols])
    vals = (_I64 * max(1, len(symbols)))(*[int(v) for v in symbols.values()])
    h = _P()
    info = psc_spec_info()
    _check(_lib.psc_dag_from_json(_b(text), names, vals, len(symbols), C.byref(h), C.byref(info)))
    return h, {f: getattr(info, f) for f, _ in psc_spec_info._fields_ if f != "reserved"}


def psc_buffer_desc(dag, bid):
    name = C.create_string_buffer(256)
    dt, par = _I(), _I()
    r, c, ro, co = _I64(), _I64(), _I64(), _I64()
    _check(_lib.psc_buffer_desc(dag, int(bid), name, 256, C.byref(dt), C.byref(r), C.byref(c), C.byref(par),
                                C.byref(ro), C.byref(co)))
    return {"name": name.value.decode(), "dtype": {PSC_F32: "f32", PSC_BF16: "bf16"}[dt.value], "rows": r.value,
            "cols": c.value, "parent": par.value, "row_off": ro.value, "col_off": co.value}


def psc_kernel_desc(dag, kid):
    name = C.create_string_buffer(256)
    kind, n_in, out, comp = _I(), _I(), _I(), _I()
    ins = (_I * 2)()
    alpha = C.c_float()
    _check(_lib.psc_kernel_desc(dag, int(kid), name, 256, C.byref(kind), ins, C.byref(n_in), C.byref(out),
                                C.byref(alpha), C.byref(comp)))
    kinds = {v: k for k, v in KINDS.items()}
    return {"name": name.value.decode(), "kind": kinds[kind.value], "inputs": list(ins)[:n_in.value],
            "output": out.value, "alpha": alpha.value, "component": comp.value}


def psc_edge_desc(dag, e):
    a, b, c, d = _I(), _I(), _I(), _I()
    _check(_lib.psc_edge_desc(dag, int(e), C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
    return a.value, b.value, c.value, d.value


def spec_from_dag(dag):
    """The DAG's buffers, kernels, edges and components as a workload spec dict (the form
    build_dag, run_spec and the oracle take)."""
    nk, nb, ne = psc_dag_info(dag)
    bufs = [psc_buffer_desc(dag, i) for i in range(nb)]
    names = [b["name"] for b in bufs]
    spec_bufs = [{"name": b["name"], "dtype": b["dtype"], "rows": b["rows"], "cols": b["cols"],
                  "view_of": names[b["parent"]] if b["parent"] >= 0 else None, "row_off": b["row_off"],
                  "col_off": b["col_off"]} for b in bufs]
    kers, comp = [], []
    for k in range(nk):
        d = psc_kernel_desc(dag, k)
        kers.append({"name": d["name"], "kind": d["kind"], "inputs": [names[i] for i in d["inputs"]],
                     "outputs": [names[d["output"]]], "alpha": d["alpha"], "tile": 0})
        comp.append(d["component"])
    edges = []
    for e in range(ne):
        sk, sb, dk, db = psc_edge_desc(dag, e)
        edges.append((sk, names[sb], dk, names[db]))
    return {"buffers": spec_bufs, "kernels": kers, "edges": edges, "component": comp}


def spec_from_json(text, symbols=None):
    """(spec dict, info dict) of a specification file, lowered by the library."""
    dag, info = psc_dag_from_json(text, symbols)
    try:
        return spec_from_dag(dag), info
    finally:
        psc_dag_destroy(dag)


def psc_buffer_id(dag, name):
    i = _I()
    _check(_lib.psc_buffer_id(dag, _b(name), C.byref(i)))
    return i.value


def psc_dag_classify(dag, component):
    nk, _, ne = psc_dag_info(dag)
    kc = (_I * max(1, nk))()
    ei = (_I * max(1, ne))()
    _check(_lib.psc_dag_classify(dag, int(component), kc, ei))
    return list(kc)[:nk], list(ei)[:ne]


def make_opts(n_streams=4, mapper="rr", copy_stream=False, use_graph=False, record_ops=False,
              device=0, cost=None, host_threads=0, mark_components=False, fault_inject_op=0,
              timeout_ms=0, dispatch="hip", out_of_order=False, copy_roots=False, exec_per_cu=0):
    o = psc_sched_opts()
    o.n_streams = int(n_streams)
    o.mapper = MAPPERS[mapper] if isinstance(mapper, str) else int(mapper)
    o.copy_stream = int(bool(copy_stream))
    o.use_graph = int(bool(use_graph))
    o.record_ops = int(bool(record_ops))
    o.device = int(device)
    o.cost = None if cost is None else C.c_void_p(int(cost.value if hasattr(cost, "value") else cost))
    o.host_threads = int(host_threads)
    o.mark_components = int(bool(mark_components))
    o.fault_inject_op = int(fault_inject_op)
    o.timeout_ms = int(timeout_ms)
    o.dispatch = DISPATCH[dispatch] if isinstance(dispatch, str) else int(dispatch)
    o.out_of_order = int(bool(out_of_order))
    o.copy_roots = int(bool(copy_roots))
    o.exec_per_cu = int(exec_per_cu)
    return o


def psc_schedule(dag, policy, opts=None, **kw):
    pol = (POLICIES[policy]
           if isinstance(policy, str) else int(policy))
    o = opts if opts is not None else make_opts(**kw)
    h = _P()
    _check(_lib.psc_schedule(dag, pol, C.byref(o), C.byref(h)))
    return h


def psc_schedule_batch(dags, policy, opts=None, **kw):
    """One schedule for the disjoint union of ``dags`` (names "<i>/<name>"; see union_spec)."""
    pol = (POLICIES[policy]
           if isinstance(policy, str) else int(policy))
    o = opts if opts is not None else make_opts(**kw)
    arr = (_P * max(1, len(dags)))(*[d.value if hasattr(d, "value") else d for d in dags])
    h = _P()
    _check(_lib.psc_schedule_batch(arr, len(dags), pol, C.byref(o), C.byref(h)))
    return h


def psc_sched_export(sched):
    n, nw = _I(), _I()
    _check(_lib.psc_sched_export(sched, None, 0, C.byref(n), None, 0, C.byref(nw)))
    ops = (psc_op * max(1, n.value))()
    waits = (_I * max(1, nw.value))()
    _check(_lib.psc_sched_export(sched, ops, n.value, C.byref(n), waits, nw.value, C.byref(nw)))
    out = []
    for i in range(n.value):
        o = ops[i]
        out.append({"id": o.id, "type": OP_TYPES[o.type], "kernel": o.kernel, "buffer": o.buffer,
                    "stream": o.stream, "pos": o.pos, "host_order": o.host_order,
                    "waits": [waits[o.wait_off + j] for j in range(o.n_waits)]})
    return out


def psc_sched_streams(sched):
    n = _I()
    _check(_lib.psc_sched_streams(sched, C.byref(n)))
    return n.value


def psc_sched_prepare(sched):
    _check(_lib.psc_sched_prepare(sched))


def psc_run(sched, io=()):
    """io: iterable of (name, host_pointer, nbytes).  Returns psc_run_stats as a dict."""
    io = list(io)
    arr = (psc_host_io * max(1, len(io)))()
    keep = []
    for i, (name, ptr, nbytes) in enumerate(io):
        nb = _b(name)
        keep.append(nb)
        arr[i] = psc_host_io(nb, C.c_void_p(int(ptr)), int(nbytes))
    st = psc_run_stats()
    _check(_lib.psc_run(sched, arr, len(io), C.byref(st)))
    return {f: getattr(st, f) for f, _ in psc_run_stats._fields_}


def psc_sched_op_times(sched):
    n = _I()
    _check(_lib.psc_sched_op_times(sched, None, 0, C.byref(n)))
    buf = (psc_op_time * max(1, n.value))()
    _check(_lib.psc_sched_op_times(sched, buf, n.value, C.byref(n)))
    return [(t.op, t.stream, t.start_us, t.end_us) for t in buf[:n.value]]


def psc_device_info(device=0):
    name, arch = C.create_string_buffer(256), C.create_string_buffer(64)
    cus, clk, mem = _I(), _I(), _I64()
    _check(_lib.psc_device_info(int(device), name, 256, arch, 64, C.byref(cus), C.byref(clk), C.byref(mem)))
    return {"name": name.value.decode(), "arch": arch.value.decode(), "compute_units": cus.value,
            "clock_mhz": clk.value, "memory_gib": mem.value / 2 ** 30}


def psc_sched_device_tasks(sched, workers):
    """Host-only plan of the device executor: ([(kernel, tile, signal)] per workgroup)."""
    import numpy as np
    n = _I()
    _check(_lib.psc_sched_device_tasks(sched, int(workers), None, 0, C.byref(n), None))
    t = np.zeros((max(1, n.value), 3), np.int32)
    off = np.zeros(int(workers) + 1, np.int32)
    _check(_lib.psc_sched_device_tasks(sched, int(workers), t.ctypes.data, n.value, C.byref(n), off.ctypes.data))
    return [[tuple(int(v) for v in t[i]) for i in range(off[w], off[w + 1])] for w in range(int(workers))]


def psc_sched_aql_check(sched):
    """(distinct kernels, "") if AQL dispatch can run every kernel of the schedule, else (-1, reason)."""
    n = _I()
    why = C.create_string_buffer(512)
    _check(_lib.psc_sched_aql_check(sched, C.byref(n), why, 512))
    return n.value, why.value.decode()


def psc_sched_component_times(sched):
    """Microseconds from the run's start mark to the end of each task component (-1: empty)."""
    import numpy as np
    n = _I()
    _check(_lib.psc_sched_component_times(sched, None, 0, C.byref(n)))
    out = np.zeros(max(1, n.value), np.float32)
    _check(_lib.psc_sched_component_times(sched, out.ctypes.data, n.value, C.byref(n)))
    return out[:n.value]


def psc_sched_samples(sched):
    """Cost-model samples of the last recorded run: (features [n, 12] float32, ln us [n])."""
    import numpy as np
    n = _I()
    _check(_lib.psc_sched_samples(sched, None, None, 0, C.byref(n)))
    f = np.zeros((max(1, n.value), PSC_FEATURES), np.float32)
    t = np.zeros(max(1, n.value), np.float32)
    _check(_lib.psc_sched_samples(sched, f.ctypes.data, t.ctypes.data, n.value, C.byref(n)))
    return f[:n.value], t[:n.value]


def _f32(a, shape=None):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def psc_mlp_create(device=0):
    h = _P()
    _check(_lib.psc_mlp_create(int(device), C.byref(h)))
    return h


def psc_mlp_destroy(m):
    _check(_lib.psc_mlp_destroy(m))


def psc_mlp_set_params(m, flat):
    flat = _f32(flat, (-1,))
    _check(_lib.psc_mlp_set_params(m, flat.ctypes.data, flat.size))


def psc_mlp_get_params(m):
    import numpy as np
    out = np.zeros(PSC_MLP_PARAMS, np.float32)
    _check(_lib.psc_mlp_get_params(m, out.ctypes.data, out.size))
    return out


def psc_mlp_set_norm(m, mean, std):
    mean, std = _f32(mean, (PSC_FEATURES,)), _f32(std, (PSC_FEATURES,))
    _check(_lib.psc_mlp_set_norm(m, mean.ctypes.data, std.ctypes.data))


def psc_mlp_predict(m, x):
    import numpy as np
    x = _f32(x, (-1, PSC_FEATURES))
    y = np.zeros(x.shape[0], np.float32)
    _check(_lib.psc_mlp_predict(m, x.ctypes.data, x.shape[0], y.ctypes.data))
    return y


def psc_mlp_grad(m, x, t):
    """(flat gradient [PSC_MLP_PARAMS], loss) of the mean squared error at the current parameters."""
    import numpy as np
    x = _f32(x, (-1, PSC_FEATURES))
    t = _f32(t, (-1,))
    g = np.zeros(PSC_MLP_PARAMS, np.float32)
    loss = C.c_double()
    _check(_lib.psc_mlp_grad(m, x.ctypes.data, t.ctypes.data, x.shape[0], g.ctypes.data, C.byref(loss)))
    return g, loss.value


def psc_mlp_grad_static(m, x, t):
    """psc_mlp_grad through the entry point that allocates no device memory (its scratch is a
    fixed per-GPU array; at most PSC_MLP_STATIC_MAX rows)."""
    import numpy as np
    x = _f32(x, (-1, PSC_FEATURES))
    t = _f32(t, (-1,))
    g = np.zeros(PSC_MLP_PARAMS, np.float32)
    loss = C.c_double()
    _check(_lib.psc_mlp_grad_static(m, x.ctypes.data, t.ctypes.data, x.shape[0], g.ctypes.data, C.byref(loss)))
    return g, loss.value


def psc_mlp_train(m, x, t, epochs=50, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, shuffle_seed=0):
    """Mini-batch Adam on the GPU; returns the per-epoch training loss."""
    import numpy as np
    x = _f32(x, (-1, PSC_FEATURES))
    t = _f32(t, (-1,))
    o = psc_mlp_train_opts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                           int(shuffle_seed))
    losses = np.zeros(int(epochs), np.float32)
    _check(_lib.psc_mlp_train(m, x.ctypes.data, t.ctypes.data, x.shape[0], C.byref(o), losses.ctypes.data))
    return losses


def psc_kernel_features(dag, kernel, in_flight=0):
    import numpy as np
    f = np.zeros(PSC_FEATURES, np.float32)
    _check(_lib.psc_kernel_features(dag, int(kernel), int(in_flight), f.ctypes.data))
    return f


def psc_cost_predict(x, m=None):
    """Predicted microseconds of feature rows under the MLP ``m`` or, with m None, the heuristic."""
    import numpy as np
    x = _f32(x, (-1, PSC_FEATURES))
    us = np.zeros(x.shape[0], np.float32)
    _check(_lib.psc_cost_predict(m, x.ctypes.data, x.shape[0], us.ctypes.data))
    return us


# flat parameter layout of the cost model
MLP_LAYOUT = (("W1", (64, PSC_FEATURES)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)),
              ("b3", (1,)))


def mlp_flatten(params):
    import numpy as np
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k, _ in MLP_LAYOUT])


def mlp_unflatten(flat):
    import numpy as np
    out, off = {}, 0
    for k, shp in MLP_LAYOUT:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[off:off + n]).reshape(shp)
        off += n
    return out


def psc_sched_device_ptr(sched, name):
    p, ld = _P(), _I64()
    _check(_lib.psc_sched_device_ptr(sched, _b(name), C.byref(p), C.byref(ld)))
    return p.value, ld.value


def psc_sched_read(sched, name, rows, cols, dtype):
    """Current device contents of buffer ``name`` (rows x cols of ``dtype``) as float32."""
    es = 2 if dtype == "bf16" else 4
    raw = np.empty(int(rows) * int(cols), np.uint16 if es == 2 else np.float32)
    _check(_lib.psc_sched_read(sched, _b(name), raw.ctypes.data, raw.nbytes))
    raw = raw.reshape(int(rows), int(cols))
    return from_bf16_bits(raw) if es == 2 else raw


def psc_kernel_time(sched, kernel, iters=20):
    t = C.c_float()
    _check(_lib.psc_kernel_time(sched, int(kernel), int(iters), C.byref(t)))
    return t.value


def psc_sched_dispatch_trace(sched, host_threads=0, jitter_us=0, seed=0):
    """Calls of the multi-threaded enqueue against a recording backend: [(kind, op, arg)]."""
    n = _I()
    cap = 3 * 16 * (len(psc_sched_export(sched)) + 64)
    buf = (_I * cap)()
    _check(_lib.psc_sched_dispatch_trace(sched, int(host_threads), int(jitter_us), int(seed), buf, cap,
                                         C.byref(n)))
    return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n.value)]


def _dt(x):
    return DTYPES[x] if isinstance(x, str) else int(x)


def psc_gemm_tile_count():
    n = _I()
    _check(_lib.psc_gemm_tile_count(C.byref(n)))
    return n.value


def psc_tile_cache_set(M, N, K, ab, c, tile):
    _check(_lib.psc_tile_cache_set(int(M), int(N), int(K), _dt(ab), _dt(c), int(tile)))


def psc_tile_cache_get(M, N, K, ab, c):
    t = _I()
    _check(_lib.psc_tile_cache_get(int(M), int(N), int(K), _dt(ab), _dt(c), C.byref(t)))
    return t.value


def psc_tile_cache_clear():
    n = _I()
    _check(_lib.psc_tile_cache_clear(C.byref(n)))
    return n.value


def psc_tile_cache_key(device=0):
    buf = C.create_string_buffer(256)
    _check(_lib.psc_tile_cache_key(int(device), buf, 256))
    return buf.value.decode()


def psc_tile_cache_save(path, key):
    _check(_lib.psc_tile_cache_save(os.fsencode(path), key.encode()))


def psc_tile_cache_load(path, key):
    n = _I()
    _check(_lib.psc_tile_cache_load(os.fsencode(path), key.encode(), C.byref(n)))
    return n.value


def psc_mlp_save(m, path):
    _check(_lib.psc_mlp_save(m, os.fsencode(path)))


def psc_mlp_load(m, path):
    _check(_lib.psc_mlp_load(m, os.fsencode(path)))


def psc_mlp_file_check(path):
    """Saved Adam step count of a valid cost-model file; PscError(PSC_ERR_IO) otherwise."""
    step = _I64()
    _check(_lib.psc_mlp_file_check(os.fsencode(path), C.byref(step)))
    return step.value


def psc_autotune_gemm(M, N, K, ab="f32", c="f32", iters=50, device=0):
    """Returns (best tile, best microseconds, {tile: microseconds})."""
    nt = psc_gemm_tile_count()
    best, us = _I(), C.c_float()
    arr = (C.c_float * nt)()
    _check(_lib.psc_autotune_gemm(int(device), int(M), int(N), int(K), _dt(ab), _dt(c), int(iters),
                                  C.byref(best), C.byref(us), arr, nt))
    return best.value, us.value, {t: arr[t] for t in range(1, nt)}


def psc_autotune_dag(dag, iters=50, device=0):
    n = _I()
    _check(_lib.psc_autotune_dag(dag, int(device), int(iters), C.byref(n)))
    return n.value


def psc_autotune_dag_in_schedule(dag, policy, top_k=3, iters=5, max_classes=8, **opts):
    """Tiles chosen by the schedule's makespan (the max_classes heaviest GEMM classes); returns the
    number of shape classes whose choice differs from the isolated winner."""
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    o = make_opts(**opts)
    n = _I()
    _check(_lib.psc_autotune_dag_in_schedule(dag, pol, C.byref(o), int(top_k), int(max_classes), int(iters),
                                             C.byref(n)))
    return n.value


def psc_autotune_schedule(dag, policy, candidates, iters=20):
    """candidates: list of make_opts() keyword dicts.  Returns (best index, [ms per run])."""
    pol = (POLICIES[policy]
           if isinstance(policy, str) else int(policy))
    arr = (psc_sched_opts * len(candidates))(*[make_opts(**c) for c in candidates])
    best = _I()
    ms = (C.c_float * len(candidates))()
    _check(_lib.psc_autotune_schedule(dag, pol, arr, len(candidates), int(iters), C.byref(best), ms))
    return best.value, list(ms)


def psc_sched_kernel_tile(sched, kernel):
    t = _I()
    _check(_lib.psc_sched_kernel_tile(sched, int(kernel), C.byref(t)))
    return t.value


def psc_sched_executor_info(sched):
    """(workers, workgroups per CU, tile-function group mask) of a prepared PSC_DEVICE schedule."""
    w, p, g = _I(), _I(), C.c_uint32()
    _check(_lib.psc_sched_executor_info(sched, C.byref(w), C.byref(p), C.byref(g)))
    return w.value, p.value, g.value


def psc_sched_destroy(sched):
    _check(_lib.psc_sched_destroy(sched))


# --- spec lowering and host marshalling ----------------------------------------------------------
def build_dag(spec, bind=None):
    """Lower a ``workloads`` DAG spec onto the C ABI; ``bind`` maps root names to (ptr, nbytes)."""
    dag = psc_dag_create()
    try:
        for b in spec["buffers"]:
            psc_add_buffer(dag, b["name"], b["dtype"], b["rows"], b["cols"], b["view_of"],
                           b["row_off"], b["col_off"])
        for k in spec["kernels"]:
            psc_add_kernel(dag, k["name"], k["kind"], k["inputs"], k["outputs"], k.get("alpha", 1.0),
                           k.get("tile", 0))
        for (s, sb, t, tb) in spec["edges"]:
            psc_add_edge(dag, s, sb, t, tb)
        for i, c in enumerate(spec.get("component", [])):
            if c:
                psc_set_component(dag, i, c)
        for name, (ptr, nbytes) in (bind or {}).items():
            psc_bind_device(dag, name, ptr, nbytes)
    except Exception:
        psc_dag_destroy(dag)
        raise
    return dag


def export_schedule(spec, sched):
    """The exported schedule in the validator's format (buffer ids replaced by names)."""
    names = [b["name"] for b in spec["buffers"]]
    ops = psc_sched_export(sched)
    for o in ops:
        o["buffer"] = names[o["buffer"]] if o["buffer"] >= 0 else None
    ooo = _I()
    _check(_lib.psc_sched_queue_order(sched, C.byref(ooo)))
    return {"n_streams": psc_sched_streams(sched), "ops": ops, "in_order": not ooo.value}


def to_bf16_bits(arr):
    """float32 array -> uint16 bfloat16 bit patterns (round to nearest even), via torch's CPU cast."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def from_bf16_bits(bits):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).view(torch.bfloat16)
    return t.to(torch.float32).numpy()


def psc_host_alloc(nbytes):
    p = _P()
    _check(_lib.psc_host_alloc(int(nbytes), C.byref(p)))
    return p.value


def psc_host_free(ptr):
    _check(_lib.psc_host_free(C.c_void_p(ptr)))


def psc_device_sync(device=0):
    _check(_lib.psc_device_sync(int(device)))


class HostBuffer:
    """Page-locked host memory from psc_host_alloc, viewed as a rows x cols numpy array."""

    def __init__(self, rows, cols, dtype):
        self.dtype = dtype
        es = 2 if dtype == "bf16" else 4
        self.nbytes = int(rows) * int(cols) * es
        self.ptr = psc_host_alloc(self.nbytes)
        raw = (C.c_uint8 * max(1, self.nbytes)).from_address(self.ptr)
        flat = np.frombuffer(raw, dtype=np.uint16 if es == 2 else np.float32,
                             count=int(rows) * int(cols))
        self.array = flat.reshape(int(rows), int(cols))

    def set(self, values):
        values = np.asarray(values, dtype=np.float32)
        self.array[...] = to_bf16_bits(values) if self.dtype == "bf16" else values

    def get(self):
        a = self.array
        return from_bf16_bits(a) if self.dtype == "bf16" else a.copy()

    def free(self):
        if self.ptr:
            psc_host_free(self.ptr)
            self.ptr = None
            self.array = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class _LazyOutputs(dict):
    """Read-back buffers made on first use (page-locked memory is only taken when needed)."""

    def __init__(self, by):
        super().__init__()
        self._by = by

    def __missing__(self, name):
        b = self._by[name]
        h = HostBuffer(b["rows"], b["cols"], b["dtype"])
        self[name] = h
        return h


class SpecRunner:
    """A scheduled spec with page-locked host staging for its inputs and outputs."""

    def __init__(self, spec, policy="fine", **opts):
        import workloads
        self.spec = spec
        self.by = {b["name"]: b for b in spec["buffers"]}
        self.dag = build_dag(spec)
        self.sched = psc_schedule(self.dag, policy, **opts)
        self.in_names = workloads.host_inputs_of(spec)
        self.out_names = workloads.host_outputs_of(spec)
        self.outputs = _LazyOutputs(self.by)
        self.inputs = {}

    def set_inputs(self, inputs):
        for n in self.in_names:
            if n in inputs:
                if n not in self.inputs:
                    b = self.by[n]
                    self.inputs[n] = HostBuffer(b["rows"], b["cols"], b["dtype"])
                self.inputs[n].set(inputs[n])

    def io(self, with_inputs=True, with_outputs=True):
        out = []
        if with_inputs:
            out += [(n, h.ptr, h.nbytes) for n, h in self.inputs.items()]
        if with_outputs:
            out += [(n, self.outputs[n].ptr, self.outputs[n].nbytes) for n in self.out_names]
        return out

    def run(self, with_inputs=True, with_outputs=True):
        return psc_run(self.sched, self.io(with_inputs, with_outputs))

    def result(self, name):
        return self.outputs[name].get()

    def read_device(self, name):
        """Any buffer's current device contents (intermediates included) as float32."""
        b = {x["name"]: x for x in self.spec["buffers"]}[name]
        return psc_sched_read(self.sched, name, b["rows"], b["cols"], b["dtype"])

    def export(self):
        return export_schedule(self.spec, self.sched)

    def samples(self):
        return psc_sched_samples(self.sched)

    def close(self):
        if self.sched is not None:
            psc_sched_destroy(self.sched)
            self.sched = None
        if self.dag is not None:
            psc_dag_destroy(self.dag)
            self.dag = None
        for h in list(self.inputs.values()) + list(self.outputs.values()):
            h.free()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def union_spec(specs):
    """The spec of the DAG psc_schedule_batch builds from ``specs``: names prefixed "<i>/",
    kernel indices offset, task components offset by the component counts before them."""
    bufs, kers, edges, comp = [], [], [], []
    c_off = 0
    for i, sp in enumerate(specs):
        pre, base = f"{i}/", len(kers)
        for b in sp["buffers"]:
            bufs.append(dict(b, name=pre + b["name"], view_of=None if b["view_of"] is None else pre + b["view_of"]))
        for k in sp["kernels"]:
            kers.append(dict(k, name=pre + k["name"], inputs=[pre + x for x in k["inputs"]],
                             outputs=[pre + x for x in k["outputs"]]))
        edges += [(s_ + base, pre + sb, t + base, pre + tb) for (s_, sb, t, tb) in sp["edges"]]
        cs = list(sp.get("component", [0] * len(sp["kernels"]))) or [0] * len(sp["kernels"])
        comp += [c + c_off for c in cs]
        c_off += (max(cs) + 1) if cs else 1
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": comp}


class BatchRunner(SpecRunner):
    """Several specs scheduled as one batch by psc_schedule_batch; buffers are named "<i>/<name>".
    The per-spec DAGs are destroyed right after scheduling (the schedule holds its own union)."""

    def __init__(self, specs, policy="fine", **opts):
        import workloads
        self.spec = union_spec(specs)
        self.by = {b["name"]: b for b in self.spec["buffers"]}
        dags = [build_dag(sp) for sp in specs]
        try:
            self.sched = psc_schedule_batch(dags, policy, **opts)
        finally:
            for d in dags:
                psc_dag_destroy(d)
        self.dag = None
        self.in_names = workloads.host_inputs_of(self.spec)
        self.out_names = workloads.host_outputs_of(self.spec)
        self.outputs = _LazyOutputs(self.by)
        self.inputs = {}


def run_spec(spec, inputs, policy="fine", **opts):
    """Schedule and run ``spec`` once on ``inputs``; returns ({output name: float32 array}, stats)."""
    r = SpecRunner(spec, policy, **opts)
    try:
        r.set_inputs(inputs)
        stats = r.run()
        return {n: r.result(n) for n in r.out_names}, stats
    finally:
        r.close()
