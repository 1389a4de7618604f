"""The specification-file frontend (Sec. IV-A) on the host: dag.json text lowered by the library
(psc_dag_from_json) into the same DAG a caller would build with the C calls; symbolic sizes bound
at load time; every malformed file rejected with a status that names the fault."""
import copy
import json
import os

import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import dag as odag

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig7_spec.json")


def fig7(all_gpu=True):
    doc = json.load(open(GOLDEN))
    if all_gpu:
        doc["kernels"][1]["dev"] = "gpu"
        doc["cq"] = {"gpu": 2}
    return doc


def test_fig7_as_printed_asks_for_the_cpu():
    """Kernel 1 of the paper's example is mapped to the CPU; this executor has one GPU only."""
    with pytest.raises(psc.PscError) as e:
        psc.psc_dag_from_json(json.dumps(fig7(all_gpu=False)), {"M": 2, "N": 2, "K": 3})
    assert e.value.name == "PSC_ERR_UNSUPPORTED" and "kernel 1" in str(e.value) and "cpu" in str(e.value)


def test_fig7_structure():
    spec, info = psc.spec_from_json(json.dumps(fig7()), {"M": 5, "N": 3, "K": 7})
    assert info == {"n_kernels": 3, "n_buffers": 7, "n_edges": 2, "n_components": 2, "gpu_queues": 2}
    by = {b["name"]: b for b in spec["buffers"]}
    assert [k["kind"] for k in spec["kernels"]] == ["gemm", "add", "gemm"]
    assert [(by[b]["rows"], by[b]["cols"]) for b in spec["kernels"][0]["inputs"]] == [(5, 7), (7, 3)]
    assert (by["k0_a2"]["rows"], by["k0_a2"]["cols"]) == (5, 3)
    assert (by["k1_a2"]["rows"], by["k1_a2"]["cols"]) == (3, 1)
    assert (by["k2_a2"]["rows"], by["k2_a2"]["cols"]) == (5, 1)
    # edge 0,2 -> 2,0: kernel 2's first input is kernel 0's output; 1,2 -> 2,1 likewise
    assert spec["kernels"][2]["inputs"] == ["k0_a2", "k1_a2"]
    assert spec["edges"] == [(0, "k0_a2", 2, "k0_a2"), (1, "k1_a2", 2, "k1_a2")]
    # tc = {{0,2},{1}}
    assert spec["component"] == [0, 1, 0]
    assert workloads.host_inputs_of(spec) == ["k0_a0", "k0_a1", "k1_a0", "k1_a1"]
    assert workloads.host_outputs_of(spec) == ["k2_a2"]


def test_fig7_classification():
    """Defs. 1-3 on the lowered DAG: in T1 = {0, 2} kernel 0 is FRONT and kernel 2 END (intra
    edge 0 -> 2); T2 = {1} is FRONT and END at once; the edge 1 -> 2 crosses components."""
    dag, _ = psc.psc_dag_from_json(json.dumps(fig7()), {"M": 2, "N": 2, "K": 3})
    try:
        c0, inter = psc.psc_dag_classify(dag, 0)
        c1, _ = psc.psc_dag_classify(dag, 1)
    finally:
        psc.psc_dag_destroy(dag)
    assert c0 == [psc.PSC_FRONT, 0, psc.PSC_END]
    assert c1 == [0, psc.PSC_FRONT | psc.PSC_END, 0]
    assert inter == [0, 1]


def test_fig7_worked_example_through_the_oracle():
    """The hand-worked values stored with the fixture: (A B)(u + v) = [7, 0]."""
    doc = fig7()
    ex = doc["_worked_example"]
    spec, _ = psc.spec_from_json(json.dumps(doc), ex["symbols"])
    inp = {k: np.array(v, np.float32) for k, v in ex["inputs"].items()}
    st = odag.run_dag(spec, inp)
    for name, want in ex["expected"].items():
        np.testing.assert_array_equal(odag.read_buffer(spec, st, name), np.array(want, np.float64))


def test_symbols_default_and_override():
    doc = fig7()
    doc["symbols"] = {"M": 4, "N": "M*2", "K": "(N + 2) / 2"}
    spec, _ = psc.spec_from_json(json.dumps(doc))
    by = {b["name"]: b for b in spec["buffers"]}
    assert (by["k0_a0"]["rows"], by["k0_a0"]["cols"], by["k0_a1"]["cols"]) == (4, 5, 8)
    spec, _ = psc.spec_from_json(json.dumps(doc), {"K": 9})
    by = {b["name"]: b for b in spec["buffers"]}
    assert by["k0_a0"]["cols"] == 9


def test_same_schedule_as_the_c_calls():
    """The lowered DAG schedules exactly like the DAG written with psc_add_* by hand."""
    spec_json, _ = psc.spec_from_json(json.dumps(fig7()), {"M": 64, "N": 32, "K": 16})
    hand = {"buffers": [], "kernels": [], "edges": [], "component": [0, 1, 0]}
    for name, r, c in (("k0_a0", 64, 16), ("k0_a1", 16, 32), ("k1_a0", 32, 1), ("k1_a1", 32, 1),
                       ("k0_a2", 64, 32), ("k1_a2", 32, 1), ("k2_a2", 64, 1)):
        hand["buffers"].append({"name": name, "dtype": "f32", "rows": r, "cols": c, "view_of": None,
                                "row_off": 0, "col_off": 0})
    hand["kernels"] = [{"name": "matmul_0", "kind": "gemm", "inputs": ["k0_a0", "k0_a1"], "outputs": ["k0_a2"]},
                       {"name": "vadd_1", "kind": "add", "inputs": ["k1_a0", "k1_a1"], "outputs": ["k1_a2"]},
                       {"name": "matmul_2", "kind": "gemm", "inputs": ["k0_a2", "k1_a2"], "outputs": ["k2_a2"]}]
    hand["edges"] = [(0, "k0_a2", 2, "k0_a2"), (1, "k1_a2", 2, "k1_a2")]
    for policy, kw in (("coarse", {}), ("fine", dict(n_streams=2, mapper="rr")),
                       ("fine", dict(n_streams=2, mapper="component", copy_stream=True))):
        exports = []
        for spec in (spec_json, hand):
            d = psc.build_dag(spec)
            s = psc.psc_schedule(d, policy, **kw)
            exports.append(psc.psc_sched_export(s))
            psc.psc_sched_destroy(s)
            psc.psc_dag_destroy(d)
        assert exports[0] == exports[1], (policy, kw)


def test_paper_heads_match_the_formula():
    """The paper's head DAG written as a specification file (Sec. V: Z_h = softmax(Q K^T) V W_h,
    heads concatenated) lowers to a DAG whose oracle run equals that formula."""
    heads, n = 3, 6
    spec, info = psc.spec_from_json(workloads.paper_heads_json(heads), {"n": n})
    assert info["n_kernels"] == 8 * heads and info["n_components"] == heads and info["gpu_queues"] == 4
    assert [k["kind"] for k in spec["kernels"][:8]] == ["gemm"] * 3 + ["transpose", "gemm", "softmax", "gemm", "gemm"]
    inp = workloads.paper_heads_inputs(0, heads, n)
    st = odag.run_dag(spec, {k: inp[k] for k in workloads.host_inputs_of(spec)})
    z = odag.read_buffer(spec, st, "Z")
    x = inp["X"].astype(np.float64)
    for h in range(heads):
        q, k, v = (x @ inp[f"{w}{h}"].astype(np.float64) for w in ("WQ", "WK", "WV"))
        a = q @ k.T
        e = np.exp(a - a.max(axis=1, keepdims=True))
        want = (e / e.sum(axis=1, keepdims=True)) @ v @ inp[f"W{h}"].astype(np.float64)
        np.testing.assert_allclose(z[:, h * n:(h + 1) * n], want, rtol=1e-12, atol=1e-12)


def _err(doc, symbols=None):
    text = doc if isinstance(doc, str) else json.dumps(doc)
    with pytest.raises(psc.PscError) as e:
        psc.psc_dag_from_json(text, symbols)
    return e.value


def test_malformed_json_names_line_and_column():
    e = _err('{"kernels": [\n  {"id": 0,,}]}')
    assert e.name == "PSC_ERR_ARG" and "line 2" in str(e)


def test_rejections():
    S = {"M": 2, "N": 2, "K": 3}
    d = fig7()
    assert "unbound symbol 'K'" in str(_err(d, {"M": 2, "N": 2}))
    bad = copy.deepcopy(d)
    bad["kernels"][0]["outputBuffers"][0]["size"] = "M*N+1"
    assert _err(bad, S).name == "PSC_ERR_SHAPE"
    bad = copy.deepcopy(d)
    bad["edges"][0] = "0,1 -> 2,0"            # argument 1 of kernel 0 is an input
    assert _err(bad, S).name == "PSC_ERR_NAME"
    bad = copy.deepcopy(d)
    bad["edges"][0] = "0,2 -> 2,2"            # argument 2 of kernel 2 is its output
    assert _err(bad, S).name == "PSC_ERR_NAME"
    bad = copy.deepcopy(d)
    bad["edges"][0] = "0,2 - 2,0"
    assert _err(bad, S).name == "PSC_ERR_ARG"
    bad = copy.deepcopy(d)
    bad["kernels"][1]["id"] = 0
    assert _err(bad, S).name == "PSC_ERR_ARG"
    bad = copy.deepcopy(d)
    bad["kernels"][0]["name"] = "conv2d"
    assert _err(bad, S).name == "PSC_ERR_UNSUPPORTED"
    bad = copy.deepcopy(d)
    bad["kernels"][0]["ioBuffers"] = [{"type": "float", "size": "M", "pos": 6}]
    assert _err(bad, S).name == "PSC_ERR_UNSUPPORTED"
    bad = copy.deepcopy(d)
    bad["kernels"][0]["varArguments"].pop()
    assert _err(bad, S).name == "PSC_ERR_ARG"
    bad = copy.deepcopy(d)
    bad["tc"] = [[0, 2], [1, 2]]
    assert _err(bad, S).name == "PSC_ERR_ARG"
    bad = copy.deepcopy(d)
    bad["cq"] = ["cpu:2"]
    assert _err(bad, S).name == "PSC_ERR_UNSUPPORTED"
    bad = copy.deepcopy(d)
    bad["kernels"][1]["inputBuffers"][0]["type"] = "int8"
    assert _err(bad, S).name == "PSC_ERR_ARG"
    bad = copy.deepcopy(d)                   # arguments sharing a name must agree on shape
    bad["kernels"][0]["inputBuffers"][0]["name"] = "A"
    bad["kernels"][1]["inputBuffers"][0]["name"] = "A"
    assert _err(bad, S).name == "PSC_ERR_SHAPE"
    bad = copy.deepcopy(d)                   # a default name taken by another buffer
    bad["kernels"][1]["inputBuffers"][0]["name"] = "k0_a0"
    assert _err(bad, S).name == "PSC_ERR_NAME"


def test_cycle_found_when_scheduling():
    """A file whose edges form a cycle lowers (the IR holds it) and psc_schedule refuses it."""
    doc = {"kernels": [
        {"id": i, "name": "add", "inputBuffers": [{"type": "float", "size": 4, "pos": 0},
                                                 {"type": "float", "size": 4, "pos": 1}],
         "outputBuffers": [{"type": "float", "size": 4, "pos": 2}],
         "varArguments": [{"type": "int", "pos": 3, "value": 2}, {"type": "int", "pos": 4, "value": 2}]}
        for i in range(2)], "edges": ["0,2 -> 1,0", "1,2 -> 0,0"]}
    # the two edges join k0's output with k1's input and k1's output with k0's input: two buffers
    dag, info = psc.psc_dag_from_json(json.dumps(doc))
    try:
        with pytest.raises(psc.PscError) as e:
            psc.psc_schedule(dag, "coarse")
        assert e.value.name == "PSC_ERR_CYCLE"
    finally:
        psc.psc_dag_destroy(dag)
