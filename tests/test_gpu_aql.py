"""The AQL dispatcher on the GPU: schedules written as AQL packets on HSA queues (barrier-AND
packets on completion signals for the cross-stream precedences, DMA-engine copies) give the
oracle's results, bit-identical to the HIP-stream dispatcher running the same kernels; timelines
respect every precedence; failure paths stay on the host."""
import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import validator
from gpu_helpers import normwise, oracle_outputs

pytestmark = pytest.mark.gpu

AQL = dict(dispatch="aql", timeout_ms=30000)
POLICIES = [("coarse", {}), ("fine", dict(n_streams=2, mapper="rr")), ("fine", dict(n_streams=3, mapper="rr")),
            ("fine", dict(n_streams=4, mapper="eft")), ("fine", dict(n_streams=4, mapper="component")),
            ("fine", dict(n_streams=4, mapper="rr", copy_stream=True)),
            ("fine", dict(n_streams=4, mapper="component", host_threads=1)),
            ("fine", dict(n_streams=8, mapper="rr", copy_stream=True, mark_components=True)),
            ("fine", dict(n_streams=1, mapper="rr", out_of_order=True)),
            ("fine", dict(n_streams=2, mapper="eft", out_of_order=True)),
            ("fine", dict(n_streams=4, mapper="component", copy_stream=True, out_of_order=True)),
            ("fine", dict(n_streams=3, mapper="rr", mark_components=True, out_of_order=True))]
IDS = ["-".join([p] + [f"{k}{int(v) if isinstance(v, bool) else v}" for k, v in kw.items()]) for p, kw in POLICIES]


@pytest.mark.parametrize("policy,kw", POLICIES, ids=IDS)
def test_forkjoin_ternary_bit_exact(policy, kw):
    print(f"aql forkjoin ternary {policy} {kw}", flush=True)
    spec = workloads.forkjoin_spec(256)
    inp = workloads.forkjoin_inputs(0, 256, ternary=True)
    out, st = psc.run_spec(spec, inp, policy, **kw, **AQL)
    np.testing.assert_array_equal(out["C3"], oracle_outputs(spec, inp)["C3"])
    assert st["aql_packets"] >= 4 and st["makespan_ms"] > 0


@pytest.fixture(scope="module")
def mha512():
    spec = workloads.mha_spec(512, 512, 8)
    inp = workloads.mha_inputs(0, 512, 512)
    return spec, inp, oracle_outputs(spec, inp)["Y0"]


@pytest.mark.parametrize("policy,kw", POLICIES, ids=IDS)
def test_mha_matches_oracle_and_hip_dispatch(mha512, policy, kw):
    print(f"aql mha512 {policy} {kw}", flush=True)
    spec, inp, ref = mha512
    a, _ = psc.run_spec(spec, inp, policy, **kw, **AQL)
    b, _ = psc.run_spec(spec, inp, policy, **{k: v for k, v in kw.items() if k != "out_of_order"})
    assert normwise(a["Y0"], ref) < 1e-4
    np.testing.assert_array_equal(a["Y0"], b["Y0"])


def test_repeated_runs_and_resident_data(mha512):
    spec, inp, _ = mha512
    r = psc.SpecRunner(spec, "fine", n_streams=4, mapper="component", copy_stream=True, **AQL)
    r.set_inputs(inp)
    r.run()
    first = r.result("Y0")
    for _ in range(5):
        r.outputs["Y0"].array[...] = 0
        r.run(with_inputs=False, with_outputs=True)     # inputs stay on the device
        np.testing.assert_array_equal(r.result("Y0"), first)
    st = r.run(with_inputs=False, with_outputs=False)     # no copies at all
    assert st["makespan_ms"] > 0
    r.close()


@pytest.mark.parametrize("seed", range(6))
def test_random_dags(seed):
    spec = workloads.random_dag_spec(seed, n_nodes=(20, 60), dim=(8, 200))
    inp = workloads.random_dag_inputs(seed, spec)
    ref = oracle_outputs(spec, inp)
    a, _ = psc.run_spec(spec, inp, "fine", n_streams=4, mapper="eft", **AQL)
    b, _ = psc.run_spec(spec, inp, "fine", n_streams=4, mapper="eft")
    for name, want in ref.items():
        assert normwise(a[name], want) < (1e-4 if spec["dtype"] == "f32" else 2e-2), (seed, name)
        np.testing.assert_array_equal(a[name], b[name])


@pytest.mark.parametrize("n,d,h,layers,dt", [(137, 64, 2, 2, "f32"), (200, 128, 4, 1, "bf16"), (64, 512, 8, 3, "bf16")])
def test_ragged_attention(n, d, h, layers, dt):
    spec = workloads.mha_spec(n, d, h, layers, gemm_dtype=dt)
    inp = workloads.mha_inputs(3, n, d, layers)
    out, _ = psc.run_spec(spec, inp, "fine", n_streams=4, copy_stream=True, **AQL)
    y = f"Y{layers - 1}"
    assert normwise(out[y], oracle_outputs(spec, inp)[y]) < (1e-4 if dt == "f32" else 2e-2)


def test_timeline_respects_precedences_and_overlaps_copies():
    """Per-op timestamps of an AQL run (queue profiler for kernels, DMA engine for copies): every
    edge's consumer starts after its producer ends, every copy precedes its readers, and with the
    copy streams an upload or read-back overlaps a kernel on a compute queue."""
    spec = workloads.mha_spec(512, 512, 8, layers=3, gemm_dtype="bf16")
    inp = workloads.mha_inputs(1, 512, 512, 3)
    r = psc.SpecRunner(spec, "fine", n_streams=4, mapper="component", copy_stream=True, record_ops=True, **AQL)
    r.set_inputs(inp)
    r.run()
    r.run()
    times = psc.psc_sched_op_times(r.sched)
    exp = r.export()
    r.close()
    t = {o["id"]: (tt[2], tt[3]) for tt, o in zip(times, exp["ops"])}
    kop = {o["kernel"]: o["id"] for o in exp["ops"] if o["type"] == "kernel"}
    for (s_, _, d_, _) in spec["edges"]:
        assert t[kop[s_]][1] <= t[kop[d_]][0] + 0.5, (s_, d_)
    for o in exp["ops"]:
        for w in o["waits"]:
            if o["type"] != "kernel" or exp["ops"][w]["type"] != "kernel":
                assert t[w][1] <= t[o["id"]][0] + 0.5, (w, o["id"])
    copies = [t[o["id"]] for o in exp["ops"] if o["type"] != "kernel"]
    kernels = [t[o["id"]] for o in exp["ops"] if o["type"] == "kernel"]
    overlapping = sum(1 for c in copies for k in kernels if c[0] < k[1] and k[0] < c[1])
    print(f"copy/kernel overlapping pairs: {overlapping}", flush=True)
    assert overlapping >= 1
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs


def test_component_marks():
    lengths = [1, 5, 64, 137, 33, 200]
    spec = workloads.batch_spec(lengths, 64, 2, 2)
    inp = workloads.batch_inputs(0, lengths, 64, 2)
    r = psc.SpecRunner(spec, "fine", n_streams=4, mapper="component", mark_components=True, **AQL)
    r.set_inputs(inp)
    for _ in range(3):
        st = r.run()
        done = psc.psc_sched_component_times(r.sched)
        assert done.shape == (len(lengths),) and np.all(done > 0)
        assert done.max() <= st["makespan_ms"] * 1000 + 100
    # BF16 GEMMs (the batch workload's dtype): 2e-2 against the exact oracle, tight against the
    # storage-emulating one (two layers: no room for the chain to amplify rounding differences)
    want = oracle_outputs(spec, inp)
    emul = oracle_outputs(spec, inp, emulate=True)
    for name, w in want.items():
        assert normwise(r.result(name), w) < 2e-2, name
        assert normwise(r.result(name), emul[name]) < 5e-3, name
    r.close()


def test_pageable_host_memory_rejected_before_enqueue():
    spec = workloads.forkjoin_spec(16)
    r = psc.SpecRunner(spec, "fine", n_streams=2, **AQL)
    a = np.zeros((16, 16), np.float32)      # ordinary (pageable) numpy memory
    with pytest.raises(psc.PscError) as e:
        psc.psc_run(r.sched, [("A0", a.ctypes.data, a.nbytes)])
    assert e.value.name == "PSC_ERR_ARG"
    # the schedule is still usable with page-locked memory
    r.set_inputs(workloads.forkjoin_inputs(0, 16))
    r.run()
    r.close()


def test_timeout_then_drain():
    """Eight dependent 4096^3 FP32 GEMMs under a 1 ms limit: PSC_ERR_TIMEOUT, the next run waits
    for the first, destroying waits too."""
    n, length = 4096, 8
    bufs = [{"name": b, "dtype": "f32", "rows": n, "cols": n, "view_of": None, "row_off": 0, "col_off": 0}
            for b in ["A", "B"] + [f"C{i}" for i in range(length)]]
    kers = [{"name": f"g{i}", "kind": "gemm", "inputs": ["A" if i == 0 else f"C{i - 1}", "B"],
             "outputs": [f"C{i}"], "alpha": 1.0, "tile": 1} for i in range(length)]
    edges = [(i - 1, f"C{i - 1}", i, f"C{i - 1}") for i in range(1, length)]
    spec = {"buffers": bufs, "kernels": kers, "edges": edges, "component": [0] * length}
    r = psc.SpecRunner(spec, "fine", n_streams=2, dispatch="aql", timeout_ms=1)
    try:
        for _ in range(2):
            with pytest.raises(psc.PscError) as e:
                r.run(with_inputs=False, with_outputs=False)
            assert e.value.name == "PSC_ERR_TIMEOUT"
    finally:
        r.close()


def test_options_rejected_on_the_host():
    spec = workloads.forkjoin_spec(16)
    d = psc.build_dag(spec)
    for kw, want in ((dict(use_graph=True), "PSC_ERR_ARG"), (dict(fault_inject_op=2), "PSC_ERR_UNSUPPORTED")):
        with pytest.raises(psc.PscError) as e:
            psc.psc_schedule(d, "fine", dispatch="aql", **kw)
        assert e.value.name == want
    with pytest.raises(psc.PscError):
        psc.psc_schedule(d, "device", dispatch="aql")
    psc.psc_dag_destroy(d)


@pytest.mark.parametrize("n_streams", [1, 4])
def test_out_of_order_queue_timeline(n_streams):
    """Out-of-order queues: per-op times (queue profiler) show every DAG edge and every copy
    precedence respected; the export validates as out-of-order queues; the results equal the
    in-order AQL schedule's bit for bit."""
    spec = workloads.mha_spec(512, 512, 8, layers=3, gemm_dtype="bf16")
    inp = workloads.mha_inputs(2, 512, 512, 3)
    r = psc.SpecRunner(spec, "fine", n_streams=n_streams, mapper="component", record_ops=True,
                       out_of_order=True, **AQL)
    r.set_inputs(inp)
    r.run()
    r.run()
    times = psc.psc_sched_op_times(r.sched)
    exp = r.export()
    got = r.result("Y2")
    r.close()
    assert exp["in_order"] is False
    t = {o["id"]: (tt[2], tt[3]) for tt, o in zip(times, exp["ops"])}
    for o in exp["ops"]:
        for w in o["waits"]:
            assert t[w][1] <= t[o["id"]][0] + 0.5, (w, o["id"])
    same_queue_overlaps = 0
    by_stream = {}
    for o in exp["ops"]:
        if o["type"] == "kernel":
            by_stream.setdefault(o["stream"], []).append(t[o["id"]])
    for iv in by_stream.values():
        iv.sort()
        same_queue_overlaps += sum(1 for a, b in zip(iv, iv[1:]) if b[0] < a[1])
    print(f"out-of-order, {n_streams} queue(s): {same_queue_overlaps} overlapping kernel pairs within a queue",
          flush=True)
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs
    ref, _ = psc.run_spec(spec, inp, "fine", n_streams=n_streams, mapper="component", **AQL)
    np.testing.assert_array_equal(got, ref["Y2"])
