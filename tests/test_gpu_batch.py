"""GPU tests of batched inference: many attention instances of uneven length in one DAG (one task
component per instance) run eagerly over streams or as one hipGraph, with per-instance completion
times from device-clock marks."""
import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from gpu_helpers import normwise, oracle_outputs

pytestmark = pytest.mark.gpu

LENGTHS = [1, 5, 64, 137, 33, 200, 96, 250]


def _instance(lengths, i, d, heads, layers, dt, inp):
    sub = workloads.mha_spec(lengths[i], d, heads, layers, dt, prefix=f"i{i}_", weight_prefix="")
    return sub, {k: inp[k] for k in workloads.host_inputs_of(sub)}


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("kw", [dict(n_streams=4, mapper="component"),
                                dict(n_streams=4, mapper="component", use_graph=True),
                                dict(n_streams=3, mapper="rr", use_graph=True, mark_components=True)],
                         ids=["eager", "graph", "graph-marked"])
def test_small_batch_against_oracle(dt, kw):
    d, heads, layers = 64, 2, 2
    print(f"batch {LENGTHS} d={d} {dt} {kw}", flush=True)
    spec = workloads.batch_spec(LENGTHS, d, heads, layers, gemm_dtype=dt)
    inp = workloads.batch_inputs(0, LENGTHS, d, layers)
    out, _ = psc.run_spec(spec, inp, "fine", **kw)
    ref = oracle_outputs(spec, inp)
    tol = 1e-4 if dt == "f32" else 2e-2
    assert len(ref) == len(LENGTHS)
    for name, want in ref.items():
        assert normwise(out[name], want) < tol, name


@pytest.mark.parametrize("policy,kw", [("fine", dict(n_streams=4, mapper="component", mark_components=True)),
                                       ("fine", dict(n_streams=8, mapper="component", use_graph=True,
                                                     mark_components=True)),
                                       ("coarse", dict(mark_components=True)),
                                       ("device", {})], ids=["eager", "graph", "coarse", "device"])
def test_component_completion_times(policy, kw):
    spec = workloads.batch_spec(LENGTHS, 64, 2, 2)
    inp = workloads.batch_inputs(0, LENGTHS, 64, 2)
    r = psc.SpecRunner(spec, policy, **kw)
    r.set_inputs(inp)
    st = None
    for _ in range(3):   # graph replays and eager reruns keep reporting consistent marks
        st = r.run(with_inputs=False, with_outputs=False)
        done = psc.psc_sched_component_times(r.sched)
        assert done.shape == (len(LENGTHS),)
        assert np.all(done > 0), done
        assert done.max() <= st["makespan_ms"] * 1000 + 100, (done.max(), st["makespan_ms"])
    if policy == "coarse":
        # one stream runs the instances in breadth-first order, so they finish in component order
        # only loosely; every instance still ends before the batch does
        assert done.max() == pytest.approx(st["makespan_ms"] * 1000, rel=0.5)
    r.close()


def test_component_times_need_a_marked_run():
    spec = workloads.batch_spec([4, 8], 16, 1, 1)
    r = psc.SpecRunner(spec, "fine", n_streams=2)
    r.run(with_inputs=False, with_outputs=False)
    with pytest.raises(psc.PscError) as e:
        psc.psc_sched_component_times(r.sched)
    assert e.value.name == "PSC_ERR_STATE"
    r.close()


def test_batch_graph_equals_eager_bit_identical():
    spec = workloads.batch_spec(LENGTHS, 64, 2, 2)
    inp = workloads.batch_inputs(1, LENGTHS, 64, 2)
    a, _ = psc.run_spec(spec, inp, "fine", n_streams=4, mapper="component")
    b, _ = psc.run_spec(spec, inp, "fine", n_streams=8, mapper="rr", use_graph=True, mark_components=True)
    c, _ = psc.run_spec(spec, inp, "coarse")
    for k in a:
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k


@pytest.mark.timeout(900)
def test_batch64_full_size_every_instance():
    """64 instances, n log-uniform in [64, 2048], d = 512, 8 heads, 6 layers, BF16 GEMMs, run as
    one graph: every instance's output against the FP64 oracle (normwise 2e-2)."""
    lengths = workloads.batch_lengths(0)
    d, heads, layers = 512, 8, 6
    spec = workloads.batch_spec(lengths, d, heads, layers, gemm_dtype="bf16")
    inp = workloads.batch_inputs(0, lengths, d, layers)
    print(f"batch64 kernels={len(spec['kernels'])} n in [{min(lengths)}, {max(lengths)}]", flush=True)
    r = psc.SpecRunner(spec, "fine", n_streams=8, mapper="component", use_graph=True, mark_components=True)
    r.set_inputs(inp)
    st = r.run()
    done = psc.psc_sched_component_times(r.sched)
    print(f"makespan with copies {st['makespan_ms']:.2f} ms; instance completion p50 "
          f"{np.percentile(done, 50) / 1000:.2f} ms p99 {np.percentile(done, 99) / 1000:.2f} ms", flush=True)
    assert np.all(done > 0)
    worst = 0.0
    for i in range(len(lengths)):
        sub, sub_inp = _instance(lengths, i, d, heads, layers, "bf16", inp)
        want = oracle_outputs(sub, sub_inp)
        for name, w in want.items():
            err = normwise(r.result(name), w)
            worst = max(worst, err)
            assert err < 2e-2, (i, lengths[i], err)
    print(f"worst instance error {worst:.2e} over {len(lengths)} instances", flush=True)
    r.close()


# --- psc_schedule_batch: separate DAGs, one schedule --------------------------------------------

@pytest.mark.parametrize("policy,kw", [("fine", dict(n_streams=4, mapper="component", mark_components=True)),
                                       ("fine", dict(n_streams=3, mapper="eft", use_graph=True)),
                                       ("fine", dict(n_streams=1)), ("device", {})],
                         ids=["eager", "graph-eft", "one-stream", "device"])
def test_schedule_batch_equals_separate_runs(policy, kw):
    """Eight attention DAGs of uneven length, each with its own inputs, scheduled as one batch:
    every output within the FP32 bar of the oracle, and bit-identical to the DAG run alone on
    streams (the device executor picks its own GEMM tiles, so its sums may round differently)."""
    d, heads, layers = 64, 2, 2
    specs = [workloads.mha_spec(n, d, heads, layers) for n in LENGTHS]
    inps = [workloads.mha_inputs(10 + i, n, d, layers) for i, n in enumerate(LENGTHS)]
    print(f"schedule_batch {LENGTHS} {policy} {kw}", flush=True)
    r = psc.BatchRunner(specs, policy, **kw)
    try:
        r.set_inputs({f"{i}/{k}": v for i, inp in enumerate(inps) for k, v in inp.items()})
        r.run()
        for i, (sp, inp) in enumerate(zip(specs, inps)):
            alone, _ = psc.run_spec(sp, inp, "coarse")
            want = oracle_outputs(sp, inp)
            for name in workloads.host_outputs_of(sp):
                got = r.result(f"{i}/{name}")
                if policy != "device":
                    assert np.array_equal(got, alone[name]), (i, name)
                assert normwise(got, want[name]) < 1e-4, (i, name)
        if kw.get("mark_components"):
            done = psc.psc_sched_component_times(r.sched)
            assert done.shape == (max(r.spec["component"]) + 1,)   # heads and joins of every DAG
            assert np.all(done > 0)
    finally:
        r.close()


# --- failure paths forced from the host ----------------------------------------------------------

@pytest.mark.parametrize("use_graph", [False, True])
def test_fault_injection_runs_the_prefix_and_reports(use_graph):
    spec = workloads.mha_spec(64, 64, 2, 1)
    inp = workloads.mha_inputs(3, 64, 64, 1)
    d = psc.build_dag(spec)
    s0 = psc.psc_schedule(d, "fine", n_streams=3)
    n_ops = len(psc.psc_sched_export(s0))
    psc.psc_sched_destroy(s0)
    psc.psc_dag_destroy(d)
    for k in (1, n_ops // 2, n_ops):
        print(f"fault at op {k - 1} of {n_ops} graph={use_graph}", flush=True)
        r = psc.SpecRunner(spec, "fine", n_streams=3, use_graph=use_graph, fault_inject_op=k)
        try:
            r.set_inputs(inp)
            for _ in range(2):      # the schedule stays usable and fails the same way
                with pytest.raises(psc.PscError) as e:
                    r.run()
                assert e.value.name == "PSC_ERR_HIP" and f"injected fault: op {k - 1} " in str(e.value)
        finally:
            r.close()
    # the same DAG without the fault: correct results
    out, _ = psc.run_spec(spec, inp, "fine", n_streams=3)
    want = oracle_outputs(spec, inp)
    for name, w in want.items():
        assert normwise(out[name], w) < 1e-4


def _gemm_chain(n, length):
    bufs = [{"name": "A", "dtype": "f32", "rows": n, "cols": n, "view_of": None, "row_off": 0, "col_off": 0},
            {"name": "B", "dtype": "f32", "rows": n, "cols": n, "view_of": None, "row_off": 0, "col_off": 0}]
    bufs += [{"name": f"C{i}", "dtype": "f32", "rows": n, "cols": n, "view_of": None, "row_off": 0, "col_off": 0}
             for i in range(length)]
    kers = [{"name": f"g{i}", "kind": "gemm", "inputs": ["A" if i == 0 else f"C{i - 1}", "B"],
             "outputs": [f"C{i}"], "alpha": 1.0, "tile": 1} for i in range(length)]
    edges = [(i - 1, f"C{i - 1}", i, f"C{i - 1}") for i in range(1, length)]
    return {"buffers": bufs, "kernels": kers, "edges": edges, "component": [0] * length}


def test_timeout_returns_and_later_calls_drain_the_run():
    """Eight dependent 4096^3 FP32 GEMMs (~10 ms) under a 1 ms limit: psc_run returns
    PSC_ERR_TIMEOUT while the GEMMs still run; the next run waits for them first; destroying the
    schedule waits too.  Operands stay on the device (no copies)."""
    spec = _gemm_chain(4096, 8)
    r = psc.SpecRunner(spec, "fine", n_streams=2, timeout_ms=1)
    try:
        for _ in range(2):
            with pytest.raises(psc.PscError) as e:
                r.run(with_inputs=False, with_outputs=False)
            assert e.value.name == "PSC_ERR_TIMEOUT"
    finally:
        r.close()
    # a generous limit: the same chain completes, on small ternary operands exactly
    spec = _gemm_chain(256, 3)
    g = np.random.default_rng(4)
    inp = {"A": g.integers(-1, 2, (256, 256)).astype(np.float32),
           "B": (np.eye(256) * g.choice([-1.0, 1.0], 256)).astype(np.float32)}
    out, _ = psc.run_spec(spec, inp, "fine", n_streams=2, timeout_ms=60000)
    np.testing.assert_array_equal(out["C2"], oracle_outputs(spec, inp)["C2"])
