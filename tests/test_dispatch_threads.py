"""Host-only tests of the multi-threaded enqueue (psc_run's dispatch threads) against a recording
backend: every op issued once, stream order kept, and every wait issued after the awaited op's
event record -- under random delays, for several thread counts and schedules."""
import pytest

import workloads
import paper_2009_07482_amd as psc


def _check_trace(exp, trace):
    ops = exp["ops"]
    seq_exec, seq_rec = {}, {}
    for i, (kind, op, arg) in enumerate(trace):
        if kind == 1:
            assert op not in seq_exec
            seq_exec[op] = i
        elif kind == 2:
            assert op not in seq_rec
            seq_rec[op] = i
    assert sorted(seq_exec) == [o["id"] for o in ops]
    for o in ops:
        if any(o["id"] in x["waits"] for x in ops):
            assert o["id"] in seq_rec and seq_rec[o["id"]] > seq_exec[o["id"]]
    waits_seen = {}
    for i, (kind, op, arg) in enumerate(trace):
        if kind == 0:
            assert seq_rec[arg] < i, "wait issued before the awaited event was recorded"
            assert i < seq_exec[op]
            waits_seen.setdefault(op, []).append(arg)
    for o in ops:
        assert sorted(waits_seen.get(o["id"], [])) == sorted(o["waits"])
    by_stream = {}
    for o in ops:
        by_stream.setdefault(o["stream"], []).append(o)
    for s, lst in by_stream.items():
        lst.sort(key=lambda o: o["pos"])
        assert all(seq_exec[a["id"]] < seq_exec[b["id"]] for a, b in zip(lst, lst[1:]))
    done = sorted(arg for kind, op, arg in trace if kind == 3)
    assert done == list(range(exp["n_streams"]))


@pytest.mark.parametrize("spec", [workloads.mha_spec(16, 16, 4), workloads.forkjoin_spec(8),
                                  workloads.random_dag_spec(5, n_nodes=(40, 60), dim=(8, 32))])
@pytest.mark.parametrize("kw", [dict(n_streams=4, mapper="rr"), dict(n_streams=3, mapper="eft", copy_stream=True),
                                dict(n_streams=8, mapper="component")])
@pytest.mark.parametrize("threads", [0, 1, 2, 3])
def test_threaded_enqueue_orders_waits_after_records(spec, kw, threads):
    dag = psc.build_dag(spec)
    s = psc.psc_schedule(dag, "fine", **kw)
    try:
        exp = psc.export_schedule(spec, s)
        for seed in range(3):
            trace = psc.psc_sched_dispatch_trace(s, host_threads=threads, jitter_us=30, seed=seed)
            _check_trace(exp, trace)
    finally:
        psc.psc_sched_destroy(s)
        psc.psc_dag_destroy(dag)


def test_threaded_enqueue_repeated_runs_without_jitter():
    spec = workloads.mha_spec(32, 32, 8, layers=2)
    dag = psc.build_dag(spec)
    s = psc.psc_schedule(dag, "fine", n_streams=4)
    exp = psc.export_schedule(spec, s)
    for _ in range(50):
        _check_trace(exp, psc.psc_sched_dispatch_trace(s))
    psc.psc_sched_destroy(s)
    psc.psc_dag_destroy(dag)
