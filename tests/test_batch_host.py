"""Host-side tests of psc_schedule_batch (the disjoint union of several DAGs planned as one
schedule) and of the failure-path options (fault_inject_op, timeout_ms): planning, validity and
argument errors.  No GPU is touched: psc_schedule plans on the host."""
import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import validator


def _err(fn):
    with pytest.raises(psc.PscError) as e:
        fn()
    return e.value


def _batch(specs, policy="fine", **kw):
    dags = [psc.build_dag(sp) for sp in specs]
    try:
        return psc.psc_schedule_batch(dags, policy, **kw), dags
    except Exception:
        for d in dags:
            psc.psc_dag_destroy(d)
        raise


SPECS = [workloads.mha_spec(n, 32, 2, 2) for n in (4, 9, 16)] + [workloads.forkjoin_spec(8)]


@pytest.mark.parametrize("policy,kw", [("coarse", {}), ("fine", dict(n_streams=3, mapper="rr")),
                                       ("fine", dict(n_streams=4, mapper="component")),
                                       ("fine", dict(n_streams=2, mapper="eft", copy_stream=True))])
def test_batch_schedule_is_valid_and_covers_every_dag(policy, kw):
    s, dags = _batch(SPECS, policy, **kw)
    try:
        u = psc.union_spec(SPECS)
        exp = psc.export_schedule(u, s)
        ok, errs, _ = validator.check_schedule(u, exp)
        assert ok, errs[:5]
        kernels = [o["kernel"] for o in exp["ops"] if o["type"] == "kernel"]
        assert sorted(kernels) == list(range(len(u["kernels"])))
        # each DAG's isolated reads are copied back exactly once, under its prefix
        h2d = [o["buffer"] for o in exp["ops"] if o["type"] == "h2d"]
        d2h = [o["buffer"] for o in exp["ops"] if o["type"] == "d2h"]
        assert len(set(d2h)) == len(d2h)
        for i, sp in enumerate(SPECS):
            assert {b for b in d2h if b.startswith(f"{i}/")} == {f"{i}/{n}" for n in workloads.host_outputs_of(sp)}
            assert any(b.startswith(f"{i}/") for b in h2d)
    finally:
        psc.psc_sched_destroy(s)
        for d in dags:
            psc.psc_dag_destroy(d)


def test_batch_matches_union_spec_and_leaves_sources_open():
    s, dags = _batch(SPECS[:2], "fine", n_streams=2)
    # the sources are neither frozen nor referenced: they can grow and be destroyed at once
    psc.psc_add_buffer(dags[0], "extra", "f32", 2, 2)
    for d in dags:
        psc.psc_dag_destroy(d)
    u = psc.union_spec(SPECS[:2])
    exp = psc.export_schedule(u, s)      # ids follow the union's order
    assert validator.check_schedule(u, exp)[0]
    psc.psc_sched_destroy(s)
    # per-DAG components are offset: mha_spec puts each head in a component of its own
    comp = u["component"]
    n0 = len(SPECS[0]["kernels"])
    assert min(comp[n0:]) == max(comp[:n0]) + 1


def test_batch_of_one_equals_plain_schedule():
    sp = SPECS[0]
    s1, dags = _batch([sp], "fine", n_streams=3, mapper="rr")
    d = psc.build_dag(sp)
    s2 = psc.psc_schedule(d, "fine", n_streams=3, mapper="rr")
    a, b = psc.psc_sched_export(s1), psc.psc_sched_export(s2)
    assert a == b
    for x in (s1, s2):
        psc.psc_sched_destroy(x)
    for x in dags + [d]:
        psc.psc_dag_destroy(x)


def test_batch_errors():
    assert _err(lambda: psc.psc_schedule_batch([], "fine")).name == "PSC_ERR_ARG"
    d = psc.build_dag(SPECS[3])
    assert _err(lambda: psc.psc_schedule_batch([d, None], "fine")).name == "PSC_ERR_ARG"
    # a race inside DAG 1 is reported with that DAG's prefix
    bad = dict(SPECS[3], edges=[e for e in SPECS[3]["edges"] if e != (0, "C0", 2, "C0")])
    b = psc.build_dag(bad)
    e = _err(lambda: psc.psc_schedule_batch([d, b], "fine"))
    assert e.name == "PSC_ERR_RACE" and "1/" in str(e)
    for x in (d, b):
        psc.psc_dag_destroy(x)


def test_failure_option_errors():
    d = psc.build_dag(SPECS[3])
    s0 = psc.psc_schedule(d, "fine", n_streams=2)
    n_ops = len(psc.psc_sched_export(s0))
    psc.psc_sched_destroy(s0)
    assert _err(lambda: psc.psc_schedule(d, "fine", fault_inject_op=n_ops + 1)).name == "PSC_ERR_ARG"
    assert _err(lambda: psc.psc_schedule(d, "fine", fault_inject_op=-1)).name == "PSC_ERR_ARG"
    assert _err(lambda: psc.psc_schedule(d, "fine", timeout_ms=-5)).name == "PSC_ERR_ARG"
    assert _err(lambda: psc.psc_schedule(d, "device", fault_inject_op=1)).name == "PSC_ERR_ARG"
    s = psc.psc_schedule(d, "fine", n_streams=2, fault_inject_op=n_ops, timeout_ms=1000)  # the last op
    psc.psc_sched_destroy(s)
    psc.psc_dag_destroy(d)
