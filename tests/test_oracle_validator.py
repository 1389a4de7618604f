"""Pins of the schedule validator: the paper's Fig. 9 example, brute force agreement, mutations."""
import copy
import itertools
import json
import os

import pytest

import workloads
from oracle import validator
from schedule_helpers import naive_schedule, from_queues


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def test_fig9_queue_structure_is_valid(golden_dir):
    g = _load(golden_dir, "fig9_setup_cq.json")
    spec = g["dag"]
    sched, ids = from_queues(spec, g["queues"], g["eq_stated"] + g["eq_derived"])
    ok, errs, bad = validator.check_schedule(spec, sched)
    assert ok, errs
    assert validator.brute_force(spec, sched) == set()
    # e2 and e3 (k1, k2) are unordered: they may run in parallel
    anc = validator.hb_closure(sched)
    a, b = ids["kernel:k1"], ids["kernel:k2"]
    assert not (anc[a] >> b) & 1 and not (anc[b] >> a) & 1


def test_fig9_without_derived_precedences_is_invalid(golden_dir):
    # rule (iii) of Sec. III: the derived pairs <e2,e4>, <e3,e5> are required
    g = _load(golden_dir, "fig9_setup_cq.json")
    spec = g["dag"]
    sched, ids = from_queues(spec, g["queues"], g["eq_stated"])
    ok, errs, bad = validator.check_schedule(spec, sched)
    assert not ok
    assert bad == validator.brute_force(spec, sched) == {ids["kernel:k3"], ids["kernel:k4"]}


def _all_assignments(n_kernels, n_streams):
    return itertools.product(range(n_streams), repeat=n_kernels)


@pytest.mark.parametrize("n_streams", [1, 2, 3])
def test_every_stream_assignment_and_every_wait_deletion_agree(n_streams):
    spec = workloads.forkjoin_spec(4)
    checked = 0
    for assign in _all_assignments(4, n_streams):
        for order in ([0, 1, 2, 3], [0, 2, 1, 3]):
            sched = naive_schedule(spec, list(assign), n_streams, order)
            ok, errs, bad = validator.check_schedule(spec, sched)
            assert ok, errs
            assert validator.brute_force(spec, sched) == set()
            for o in sched["ops"]:
                for w in o["waits"]:
                    mut = copy.deepcopy(sched)
                    mut["ops"][o["id"]]["waits"].remove(w)
                    ok2, _, bad2 = validator.check_schedule(spec, mut)
                    bf = validator.brute_force(spec, mut)
                    assert bad2 == bf
                    assert ok2 == (not bf)
                    checked += 1
    if n_streams > 1:
        assert checked > 0


def test_two_head_attention_assignments_agree():
    spec = workloads.mha_spec(4, 4, 1)      # 8 kernels, 1 head
    import random
    r = random.Random(0)
    for _ in range(30):
        assign = [r.randrange(3) for _ in spec["kernels"]]
        sched = naive_schedule(spec, assign, 3)
        ok, errs, bad = validator.check_schedule(spec, sched)
        assert ok, errs
        waits = [(o["id"], w) for o in sched["ops"] for w in o["waits"]]
        if waits:
            oid, w = waits[r.randrange(len(waits))]
            mut = copy.deepcopy(sched)
            mut["ops"][oid]["waits"].remove(w)
            ok2, _, bad2 = validator.check_schedule(spec, mut)
            assert bad2 == validator.brute_force(spec, mut, limit=50000)


def test_structural_errors_are_reported():
    spec = workloads.forkjoin_spec(4)
    sched = naive_schedule(spec, [0, 1, 0, 0], 2)
    mut = copy.deepcopy(sched)
    # make a wait refer to an op the host enqueues later
    k1 = next(o for o in mut["ops"] if o["type"] == "kernel" and o["kernel"] == 1)
    k3 = next(o for o in mut["ops"] if o["type"] == "kernel" and o["kernel"] == 3)
    k1["waits"].append(k3["id"])
    ok, errs, _ = validator.check_schedule(spec, mut)
    assert not ok and any("enqueued later" in e for e in errs)
    # drop a kernel
    mut = copy.deepcopy(sched)
    mut["ops"] = [o for o in mut["ops"] if not (o["type"] == "kernel" and o["kernel"] == 2)]
    for i, o in enumerate(mut["ops"]):
        pass
    ok, errs, _ = validator.check_schedule(spec, mut)
    assert not ok


def test_missing_h2d_and_double_d2h_are_reported():
    spec = workloads.forkjoin_spec(4)
    sched = naive_schedule(spec, [0, 0, 0, 0], 1)
    ops = sched["ops"]
    d2h = next(o for o in ops if o["type"] == "d2h")
    extra = dict(d2h, id=len(ops), pos=max(o["pos"] for o in ops) + 1, host_order=len(ops),
                 waits=[])
    ok, errs, _ = validator.check_schedule(spec, {"n_streams": 1, "ops": ops + [extra]})
    assert not ok and any("D2H" in e for e in errs)


def test_coarse_single_stream_schedule_needs_no_waits():
    spec = workloads.mha_spec(8, 8, 2)
    sched = naive_schedule(spec, [0] * len(spec["kernels"]), 1)
    assert all(not o["waits"] for o in sched["ops"])
    ok, errs, _ = validator.check_schedule(spec, sched)
    assert ok, errs


def _with_every_direct_wait(spec, sched):
    """The same ops, each waiting for every op it reads from (same stream included)."""
    out = copy.deepcopy(sched)
    ops = out["ops"]
    kop = {o["kernel"]: o["id"] for o in ops if o["type"] == "kernel"}
    h2d = {o["buffer"]: o["id"] for o in ops if o["type"] == "h2d"}
    writes, _ = validator.isolated_io(spec)
    producer = {}
    for (src, sb, _, _) in spec["edges"]:
        producer[sb] = src
    for k in spec["kernels"]:
        for b in k["outputs"]:
            producer.setdefault(b, spec["kernels"].index(k))
    for o in ops:
        if o["type"] == "kernel":
            k = o["kernel"]
            w = [kop[src] for (src, _, dst, _) in spec["edges"] if dst == k]
            w += [h2d[validator._region(spec, b)[0]] for (ki, b) in writes if ki == k]
        elif o["type"] == "d2h":
            w = [kop[producer[o["buffer"]]]]
        else:
            w = []
        o["waits"] = sorted(set(w))
    return out


@pytest.mark.parametrize("n_streams", [1, 2])
def test_out_of_order_queues_need_every_precedence_as_a_wait(n_streams):
    """Out-of-order queues (OpenCL's out-of-order execution mode): a queue position orders
    nothing, so the in-order schedules that lean on stream order become invalid, and adding every
    direct precedence as a wait makes them valid again; brute force agrees every time."""
    spec = workloads.forkjoin_spec(4)
    assigns = list(_all_assignments(4, n_streams))
    if n_streams > 1:
        assigns = [(0, 0, 1, 0), (0, 1, 0, 1), (1, 0, 1, 1)]   # a kernel on each side of every edge
    for assign in assigns:
        sched = naive_schedule(spec, list(assign), n_streams)
        ooo = dict(copy.deepcopy(sched), in_order=False)
        ok, _, bad = validator.check_schedule(spec, ooo)
        assert not ok and bad == validator.brute_force(spec, ooo) != set()
        full = dict(_with_every_direct_wait(spec, sched), in_order=False)
        ok, errs, bad = validator.check_schedule(spec, full)
        assert ok, errs
        assert validator.brute_force(spec, full) == set()
        # and then dropping any one wait breaks it
        for o in full["ops"]:
            for w in o["waits"]:
                mut = copy.deepcopy(full)
                mut["ops"][o["id"]]["waits"].remove(w)
                ok2, _, bad2 = validator.check_schedule(spec, mut)
                assert not ok2 and bad2 == validator.brute_force(spec, mut)
