"""Host-side tests of the C ABI (no GPU): symbol export, IR errors, classification, and the
command-queue structures the schedulers build, checked by the oracle's validator."""
import json
import os
import re

import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import validator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "psc.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^\S.*?\b(psc_\w+)\(", hdr, flags=re.M))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(psc._lib, name), name
    assert declared <= set(psc.EXPORTED)
    assert psc.psc_abi_version() == 1


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def test_fig6_classification(golden_dir):
    g = _load(golden_dir, "fig6_classification.json")
    spec = g["dag"]
    dag = psc.build_dag(spec)
    try:
        kclass, inter = psc.psc_dag_classify(dag, g["component"])
    finally:
        psc.psc_dag_destroy(dag)
    names = [k["name"] for k in spec["kernels"]]
    front = sorted(n for n, c in zip(names, kclass) if c & psc.PSC_FRONT)
    end = sorted(n for n, c in zip(names, kclass) if c & psc.PSC_END)
    inn = sorted(n for n, c in zip(names, kclass) if c & psc.PSC_IN)
    assert front == g["front"] and end == g["end"] and inn == g["in"]
    pairs = [(e[1], e[3]) for e in spec["edges"]]
    got_inter = sorted(list(p) for p, x in zip(pairs, inter) if x)
    got_intra = sorted(list(p) for p, x in zip(pairs, inter) if not x)
    assert got_inter == sorted(g["inter_edges"])
    assert got_intra == sorted(g["intra_edges"])
    # isolated writes of T: inputs of T's kernels that no edge feeds
    writes, _ = validator.isolated_io(spec)
    tk = {i for i, c in enumerate(spec["component"]) if c == g["component"]}
    iso_t = sorted([b, names[k]] for (k, b) in writes if k in tk)
    assert iso_t == sorted(g["isolated_writes_in_T"])


def _queues(exp):
    qs = {}
    for o in sorted(exp["ops"], key=lambda o: (o["stream"], o["pos"])):
        qs.setdefault(o["stream"], []).append(o)
    return [qs[s] for s in sorted(qs)]


def _label(spec, o):
    if o["type"] == "kernel":
        return "kernel:" + spec["kernels"][o["kernel"]]["name"]
    return f"{o['type']}:{o['buffer']}"


def test_fig9_setup_cq_round_robin(golden_dir):
    g = _load(golden_dir, "fig9_setup_cq.json")
    spec = g["dag"]
    dag = psc.build_dag(spec)
    s = psc.psc_schedule(dag, "fine", n_streams=g["n_streams"], mapper="rr")
    try:
        exp = psc.export_schedule(spec, s)
    finally:
        psc.psc_sched_destroy(s)
        psc.psc_dag_destroy(dag)
    assert [[_label(spec, o) for o in q] for q in _queues(exp)] == g["queues"]
    by_id = {o["id"]: o for o in exp["ops"]}
    eq = sorted([_label(spec, by_id[w]), _label(spec, o)] for o in exp["ops"] for w in o["waits"])
    assert eq == sorted(g["eq_stated"] + g["eq_derived"])
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs
    assert validator.brute_force(spec, exp) == set()


def _schedules(spec, configs):
    dag = psc.build_dag(spec)
    out = []
    try:
        for policy, kw in configs:
            s = psc.psc_schedule(dag, policy, **kw)
            out.append(((policy, tuple(sorted(kw.items()))), psc.export_schedule(spec, s)))
            psc.psc_sched_destroy(s)
    finally:
        psc.psc_dag_destroy(dag)
    return out


CONFIGS = [("coarse", {}), ("device", {})] + [
    ("fine", dict(n_streams=s, mapper=m, copy_stream=c))
    for s in (1, 2, 3, 4, 8) for m in ("rr", "eft", "component") for c in (False, True)] + [
    ("fine", dict(n_streams=s, mapper=m, copy_stream=c, dispatch="aql", out_of_order=True))
    for s in (1, 2, 4) for m in ("rr", "eft", "component") for c in (False, True)] + [
    ("coarse", dict(copy_roots=True)), ("device", dict(copy_roots=True)),
    ("fine", dict(n_streams=4, mapper="component", copy_stream=True, copy_roots=True)),
    ("fine", dict(n_streams=2, mapper="rr", dispatch="aql", out_of_order=True, copy_roots=True))]


@pytest.mark.parametrize("name,spec", [
    ("forkjoin", workloads.forkjoin_spec(64)),
    ("mha1", workloads.mha_spec(64, 64, 4)),
    ("mha2x", workloads.mha_spec(32, 32, 2, layers=2)),
    ("mha_bf16", workloads.mha_spec(64, 64, 2, gemm_dtype="bf16")),
    ("random", workloads.random_dag_spec(3, n_nodes=(20, 40), dim=(8, 64))),
    ("batch", workloads.batch_spec([5, 17, 9], d=16, heads=2, layers=2)),
])
def test_every_schedule_is_valid(name, spec):
    for key, exp in _schedules(spec, CONFIGS):
        ok, errs, _ = validator.check_schedule(spec, exp)
        assert ok, (key, errs[:5])
        if key[0] == "coarse":
            assert exp["n_streams"] == 1 and all(not o["waits"] for o in exp["ops"])
        if key[0] == "device":
            kern = [o for o in exp["ops"] if o["type"] == "kernel"]
            assert all(o["pos"] == 0 for o in kern) and len({o["stream"] for o in kern}) == len(kern)


def test_tiny_schedules_agree_with_brute_force():
    spec = workloads.forkjoin_spec(8)
    for key, exp in _schedules(spec, CONFIGS):
        assert validator.brute_force(spec, exp) == set(), key


def test_schedules_are_deterministic():
    spec = workloads.mha_spec(32, 32, 4)
    a = _schedules(spec, CONFIGS)
    b = _schedules(spec, CONFIGS)
    assert a == b


def test_fine_round_robin_spreads_heads_and_reduces_waits():
    spec = workloads.mha_spec(512, 512, 8)
    (_, exp), = _schedules(spec, [("fine", dict(n_streams=4, mapper="rr"))])
    kern = [o for o in exp["ops"] if o["type"] == "kernel"]
    assert sorted({o["stream"] for o in kern}) == [0, 1, 2, 3]
    assert len(kern) == 57
    assert sum(1 for o in exp["ops"] if o["type"] == "h2d") == 1 + 3 * 8 + 1   # X, 24 slices, Wo
    assert sum(1 for o in exp["ops"] if o["type"] == "d2h") == 1
    # every wait is needed: no wait is implied by the stream order plus the other waits
    anc = validator.hb_closure(exp)
    for o in exp["ops"]:
        for w in o["waits"]:
            others = [x for x in o["waits"] if x != w]
            prev = [p["id"] for p in exp["ops"] if p["stream"] == o["stream"] and p["pos"] == o["pos"] - 1]
            implied = any((anc[x] >> w) & 1 or x == w for x in others + prev)
            assert not implied


def _err(fn):
    with pytest.raises(psc.PscError) as e:
        fn()
    return e.value.name


def _dag_from(spec):
    return psc.build_dag(spec)


def test_ir_errors():
    # cycle
    spec = workloads.forkjoin_spec(4)
    d = psc.psc_dag_create()
    for b in spec["buffers"]:
        psc.psc_add_buffer(d, b["name"], "f32", 4, 4)
    k0 = psc.psc_add_kernel(d, "a", "add", ["A0", "B0"], ["C0"])
    k1 = psc.psc_add_kernel(d, "b", "add", ["C0", "B1"], ["A0"])
    psc.psc_add_edge(d, k0, "C0", k1, "C0")
    psc.psc_add_edge(d, k1, "A0", k0, "A0")
    assert _err(lambda: psc.psc_schedule(d, "coarse")) == "PSC_ERR_CYCLE"
    psc.psc_dag_destroy(d)
    # unknown name, duplicate, wrong arity, bad view
    d = psc.psc_dag_create()
    psc.psc_add_buffer(d, "A", "f32", 4, 8)
    assert _err(lambda: psc.psc_add_buffer(d, "A", "f32", 4, 8)) == "PSC_ERR_NAME"
    assert _err(lambda: psc.psc_add_kernel(d, "k", "transpose", ["nope"], ["A"])) == "PSC_ERR_NAME"
    assert _err(lambda: psc.psc_add_kernel(d, "k", "gemm", ["A"], ["A"])) == "PSC_ERR_ARG"
    assert _err(lambda: psc.psc_add_buffer(d, "V", "f32", 4, 4, "A", 0, 5)) == "PSC_ERR_SHAPE"
    assert _err(lambda: psc.psc_add_buffer(d, "V", "bf16", 4, 4, "A", 0, 0)) == "PSC_ERR_SHAPE"
    psc.psc_dag_destroy(d)
    # shape mismatch in a GEMM
    d = psc.psc_dag_create()
    for n, r, c in (("A", 4, 5), ("B", 6, 3), ("C", 4, 3)):
        psc.psc_add_buffer(d, n, "f32", r, c)
    psc.psc_add_kernel(d, "g", "gemm", ["A", "B"], ["C"])
    assert _err(lambda: psc.psc_schedule(d, "fine")) == "PSC_ERR_SHAPE"
    psc.psc_dag_destroy(d)


def test_race_and_state_errors():
    # an input produced by a kernel but with no edge feeding it
    spec = workloads.forkjoin_spec(4)
    bad = dict(spec, edges=[e for e in spec["edges"] if e != (0, "C0", 2, "C0")])
    d = _dag_from(bad)
    assert _err(lambda: psc.psc_schedule(d, "fine")) == "PSC_ERR_RACE"
    psc.psc_dag_destroy(d)
    # two unordered writers of one buffer
    d = psc.psc_dag_create()
    for n in ("A", "B", "C"):
        psc.psc_add_buffer(d, n, "f32", 4, 4)
    psc.psc_add_kernel(d, "t1", "transpose", ["A"], ["C"])
    psc.psc_add_kernel(d, "t2", "transpose", ["B"], ["C"])
    assert _err(lambda: psc.psc_schedule(d, "fine")) == "PSC_ERR_RACE"
    psc.psc_dag_destroy(d)
    # in-place kernel
    d = psc.psc_dag_create()
    psc.psc_add_buffer(d, "A", "f32", 4, 4)
    psc.psc_add_buffer(d, "B", "f32", 4, 4)
    psc.psc_add_kernel(d, "s", "add", ["A", "B"], ["A"])
    assert _err(lambda: psc.psc_schedule(d, "fine")) == "PSC_ERR_SHAPE"
    psc.psc_dag_destroy(d)
    # partly produced input: only one head writes into Ocat
    spec = workloads.mha_spec(8, 8, 2)
    bad = dict(spec, edges=[e for e in spec["edges"] if not (e[1] == "L0H1_O")])
    d = _dag_from(bad)
    assert _err(lambda: psc.psc_schedule(d, "fine")) in ("PSC_ERR_RACE", "PSC_ERR_SHAPE")
    psc.psc_dag_destroy(d)
    # frozen after scheduling; DAG outlives schedules
    d = _dag_from(workloads.forkjoin_spec(4))
    s = psc.psc_schedule(d, "coarse")
    assert _err(lambda: psc.psc_add_buffer(d, "Z", "f32", 1, 1)) == "PSC_ERR_STATE"
    assert _err(lambda: psc.psc_dag_destroy(d)) == "PSC_ERR_STATE"
    psc.psc_sched_destroy(s)
    psc.psc_dag_destroy(d)
    # edge between buffers that share no storage
    d = _dag_from(dict(workloads.forkjoin_spec(4), edges=[]))
    assert _err(lambda: psc.psc_add_edge(d, 0, "C0", 1, "B1")) == "PSC_ERR_SHAPE"
    assert _err(lambda: psc.psc_add_edge(d, 0, "A0", 1, "C0")) == "PSC_ERR_NAME"
    psc.psc_dag_destroy(d)
    assert psc.psc_last_error() == ""          # the last call succeeded


def test_classify_default_component_is_whole_dag():
    spec = workloads.mha_spec(16, 16, 2)
    spec = dict(spec, component=[0] * len(spec["kernels"]))
    d = _dag_from(spec)
    kc, inter = psc.psc_dag_classify(d, 0)
    psc.psc_dag_destroy(d)
    names = [k["name"] for k in spec["kernels"]]
    front = {n for n, c in zip(names, kc) if c & psc.PSC_FRONT}
    end = {n for n, c in zip(names, kc) if c & psc.PSC_END}
    assert front == {f"L0H{h}_{x}" for h in range(2) for x in "qkv"}
    assert end == {"L0_y"}
    assert not any(inter)


def test_tile_cache_roundtrip():
    n = psc.psc_gemm_tile_count()
    assert n == 22   # automatic (0) + 5 large + 7 LDS K-split + 3 direct K-split + 256x256 BF16 + 3 deep K-split
    #                  + 256x256 BF16 with direct copies, four and eight wavefronts
    psc.psc_tile_cache_clear()
    assert psc.psc_tile_cache_get(512, 64, 512, "f32", "f32") == 0
    psc.psc_tile_cache_set(512, 64, 512, "f32", "f32", 9)
    psc.psc_tile_cache_set(512, 64, 512, "bf16", "f32", 12)
    assert psc.psc_tile_cache_get(512, 64, 512, "f32", "f32") == 9
    assert psc.psc_tile_cache_get(512, 64, 512, "bf16", "f32") == 12
    psc.psc_tile_cache_set(512, 64, 512, "f32", "f32", 0)
    assert psc.psc_tile_cache_get(512, 64, 512, "f32", "f32") == 0
    assert psc.psc_tile_cache_clear() == 1
    with pytest.raises(psc.PscError):
        psc.psc_tile_cache_set(1, 1, 1, "f32", "f32", n)


def test_kernel_features_and_heuristic_cost():
    """Feature rows of the cost model and the roofline heuristic's closed form on them."""
    import math
    import numpy as np
    spec = workloads.mha_spec(512, 512, 8)
    dag = psc.build_dag(spec)
    with pytest.raises(psc.PscError) as e:
        psc.psc_kernel_features(dag, 0)
    assert e.value.name == "PSC_ERR_STATE"
    s = psc.psc_schedule(dag, "fine", n_streams=4, mapper="eft")
    names = [k["name"] for k in spec["kernels"]]
    q = psc.psc_kernel_features(dag, names.index("L0H0_q"), 2)
    assert q[:6].tolist() == [1, 0, 0, 0, 0, 0]
    assert q[6:9].tolist() == [9, 6, 9] and q[10] == 0 and q[11] == 2
    assert q[9] == pytest.approx(math.log2(4 * (512 * 512 + 512 * 64 + 512 * 64)))
    kt = psc.psc_kernel_features(dag, names.index("L0H0_kt"), 0)
    assert kt[:6].tolist() == [0, 1, 0, 0, 0, 0] and kt[6:9].tolist() == [6, 9, 0]
    p = psc.psc_kernel_features(dag, names.index("L0H0_p"), 0)
    assert p[:6].tolist() == [0, 0, 1, 0, 0, 0] and p[9] == pytest.approx(math.log2(2 * 4 * 512 * 512))
    # heuristic: 3 us + 2MNK / (90 TF/s * share of 256 CUs) for this GEMM, +15% per busy stream
    share = min(1.0, (512 / 64) * (64 / 64) / 256)
    t0 = 3.0 + max(2 * 512 * 64 * 512 / (9e13 * share), 2 ** q[9] / 4e12) * 1e6
    us = psc.psc_cost_predict(np.stack([q, q * np.r_[np.ones(11), 0]]))
    assert us[0] == pytest.approx(t0 * 1.3, rel=1e-5) and us[1] == pytest.approx(t0, rel=1e-5)
    cp = np.zeros(12, np.float32)
    cp[4], cp[6], cp[7], cp[9] = 1, 9, 9, math.log2(512 * 512 * 4)
    assert psc.psc_cost_predict(cp[None])[0] == pytest.approx(4.0 + 512 * 512 * 4 / 50e9 * 1e6, rel=1e-5)
    with pytest.raises(psc.PscError):
        psc.psc_sched_samples(s)          # no recorded run
    psc.psc_sched_destroy(s)
    psc.psc_dag_destroy(dag)


def test_eft_spreads_work_over_every_stream():
    spec = workloads.mha_spec(512, 512, 4)
    dag = psc.build_dag(spec)
    s = psc.psc_schedule(dag, "fine", n_streams=4, mapper="eft")
    exp = psc.export_schedule(spec, s)
    psc.psc_sched_destroy(s)
    psc.psc_dag_destroy(dag)
    names = [k["name"] for k in spec["kernels"]]
    stream_of = {names[o["kernel"]]: o["stream"] for o in exp["ops"] if o["type"] == "kernel"}
    assert set(stream_of.values()) == {0, 1, 2, 3}
    # the four heads' first projections start in parallel, one per stream
    assert len({stream_of[f"L0H{h}_k"] for h in range(4)}) == 4
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs


@pytest.mark.parametrize("name,spec,workers", [
    ("mha512", workloads.mha_spec(512, 512, 8), 256),
    ("mha_bf16_2x", workloads.mha_spec(200, 128, 4, layers=2, gemm_dtype="bf16"), 37),
    ("batch", workloads.batch_spec([5, 130, 64, 1], d=64, heads=2, layers=2), 256),
    ("random", workloads.random_dag_spec(5, n_nodes=(30, 60), dim=(8, 300)), 16),
    ("forkjoin", workloads.forkjoin_spec(256), 3),
])
def test_device_executor_plan_cannot_deadlock(name, spec, workers):
    """The PSC_DEVICE task lists: every tile of every node (the kernels, then the host copies the
    executor runs: the schedule's uploads and read-backs in op order) exactly once, published
    exactly once (signals of a node add up to its tile count, each at the end of a run of its
    tiles), and the wait-for relation -- list order within a workgroup plus 'a node's tasks wait
    for all tasks of its predecessors' (a kernel's: its predecessor kernels and its inputs'
    uploads; a read-back's: the kernel writing it) -- is acyclic, which with all workgroups
    resident means every wait ends.  Copy tasks sit on the last W / 16 (at most 32) workgroups,
    which run nothing else."""
    import numpy as np
    dag = psc.build_dag(spec)
    s = psc.psc_schedule(dag, "device")
    lists = psc.psc_sched_device_tasks(s, workers)
    ops = psc.psc_sched_export(s)
    psc.psc_sched_destroy(s)
    psc.psc_dag_destroy(dag)
    nk = len(spec["kernels"])
    copy_ops = [o for o in ops if o["type"] != "kernel"]
    node_of_op = {o["id"]: nk + i for i, o in enumerate(copy_ops)}
    node_of_op.update({o["id"]: o["kernel"] for o in ops if o["type"] == "kernel"})
    nn = nk + len(copy_ops)
    tiles = {}
    for w, L in enumerate(lists):
        for (k, t, _) in L:
            tiles.setdefault(k, []).append(t)
    copy_workers = {w for w, L in enumerate(lists) if any(k >= nk for (k, _, _) in L)}
    if workers >= 2:
        # copy tasks only on workgroups that run no kernel task, and at most 32 of them
        assert all(all(k >= nk for (k, _, _) in lists[w]) for w in copy_workers)
        assert len(copy_workers) <= 32
    assert sorted(tiles) == list(range(nn))
    ntiles = {k: len(v) for k, v in tiles.items()}
    for k, v in tiles.items():
        assert sorted(v) == list(range(len(v))), k
    signalled = {k: 0 for k in range(nn)}
    for L in lists:
        for i, (k, t, sig) in enumerate(L):
            last_of_run = i + 1 == len(L) or L[i + 1][0] != k
            assert (sig > 0) == last_of_run
            if sig:
                run = 1
                while i - run >= 0 and L[i - run][0] == k:
                    run += 1
                assert sig == run
                signalled[k] += sig
    assert signalled == ntiles
    # wait-for graph on kernel "stages": a task of kernel k at list position i waits for every task
    # of k's predecessors and for the task before it in its list.  Acyclic iff a topological order
    # of all tasks exists; check with Kahn's algorithm over tasks.
    preds = {k: set() for k in range(nn)}
    for (src, _, dst, _) in spec["edges"]:
        preds[dst].add(src)
    for o in ops:   # uploads before their readers, read-backs after their writers
        for w in o["waits"]:
            if o["type"] != "h2d":
                preds[node_of_op[o["id"]]].add(node_of_op[w])
    ids = {}
    for w, L in enumerate(lists):
        for i, (k, t, _) in enumerate(L):
            ids[(k, t)] = (w, i)
    indeg = {}
    succ = {}
    for w, L in enumerate(lists):
        for i, (k, t, _) in enumerate(L):
            deps = [(L[i - 1][0], L[i - 1][1])] if i else []
            for p in preds[k]:
                deps += [(p, tt) for tt in range(ntiles[p])]
            indeg[(k, t)] = len(deps)
            for d in deps:
                succ.setdefault(d, []).append((k, t))
    queue = [x for x, d in indeg.items() if d == 0]
    seen = 0
    while queue:
        x = queue.pop()
        seen += 1
        for y in succ.get(x, []):
            indeg[y] -= 1
            if indeg[y] == 0:
                queue.append(y)
    assert seen == len(indeg), "wait-for cycle"
    assert len([L for L in lists if L]) == min(workers, len(indeg))


def test_aql_code_object_covers_every_kernel():
    """Host-only: the code object beside libpsc.so and its argument table name every kernel the
    schedules of the workloads launch, with only implicit arguments the AQL dispatcher fills."""
    specs = [workloads.forkjoin_spec(256), workloads.mha_spec(512, 512, 8),
             workloads.mha_spec(1024, 1024, 16, 2, "bf16"), workloads.mha_spec(137, 64, 2, 2, "f32")]
    specs += [workloads.random_dag_spec(s) for s in range(4)]
    for spec in specs:
        d = psc.build_dag(spec)
        s = psc.psc_schedule(d, "fine", n_streams=4, dispatch="aql")
        n, why = psc.psc_sched_aql_check(s)
        assert n >= 2 and why == "", why
        psc.psc_sched_destroy(s)
        psc.psc_dag_destroy(d)


def test_dynamic_policies_validate_options_on_the_host():
    spec = workloads.forkjoin_spec(16)
    d = psc.build_dag(spec)
    for pol in ("eager", "heft"):
        s = psc.psc_schedule(d, pol, n_streams=2)
        with pytest.raises(psc.PscError) as e:
            psc.psc_sched_export(s)
        assert e.value.name == "PSC_ERR_STATE"
        assert psc.psc_sched_streams(s) == 2
        psc.psc_sched_destroy(s)
        for kw, want in ((dict(use_graph=True), "PSC_ERR_ARG"), (dict(timeout_ms=5), "PSC_ERR_UNSUPPORTED"),
                         (dict(dispatch="aql"), "PSC_ERR_UNSUPPORTED"), (dict(mark_components=True), "PSC_ERR_UNSUPPORTED")):
            with pytest.raises(psc.PscError) as e:
                psc.psc_schedule(d, pol, **kw)
            assert e.value.name == want, (pol, kw)
    psc.psc_dag_destroy(d)


def test_out_of_order_queues_issue_kernels_by_level_with_every_wait():
    """Out-of-order queues: each stream's kernels by DAG level, every direct precedence a wait
    (same stream included), and the export marked out of order and valid under that reading."""
    spec = workloads.mha_spec(64, 64, 4, layers=2)
    dag = psc.build_dag(spec)
    try:
        sched = psc.psc_schedule(dag, "fine", n_streams=2, mapper="component", dispatch="aql", out_of_order=True)
        exp = psc.export_schedule(spec, sched)
        psc.psc_sched_destroy(sched)
    finally:
        psc.psc_dag_destroy(dag)
    assert exp["in_order"] is False
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs[:5]
    # levels: longest path from a root
    n = len(spec["kernels"])
    pred = [set() for _ in range(n)]
    for (a, _, b, _) in spec["edges"]:
        pred[b].add(a)
    level = [None] * n
    def lv(k):
        if level[k] is None:
            level[k] = 1 + max((lv(p) for p in pred[k]), default=-1)
        return level[k]
    kops = sorted((o for o in exp["ops"] if o["type"] == "kernel"), key=lambda o: (o["stream"], o["pos"]))
    for a, b in zip(kops, kops[1:]):
        if a["stream"] == b["stream"]:
            assert lv(a["kernel"]) <= lv(b["kernel"])
    # every DAG edge is a wait of the consumer's op
    kop = {o["kernel"]: o["id"] for o in kops}
    for (a, _, b, _) in spec["edges"]:
        assert kop[a] in exp["ops"][kop[b]]["waits"]
    # one stream: all 12 projections of layer 0 come first, before any transpose
    dag = psc.build_dag(spec)
    try:
        sched = psc.psc_schedule(dag, "fine", n_streams=1, mapper="rr", dispatch="aql", out_of_order=True)
        one = psc.export_schedule(spec, sched)
        psc.psc_sched_destroy(sched)
    finally:
        psc.psc_dag_destroy(dag)
    first = [spec["kernels"][o["kernel"]]["name"] for o in sorted(one["ops"], key=lambda o: o["pos"])
             if o["type"] == "kernel"][:12]
    assert all(nm.endswith(("_q", "_k", "_v")) for nm in first)
    ok, errs, _ = validator.check_schedule(spec, one)
    assert ok, errs[:5]


def test_exec_per_cu_must_not_be_negative():
    dag = psc.build_dag(workloads.forkjoin_spec(4))
    try:
        with pytest.raises(psc.PscError) as e:
            psc.psc_schedule(dag, "device", exec_per_cu=-1)
        assert e.value.status == psc.PSC_ERR_ARG
        psc.psc_sched_destroy(psc.psc_schedule(dag, "device", exec_per_cu=1))
    finally:
        psc.psc_dag_destroy(dag)


def test_out_of_order_needs_fine_aql():
    spec = workloads.forkjoin_spec(16)
    dag = psc.build_dag(spec)
    try:
        for policy, kw in (("fine", dict(dispatch="hip")), ("coarse", dict(dispatch="aql")),
                           ("device", {}), ("eager", dict(n_streams=2))):
            with pytest.raises(psc.PscError) as e:
                psc.psc_schedule(dag, policy, out_of_order=True, **kw)
            assert e.value.status in (psc.PSC_ERR_UNSUPPORTED, psc.PSC_ERR_ARG)
    finally:
        psc.psc_dag_destroy(dag)


def test_copy_roots_uploads_each_read_only_root_once():
    """copy_roots: the per-head weight windows of an attention layer are uploaded as one dense
    copy of each weight matrix (and X once), every reader of a window waiting for it."""
    spec = workloads.mha_spec(64, 64, 4, layers=2)
    for policy, kw in (("coarse", {}), ("fine", dict(n_streams=4, mapper="component", copy_stream=True)),
                       ("eager", dict(n_streams=2))):
        dag = psc.build_dag(spec)
        try:
            sched = psc.psc_schedule(dag, policy, copy_roots=True, **kw)
            if policy == "eager":
                psc.psc_sched_destroy(sched)
                continue       # its structure is known after a run only
            exp = psc.export_schedule(spec, sched)
            psc.psc_sched_destroy(sched)
        finally:
            psc.psc_dag_destroy(dag)
        ups = sorted(o["buffer"] for o in exp["ops"] if o["type"] == "h2d")
        assert ups == sorted(["X"] + [f"{w}{l}" for l in range(2) for w in ("Wq", "Wk", "Wv", "Wo")]), ups
        ok, errs, _ = validator.check_schedule(spec, exp)
        assert ok, errs[:5]
