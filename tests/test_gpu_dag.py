"""DAG-level parity on the GPU: the fork-join and attention DAGs under every policy against the
FP64 oracle; coarse, fine, graph and device-resident runs bit-identical to each other; the fine
schedule's timeline shows concurrent kernels."""
import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import dag as odag
from oracle import validator
from gpu_helpers import normwise, oracle_outputs

pytestmark = pytest.mark.gpu

POLICIES = [("coarse", {}), ("fine", dict(n_streams=2, mapper="rr")), ("fine", dict(n_streams=3, mapper="rr")),
            ("fine", dict(n_streams=4, mapper="eft")), ("fine", dict(n_streams=4, mapper="component")),
            ("fine", dict(n_streams=4, mapper="rr", copy_stream=True)),
            ("fine", dict(n_streams=4, mapper="rr", use_graph=True)), ("device", {})]


def _pid(p):
    policy, kw = p
    return "-".join([policy] + [f"{k}{int(v) if isinstance(v, bool) else v}" for k, v in kw.items()]).replace(
        "use_graph1", "graph")


POLICY_PARAMS = [pytest.param(p, kw, id=_pid((p, kw))) for p, kw in POLICIES]


@pytest.mark.parametrize("policy,kw", POLICY_PARAMS)
def test_forkjoin_ternary_bit_exact(policy, kw):
    print(f"forkjoin ternary {policy} {kw}", flush=True)
    spec = workloads.forkjoin_spec(256)
    inp = workloads.forkjoin_inputs(0, 256, ternary=True)
    out, st = psc.run_spec(spec, inp, policy, **kw)
    np.testing.assert_array_equal(out["C3"], oracle_outputs(spec, inp)["C3"])
    assert st["n_kernels"] == 4


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("policy,kw", POLICY_PARAMS)
def test_forkjoin_uniform(seed, policy, kw):
    spec = workloads.forkjoin_spec(256)
    inp = workloads.forkjoin_inputs(seed, 256)
    out, _ = psc.run_spec(spec, inp, policy, **kw)
    assert normwise(out["C3"], oracle_outputs(spec, inp)["C3"]) < 1e-4


def test_forkjoin_bf16_c0_ternary_exact():
    spec = workloads.forkjoin_spec(256, dtype="bf16", c0_dtype="bf16")
    inp = workloads.forkjoin_inputs(1, 256, ternary=True)
    out, _ = psc.run_spec(spec, inp, "fine", n_streams=3)
    np.testing.assert_array_equal(out["C3"], oracle_outputs(spec, inp)["C3"])


@pytest.fixture(scope="module")
def mha512():
    spec = workloads.mha_spec(512, 512, 8)
    inp = workloads.mha_inputs(0, 512, 512)
    ref = oracle_outputs(spec, inp)["Y0"]
    return spec, inp, ref


@pytest.mark.parametrize("policy,kw", POLICY_PARAMS + [pytest.param("fine", dict(n_streams=8, mapper="rr"), id="fine-8rr")])
def test_mha_fp32_against_oracle(mha512, policy, kw):
    print(f"mha512 {policy} {kw}", flush=True)
    spec, inp, ref = mha512
    out, _ = psc.run_spec(spec, inp, policy, **kw)
    assert normwise(out["Y0"], ref) < 1e-4


def test_mha_coarse_fine_resident_bit_identical(mha512):
    spec, inp, _ = mha512
    outs = []
    for policy, kw in [p for p in POLICIES if not p[1].get("use_graph") and p[0] != "device"]:
        r = psc.SpecRunner(spec, policy, **kw)
        r.set_inputs(inp)
        r.run()
        outs.append(r.result("Y0"))
        # device-resident second run: no copies in, results stay on the device and are read back
        r.run(with_inputs=False, with_outputs=False)
        r.run(with_inputs=False, with_outputs=True)
        outs.append(r.result("Y0"))
        r.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_graph_matches_eager_bit_identical(mha512):
    spec, inp, _ = mha512
    outs = []
    for kw in (dict(n_streams=4, mapper="rr"), dict(n_streams=4, mapper="rr", use_graph=True)):
        r = psc.SpecRunner(spec, "fine", **kw)
        r.set_inputs(inp)
        r.run()
        outs.append(r.result("Y0"))
        r.run(with_inputs=False, with_outputs=True)
        outs.append(r.result("Y0"))
        r.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_graph_replays_match_eager(mha512):
    spec, inp, _ = mha512
    eager = psc.SpecRunner(spec, "fine", n_streams=4)
    eager.set_inputs(inp)
    eager.run()
    want = eager.result("Y0")
    g = psc.SpecRunner(spec, "fine", n_streams=4, use_graph=True)
    g.set_inputs(inp)
    for i in range(4):
        g.outputs["Y0"].array[...] = 0
        g.run()
        np.testing.assert_array_equal(g.result("Y0"), want)
        eager.run()  # eager work between replays
    eager.close()
    g.close()


def test_fine_timeline_overlaps_kernels(mha512):
    spec, inp, _ = mha512
    r = psc.SpecRunner(spec, "fine", n_streams=4, record_ops=True)
    r.set_inputs(inp)
    r.run()
    r.run()
    times = psc.psc_sched_op_times(r.sched)
    exp = r.export()
    r.close()
    kern = [(t[1], t[2], t[3]) for t, o in zip(times, exp["ops"]) if o["type"] == "kernel"]
    overlaps = 0
    for i in range(len(kern)):
        for j in range(i + 1, len(kern)):
            a, b = kern[i], kern[j]
            if a[0] != b[0] and a[1] < b[2] and b[1] < a[2]:
                overlaps += 1
    print("overlapping kernel pairs on different streams:", overlaps)
    assert overlaps >= 1
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs


@pytest.mark.parametrize("n,d,h,layers,dt", [(137, 64, 2, 2, "f32"), (200, 128, 4, 1, "bf16"),
                                             (1000, 64, 1, 1, "f32"), (64, 512, 8, 3, "bf16")])
def test_ragged_attention(n, d, h, layers, dt):
    print(f"ragged mha n={n} d={d} h={h} L={layers} {dt}", flush=True)
    spec = workloads.mha_spec(n, d, h, layers, gemm_dtype=dt)
    inp = workloads.mha_inputs(3, n, d, layers)
    out, _ = psc.run_spec(spec, inp, "fine", n_streams=4, copy_stream=True)
    y = f"Y{layers - 1}"
    exact = oracle_outputs(spec, inp)[y]
    assert normwise(out[y], exact) < (1e-4 if dt == "f32" else 2e-2)


@pytest.mark.parametrize("policy,kw", [("coarse", {}), ("fine", dict(n_streams=4, mapper="eft")), ("device", {})],
                         ids=["coarse", "fine-eft", "device"])
def test_random_dags_against_oracle(policy, kw):
    """Random layered DAGs (seeds 0-7: six draw BF16, two FP32).  Every output against the exact
    FP64 oracle (1e-4 FP32, 2e-2 BF16) and, for BF16, against the storage-emulating oracle, which
    rounds exactly where the GPU stores: what is left there is FP32 accumulation order and the
    rare rounding decision it flips, so the bar is 5e-3, below the ~4e-3 that BF16 storage
    itself costs against the exact result on these DAGs."""
    for seed in range(8):
        spec = workloads.random_dag_spec(seed, n_nodes=(20, 40), dim=(8, 160))
        inp = workloads.random_dag_inputs(seed, spec)
        ref = oracle_outputs(spec, inp)
        emul = oracle_outputs(spec, inp, emulate=True) if spec["dtype"] == "bf16" else None
        out, _ = psc.run_spec(spec, inp, policy, **kw)
        worst = (0.0, 0.0)
        for name, want in ref.items():
            e = normwise(out[name], want)
            assert e < (1e-4 if spec["dtype"] == "f32" else 2e-2), (seed, policy, name, e)
            if emul is not None:
                e2 = normwise(out[name], emul[name])
                assert e2 < 5e-3, (seed, policy, name, e2)
                worst = (max(worst[0], e), max(worst[1], e2))
        print(f"seed {seed} {spec['dtype']}: worst error vs exact {worst[0]:.2e}, vs emulating {worst[1]:.2e}",
              flush=True)


def test_io_errors():
    spec = workloads.forkjoin_spec(16)
    r = psc.SpecRunner(spec, "fine")
    with pytest.raises(psc.PscError) as e:
        psc.psc_run(r.sched, [("C1", 0, 16 * 16 * 4)])   # C1 is neither written nor read back
    assert e.value.name in ("PSC_ERR_NAME", "PSC_ERR_ARG")
    with pytest.raises(psc.PscError) as e:
        t = psc.HostBuffer(16, 16, "f32")
        psc.psc_run(r.sched, [("A0", t.ptr, 7)])
    assert e.value.name == "PSC_ERR_ARG"
    r.close()


def test_device_executor_matches_streams_bit_identical(mha512):
    # the executor's GEMM tiles may differ from the standalone choice, so compare to the oracle and
    # check repeated device runs agree bit for bit with each other
    spec, inp, ref = mha512
    r = psc.SpecRunner(spec, "device")
    r.set_inputs(inp)
    r.run()
    first = r.result("Y0")
    assert normwise(first, ref) < 1e-4
    for _ in range(5):
        r.run(with_inputs=False, with_outputs=True)
        np.testing.assert_array_equal(r.result("Y0"), first)
    r.close()


@pytest.mark.parametrize("gemm_dtype", ["f32", "bf16"])
def test_device_executor_takes_a_smaller_instance(gemm_dtype):
    # an attention DAG needs the 64 x 64 and direct-load GEMM tiles and the element-wise kernels
    # only: the executor takes an instance holding just those (FP32: two per CU on the MI355X
    # boxes measured, 244-256 registers; BF16 with K >= 256: its 64 x 64 K-split tile is held by
    # the every-BF16-tile instance, one per CU), not the one holding every tile function, with as
    # many workgroups as the runtime says the device holds of it; its results match the oracle
    spec = workloads.mha_spec(512, 512, 8, gemm_dtype=gemm_dtype)
    inp = workloads.mha_inputs(1, 512, 512)
    ref = odag.read_buffer(spec, odag.run_dag(spec, inp), "Y0")
    r = psc.SpecRunner(spec, "device")
    psc.psc_sched_prepare(r.sched)
    workers, per_cu, groups = psc.psc_sched_executor_info(r.sched)
    cus = psc.psc_device_info(0)["compute_units"]
    print(f"{gemm_dtype}: {workers} workers, {per_cu} per CU on {cus} CUs, groups {groups:#x}", flush=True)
    assert per_cu >= 1 and 0 < workers <= per_cu * cus
    assert groups != 0x7FFF and groups & (1 << 13)
    assert not groups & 0x3F if gemm_dtype == "bf16" else not groups & 0x1FC0
    r.set_inputs(inp)
    r.run()
    assert normwise(r.result("Y0"), ref) < (1e-4 if gemm_dtype == "f32" else 2e-2)
    r.close()


def _independent_gemms_spec(count, M, N, K):
    """`count` independent BF16 GEMMs C_i = A_i B_i (M x K times K x N), outputs alternately FP32
    and BF16: with this many kernels side by side each expects few workgroups, so the executor
    gives them 64 x 64 tasks, which for BF16 with K >= 256 run K-split."""
    bufs, kers = [], []
    for i in range(count):
        bufs += [{"name": f"A{i}", "dtype": "bf16", "rows": M, "cols": K, "view_of": None, "row_off": 0, "col_off": 0},
                 {"name": f"B{i}", "dtype": "bf16", "rows": K, "cols": N, "view_of": None, "row_off": 0, "col_off": 0},
                 {"name": f"C{i}", "dtype": "bf16" if i % 2 else "f32", "rows": M, "cols": N, "view_of": None,
                  "row_off": 0, "col_off": 0}]
        kers.append({"name": f"g{i}", "kind": "gemm", "inputs": [f"A{i}", f"B{i}"], "outputs": [f"C{i}"], "alpha": 1.0})
    return {"buffers": bufs, "kernels": kers, "edges": [], "component": list(range(count))}


@pytest.mark.parametrize("values", ["ternary", "uniform"])
def test_device_executor_ksplit_64x64_tasks(values):
    """The executor's 64 x 64 K-split BF16 task (each wavefront a quarter of K, partial blocks
    summed through LDS) on ragged shapes: M = 200 and N = 136 leave partial row and column tiles,
    K = 1000 a partial last 64-deep chunk.  Ternary operands make every product sum an integer
    below 2^24, exact in FP32 whatever the summation order: FP32 outputs equal the oracle bit for
    bit, BF16 outputs equal its storage-rounding emulation.  Uniform operands: the exact oracle
    (unrounded inputs) within the BF16 bar of 2e-2, the emulating one (inputs and outputs rounded
    where the GPU stores them) within 1e-5 for FP32 outputs and 5e-3 for BF16 outputs."""
    M, N, K, count = 200, 136, 1000, 32
    spec = _independent_gemms_spec(count, M, N, K)
    g = np.random.default_rng(7)
    inp = {}
    for i in range(count):
        for name, shape in ((f"A{i}", (M, K)), (f"B{i}", (K, N))):
            inp[name] = (g.integers(-1, 2, size=shape).astype(np.float32) if values == "ternary"
                         else g.uniform(-1.0, 1.0, size=shape).astype(np.float32))
    r = psc.SpecRunner(spec, "device")
    psc.psc_sched_prepare(r.sched)
    workers, per_cu, groups = psc.psc_sched_executor_info(r.sched)
    print(f"{workers} workers, {per_cu} per CU, groups {groups:#x}", flush=True)
    assert groups & (1 << 14), "the plan does not use the K-split 64 x 64 task"
    r.set_inputs(inp)
    r.run()
    out = {n: r.result(n) for n in r.out_names}
    r.close()
    exact = oracle_outputs(spec, inp)
    emul = oracle_outputs(spec, inp, emulate=True)
    for i in range(count):
        name = f"C{i}"
        if values == "ternary":
            np.testing.assert_array_equal(out[name], emul[name], err_msg=name)
            if i % 2 == 0:
                np.testing.assert_array_equal(out[name], exact[name], err_msg=name)
        else:
            assert normwise(out[name], exact[name]) < 2e-2, name
            assert normwise(out[name], emul[name]) < (5e-3 if i % 2 else 1e-5), name


def test_device_executor_one_workgroup_per_cu_on_request():
    # exec_per_cu = 1 caps the executor at one workgroup per CU; same results as the default
    spec = workloads.mha_spec(512, 512, 8)
    inp = workloads.mha_inputs(1, 512, 512)
    ref = odag.read_buffer(spec, odag.run_dag(spec, inp), "Y0")
    cus = psc.psc_device_info(0)["compute_units"]
    r = psc.SpecRunner(spec, "device", exec_per_cu=1)
    psc.psc_sched_prepare(r.sched)
    workers, per_cu, groups = psc.psc_sched_executor_info(r.sched)
    print(f"{workers} workers, {per_cu} per CU, groups {groups:#x}", flush=True)
    assert per_cu == 1 and 0 < workers <= cus
    r.set_inputs(inp)
    r.run()
    assert normwise(r.result("Y0"), ref) < 1e-4
    r.close()


def test_device_executor_runs_copies_beside_kernels():
    """PSC_DEVICE with page-locked host buffers: the executor's own workgroups run the uploads
    and the read-back as tasks, so later layers' weights arrive while the first layer computes.
    Per-op device clocks: every upload ends before its readers start, the read-back starts after
    its writer ends, an upload overlaps a kernel, and the output matches the oracle."""
    spec = workloads.mha_spec(512, 512, 8, layers=3, gemm_dtype="bf16")
    inp = workloads.mha_inputs(1, 512, 512, 3)
    ref = odag.read_buffer(spec, odag.run_dag(spec, inp), "Y2")
    r = psc.SpecRunner(spec, "device", record_ops=True)
    r.set_inputs(inp)
    r.run()
    r.run()
    got = r.result("Y2")
    times = psc.psc_sched_op_times(r.sched)
    exp = r.export()
    r.close()
    assert normwise(got, ref) < 2e-2
    t = {o["id"]: (tt[2], tt[3]) for tt, o in zip(times, exp["ops"])}
    copies = [o for o in exp["ops"] if o["type"] != "kernel"]
    if not any(t[o["id"]][1] > 0 for o in copies):
        pytest.skip("this runtime does not map page-locked host memory at the same device address: "
                    "every copy ran by DMA")
    assert all(t[o["id"]][1] > 0 for o in copies), "a copy was not run by the executor"
    for o in exp["ops"]:
        for w in o["waits"]:
            if o["type"] != "kernel" or exp["ops"][w]["type"] != "kernel":
                assert t[w][1] <= t[o["id"]][0] + 0.5, (w, o["id"])
    kernels = [t[o["id"]] for o in exp["ops"] if o["type"] == "kernel"]
    ups = [t[o["id"]] for o in copies if o["type"] == "h2d"]
    overlapping = sum(1 for c in ups for k in kernels if c[0] < k[1] and k[0] < c[1])
    print(f"upload/kernel overlapping pairs: {overlapping}", flush=True)
    assert overlapping >= 1


@pytest.mark.parametrize("pageable", ["all", "weights"])
def test_device_executor_copies_pageable_memory_by_dma(pageable):
    """Host memory the device cannot address (ordinary pageable arrays) is copied by DMA before
    and after the executor: with every array pageable the kernels-only plan runs, with only the
    weights pageable the copy plan runs with those upload nodes empty.  Results match the oracle
    either way, and only executor-run copies carry device times."""
    spec = workloads.mha_spec(256, 256, 4, layers=2, gemm_dtype="bf16")
    inp = workloads.mha_inputs(2, 256, 256, 2)
    ref = odag.read_buffer(spec, odag.run_dag(spec, inp), "Y1")
    r = psc.SpecRunner(spec, "device", copy_roots=True, record_ops=True)
    r.set_inputs(inp)
    io, keep = [], []
    for n, h in r.inputs.items():
        if pageable == "all" or n != "X":
            a = np.array(h.array, copy=True)   # ordinary (pageable) memory, same bytes
            keep.append(a)
            io.append((n, a.ctypes.data, a.nbytes))
        else:
            io.append((n, h.ptr, h.nbytes))
    out = np.zeros((256, 256), np.float32) if pageable == "all" else None
    if out is not None:
        io.append(("Y1", out.ctypes.data, out.nbytes))
    else:
        io += [(n, r.outputs[n].ptr, r.outputs[n].nbytes) for n in r.out_names]
    psc.psc_run(r.sched, io)
    got = out if out is not None else r.result("Y1")
    times = psc.psc_sched_op_times(r.sched)
    exp = r.export()
    r.close()
    assert normwise(got, ref) < 2e-2
    timed = {o["type"]: 0 for o in exp["ops"]}
    for tt, o in zip(times, exp["ops"]):
        if tt[3] > 0:
            timed[o["type"]] += 1
    print(f"{pageable} pageable: ops with device times {timed}", flush=True)
    assert timed["kernel"] == len(spec["kernels"])
    if pageable == "all":
        assert timed["h2d"] == 0 and timed["d2h"] == 0
    elif timed["h2d"] + timed["d2h"] == 0:
        pytest.skip("this runtime does not map page-locked host memory at the same device address")
    else:
        assert timed["h2d"] == 1 and timed["d2h"] == 1   # X and Y1 by the executor, weights by DMA


def test_device_executor_node_times_respect_dependencies():
    spec = workloads.mha_spec(256, 256, 4, layers=2)
    inp = workloads.mha_inputs(2, 256, 256, 2)
    r = psc.SpecRunner(spec, "device", record_ops=True)
    r.set_inputs(inp)
    r.run()
    times = psc.psc_sched_op_times(r.sched)
    exp = r.export()
    r.close()
    t = {o["kernel"]: (tt[2], tt[3]) for tt, o in zip(times, exp["ops"]) if o["type"] == "kernel"}
    for (s_, _, d_, _) in spec["edges"]:
        assert t[s_][1] <= t[d_][0] + 1e-3, (s_, d_, t[s_], t[d_])


@pytest.fixture(scope="module")
def mha12():
    """12 stacked layers, 16 heads, d_model = n = 1024, BF16 GEMM operands (FP32 accumulation),
    FP32 softmax: the last layer's output from the exact FP64 oracle."""
    n, d, h, L = 1024, 1024, 16, 12
    spec = workloads.mha_spec(n, d, h, L, gemm_dtype="bf16")
    inp = workloads.mha_inputs(0, n, d, L)
    y = f"Y{L - 1}"
    exact = odag.read_buffer(spec, odag.run_dag(spec, inp), y)
    return spec, inp, (n, d, h, L), exact, {}


# Layers checked one at a time against the storage-emulating oracle.  The stacked layers have no
# residual or normalisation and amplify rounding-order differences: two valid emulations of the
# BF16 storage (the oracle's FP64 accumulation, and FP32 accumulation like the GPU's) differ by
# 1.0e-3 normwise after one layer but 9.7e-3 after twelve.  So the emulating oracle is a tight
# reference only layer by layer, fed the GPU's own output of the previous layer.
CHECK_LAYERS = (0, 5, 11)
LAYER_TOL = 3e-3


def _layer_errors(r, inp, shape):
    n, d, h, L = shape
    errs = {}
    for l in CHECK_LAYERS:
        x = inp["X"] if l == 0 else r.read_device(f"Y{l - 1}")
        one = workloads.mha_spec(n, d, h, 1, gemm_dtype="bf16", final_dtype="f32" if l == L - 1 else "bf16")
        oinp = {"X": x, **{f"{w}0": inp[f"{w}{l}"] for w in ("Wq", "Wk", "Wv", "Wo")}}
        ref = oracle_outputs(one, oinp, emulate=True)["Y0"]
        errs[l] = normwise(r.read_device(f"Y{l}"), ref)
    return errs


@pytest.mark.timeout(900)
@pytest.mark.parametrize("policy,kw", [("coarse", {}), ("fine", dict(n_streams=4, mapper="rr")),
                                       ("fine", dict(n_streams=4, mapper="component", copy_stream=True)),
                                       ("device", {})],
                         ids=["coarse", "fine-rr", "fine-component-copystream", "device"])
def test_mha_12_layers_bf16_full_size(mha12, policy, kw):
    """The full-size 12-layer DAG under each schedule: the final output Y11 within 2e-2 of the
    exact FP64 oracle; layers 0, 5 and 11, each recomputed by the storage-emulating oracle from
    the GPU's own input to that layer, within 3e-3; the stream schedules bit-identical to each
    other (same kernels, no atomics, fixed reduction order).  The device executor picks its own
    GEMM tiles, so it is held to the oracles only."""
    spec, inp, shape, exact, seen = mha12
    y = f"Y{shape[3] - 1}"
    print(f"mha 12x1024 bf16 {policy} {kw}", flush=True)
    r = psc.SpecRunner(spec, policy, **kw)
    try:
        r.set_inputs(inp)
        st = r.run()
        got = r.result(y)
        np.testing.assert_array_equal(r.read_device(y), got)
        # per-layer checks once for the stream schedules (they are bit-identical), and for the executor
        layer = _layer_errors(r, inp, shape) if policy in ("coarse", "device") else None
    finally:
        r.close()
    e1 = normwise(got, exact)
    print(f"makespan with copies {st['makespan_ms']:.3f} ms; {y} error vs exact {e1:.3e}; "
          f"per-layer vs emulating {layer}", flush=True)
    assert e1 < 2e-2
    if layer is not None:
        assert all(v < LAYER_TOL for v in layer.values()), layer
    if policy != "device":
        if "streams" in seen:
            np.testing.assert_array_equal(got, seen["streams"])
        else:
            seen["streams"] = got
