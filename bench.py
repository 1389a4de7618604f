"""Benchmark: makespan and inferences/s of the attention DAG under coarse- and fine-grained
schedules on one MI355X, with a roofline figure for the dominant kernel and the CPU oracle's
throughput beside it.

Default workload: one multi-head attention layer, n = d = 512, 8 heads of dim 64, FP32 (57
kernels: per head three projection GEMMs, a transpose, the score GEMM, a row softmax and the
P*V GEMM; then the output projection).  A step is one pass of the whole DAG -- every kernel
enqueued on the schedule's streams with its event waits, then a join -- over device-resident
inputs.  ``value`` is inferences/s of the fine-grained schedule: the clustering scheme of Sec. V
(each head's kernels form one task component, components on 4 HIP streams), each stream enqueued
by its own host thread.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config mha512|mha1024x12|forkjoin]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"mfma_f32": 157.3e12, "mfma_bf16": 2.5e15, "hbm": 8.0e12}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--config", default="mha512")
    p.add_argument("--streams", type=int, default=4)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--graph", action="store_true", help="also time the schedule launched as one hipGraph")
    p.add_argument("--kernel-iters", type=int, default=200)
    return p.parse_args()


def workload(name):
    import workloads
    if name == "mha512":
        n, d, h, L, dt = 512, 512, 8, 1, "f32"
    elif name == "mha1024x12":
        n, d, h, L, dt = 1024, 1024, 16, 12, "bf16"
    elif name == "forkjoin":
        spec = workloads.forkjoin_spec(256)
        return spec, workloads.forkjoin_inputs(0, 256), {"workload": "fork-join 4 GEMM/add, 256x256, FP32"}
    else:
        raise SystemExit(f"unknown config {name}")
    spec = workloads.mha_spec(n, d, h, L, gemm_dtype=dt)
    inp = workloads.mha_inputs(0, n, d, L)
    desc = {"workload": f"multi-head attention inference DAG, {L} layer(s), n={n}, d_model={d}, "
                        f"{h} heads of dim {d // h}, GEMM {dt.upper()}",
            "seq_len": n, "d_model": d, "heads": h, "layers": L, "gemm_dtype": dt}
    return spec, inp, desc


def kernel_class(spec, k):
    by = {b["name"]: b for b in spec["buffers"]}
    ker = spec["kernels"][k]
    ins = [by[b] for b in ker["inputs"]]
    out = by[ker["outputs"][0]]
    if ker["kind"] == "gemm":
        m, kk, n = ins[0]["rows"], ins[0]["cols"], ins[1]["cols"]
        return (f"gemm {m}x{n}x{kk} {ins[0]['dtype']}->{out['dtype']}",
                2.0 * m * n * kk, "mfma", ins[0]["dtype"])
    es = {"f32": 4, "bf16": 2}
    nbytes = sum(b["rows"] * b["cols"] * es[b["dtype"]] for b in ins) + out["rows"] * out["cols"] * es[out["dtype"]]
    shape = "x".join(str(v) for v in (ins[0]["rows"], ins[0]["cols"]))
    return (f"{ker['kind']} {shape} {ins[0]['dtype']}->{out['dtype']}", float(nbytes), "hbm", None)


def timed(runner, steps, warmup):
    import paper_2009_07482_amd as psc
    for _ in range(warmup):
        runner.run(with_inputs=False, with_outputs=False)
    psc.psc_device_sync(0)
    mk = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = runner.run(with_inputs=False, with_outputs=False)
        mk.append(st["makespan_ms"])
    psc.psc_device_sync(0)
    wall = time.perf_counter() - t0
    return wall, np.array(mk), st


def cpu_baseline(spec, inp, seconds):
    from oracle import dag as odag
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    n = 0
    t0 = time.perf_counter()
    while True:
        odag.run_dag(spec, inp)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    return {"value": n / el, "unit": "inferences/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} full runs of the same DAG in FP64 (numpy), {el:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import paper_2009_07482_amd as psc

    spec, inp, desc = workload(a.config)
    runners = {
        "coarse": psc.SpecRunner(spec, "coarse"),
        "fine": psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="component"),
        "fine_1thread": psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="component", host_threads=1),
        "fine_rr": psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="rr"),
        "fine_rr_1thread": psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="rr", host_threads=1),
        "fine_eft": psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="eft"),
        "fine_8streams": psc.SpecRunner(spec, "fine", n_streams=8, mapper="component"),
        "device": psc.SpecRunner(spec, "device"),
    }
    if a.graph:
        runners["fine_graph"] = psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="rr", use_graph=True)
    res = {}
    for name, r in runners.items():
        r.set_inputs(inp)
        st_io = r.run()                      # uploads inputs (and measures the PCIe-inclusive makespan)
        for _ in range(3):
            st_io = r.run()
        wall, mk, st = timed(r, a.steps, a.warmup)
        res[name] = {"ms_per_step": wall / a.steps * 1e3, "makespan_ms_median": float(np.median(mk)),
                     "makespan_ms_p5": float(np.percentile(mk, 5)), "makespan_ms_p95": float(np.percentile(mk, 95)),
                     "host_enqueue_ms": st["host_enqueue_ms"], "makespan_with_copies_ms": st_io["makespan_ms"],
                     "n_waits": st["n_waits"], "n_streams": st["n_streams"]}
        print(f"# {name}: {json.dumps(res[name])}", file=sys.stderr, flush=True)

    # Dominant kernel: per kernel class, the mean duration of back-to-back launches on the
    # class's own stream (HIP events around the launches, on that stream) times its launches per
    # step; the class with the largest product dominates the step.
    r = runners["fine"]
    kers = {}
    for k in range(len(spec["kernels"])):
        key, work, bound, dt = kernel_class(spec, k)
        kers.setdefault(key, {"work": work, "bound": bound, "dtype": dt, "ids": []})["ids"].append(k)
    for key, c in kers.items():
        psc.psc_kernel_time(r.sched, c["ids"][0], 10)
        c["avg_us"] = psc.psc_kernel_time(r.sched, c["ids"][0], a.kernel_iters)
        c["total_us"] = c["avg_us"] * len(c["ids"])
    print("# kernel classes (isolated mean us per launch x launches per step):", file=sys.stderr)
    for key, c in sorted(kers.items(), key=lambda kv: -kv[1]["total_us"]):
        print(f"#   {key}: {c['avg_us']:.2f} us x {len(c['ids'])}", file=sys.stderr)
    dom_key = max(kers, key=lambda k: kers[k]["total_us"])
    dom = kers[dom_key]
    avg_us = dom["avg_us"]
    achieved = dom["work"] / (avg_us * 1e-6)
    if dom["bound"] == "mfma":
        peak = PEAK["mfma_bf16"] if dom["dtype"] == "bf16" else PEAK["mfma_f32"]
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None}
    else:
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                "frac": achieved / PEAK["hbm"], "traffic": None}
    roof.update({"kernel": dom_key, "avg_us": avg_us, "launches_per_step": len(dom["ids"]),
                 "work_per_launch": dom["work"], "timing": f"{a.kernel_iters} back-to-back launches, HIP events on its stream"})

    # per-op timeline of the fine schedule (start/end events around every op): concurrency
    rec = psc.SpecRunner(spec, "fine", n_streams=a.streams, mapper="component", record_ops=True)
    rec.set_inputs(inp)
    rec.run()
    rec.run(with_inputs=False, with_outputs=False)
    times = psc.psc_sched_op_times(rec.sched)
    rec.close()
    ivals = sorted((t[2], t[3]) for t in times)
    busy, cur_s, cur_e = 0.0, None, None
    for s0, e0 in ivals:
        if cur_e is None or s0 > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    if cur_e is not None:
        busy += cur_e - cur_s
    op_sum = sum(e0 - s0 for s0, e0 in ivals)
    concurrency = op_sum / busy if busy > 0 else 0.0

    fine = res["fine"]
    value = 1e3 / fine["ms_per_step"]
    line = {
        "metric": "DAG makespan (ms) + inferences/s, fine vs coarse schedule, BF16 vs FP32",
        "value": value, "unit": "inferences/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": fine["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if desc.get("gemm_dtype", "f32") == "f32" else "bf16",
        "data": "synthetic (seeded N(0,1) inputs, N(0,1/d) weights)",
        "config": dict(desc, schedule=f"fine (clustering: one task component per head), {a.streams} HIP streams, "
                                      f"one enqueue thread per stream",
                       inputs="device-resident"),
        "makespan_ms": {k: v["makespan_ms_median"] for k, v in res.items()},
        "ms_per_step_by_schedule": {k: v["ms_per_step"] for k, v in res.items()},
        "makespan_with_copies_ms": {k: v["makespan_with_copies_ms"] for k, v in res.items()},
        "fine_vs_coarse_speedup": res["coarse"]["ms_per_step"] / fine["ms_per_step"],
        "fine_mean_ops_in_flight": concurrency,
        "roofline": roof,
    }
    for r in runners.values():
        r.close()
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(spec, inp, a.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
