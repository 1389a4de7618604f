"""The dynamic coarse-grained baselines (eager, HEFT; Sec. V, Experiments 2 and 3) on the GPU:
kernels dispatched one at a time at run time from a ready queue that completion callbacks update.
Results equal the static schedules' bit for bit, the structure each run realised passes the
validator, and the timeline shows the callback gap between dependent kernels that the static
schedules do not have."""
import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from oracle import validator
from gpu_helpers import normwise, oracle_outputs

pytestmark = pytest.mark.gpu

CASES = [("eager", dict(n_streams=1)), ("heft", dict(n_streams=1)), ("eager", dict(n_streams=3)),
         ("heft", dict(n_streams=4))]
IDS = [f"{p}-{kw['n_streams']}q" for p, kw in CASES]


@pytest.mark.parametrize("policy,kw", CASES, ids=IDS)
def test_forkjoin_ternary_bit_exact(policy, kw):
    spec = workloads.forkjoin_spec(256)
    inp = workloads.forkjoin_inputs(0, 256, ternary=True)
    out, st = psc.run_spec(spec, inp, policy, **kw)
    np.testing.assert_array_equal(out["C3"], oracle_outputs(spec, inp)["C3"])
    assert st["n_kernels"] == 4


@pytest.mark.parametrize("policy,kw", CASES, ids=IDS)
def test_mha_matches_static_schedule_and_validates(policy, kw):
    print(f"dynamic mha512 {policy} {kw}", flush=True)
    spec = workloads.mha_spec(512, 512, 8)
    inp = workloads.mha_inputs(0, 512, 512)
    r = psc.SpecRunner(spec, policy, **kw)
    with pytest.raises(psc.PscError) as e:
        r.export()                       # no structure before the first run
    assert e.value.name == "PSC_ERR_STATE"
    r.set_inputs(inp)
    r.run()
    got = r.result("Y0")
    exp = r.export()
    r.run(with_inputs=False, with_outputs=True)
    again = r.result("Y0")
    r.close()
    coarse, _ = psc.run_spec(spec, inp, "coarse")
    np.testing.assert_array_equal(got, coarse["Y0"])
    np.testing.assert_array_equal(again, got)
    assert normwise(got, oracle_outputs(spec, inp)["Y0"]) < 1e-4
    ok, errs, _ = validator.check_schedule(spec, exp)
    assert ok, errs
    assert {o["stream"] for o in exp["ops"]} <= set(range(kw["n_streams"]))


@pytest.mark.parametrize("policy", ["eager", "heft"])
def test_callback_gap_between_dependent_kernels(policy):
    """One queue: every kernel starts only after the host has seen its predecessor's callback, so
    the gap between consecutive kernels exceeds that of the static coarse schedule, which
    enqueues everything up front."""
    spec = workloads.mha_spec(256, 256, 4)
    inp = workloads.mha_inputs(1, 256, 256)
    gaps = {}
    for name, pol, kw in ((policy, policy, dict(n_streams=1)), ("coarse", "coarse", {})):
        r = psc.SpecRunner(spec, pol, record_ops=True, **kw)
        r.set_inputs(inp)
        r.run()
        r.run(with_inputs=False, with_outputs=False)
        t = sorted((tt[2], tt[3]) for tt, o in zip(psc.psc_sched_op_times(r.sched), r.export()["ops"])
                   if o["type"] == "kernel")
        r.close()
        gaps[name] = float(np.median([b[0] - a[1] for a, b in zip(t, t[1:])]))
    print(f"median gap between consecutive kernels: {policy} {gaps[policy]:.1f} us, coarse {gaps['coarse']:.1f} us",
          flush=True)
    assert gaps[policy] > gaps["coarse"]


def test_heft_and_eager_on_random_dags():
    for seed in range(3):
        spec = workloads.random_dag_spec(seed, n_nodes=(20, 40), dim=(8, 160))
        inp = workloads.random_dag_inputs(seed, spec)
        ref, _ = psc.run_spec(spec, inp, "coarse")
        for policy in ("eager", "heft"):
            out, _ = psc.run_spec(spec, inp, policy, n_streams=3)
            for k in ref:
                np.testing.assert_array_equal(out[k], ref[k])
