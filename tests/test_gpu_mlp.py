"""GPU tests of the learned cost model: forward, gradients and Adam against the FP64 oracle, the
runtime's samples, and the held-out comparison with the roofline heuristic."""
import numpy as np
import pytest

import workloads
import paper_2009_07482_amd as psc
from paper_2009_07482_amd import costmodel
from oracle import mlp as omlp
from oracle import validator
from gpu_helpers import normwise, oracle_outputs

pytestmark = pytest.mark.gpu

F = psc.PSC_FEATURES


def _data(seed, n):
    g = np.random.default_rng(seed)
    x = g.normal(0.0, 1.0, size=(n, F)).astype(np.float32)
    # a smooth target that depends on several features
    t = (0.8 * x[:, 0] - 0.5 * x[:, 3] * x[:, 4] + np.sin(x[:, 6]) + 0.3 * x[:, 11] ** 2).astype(np.float32)
    return x, t


@pytest.fixture
def model():
    m = psc.psc_mlp_create(0)
    yield m
    psc.psc_mlp_destroy(m)


@pytest.mark.parametrize("n", [1, 63, 64, 300])
def test_forward_matches_oracle(model, n):
    p = workloads.mlp_init(3, F)
    x, _ = _data(n, n)
    psc.psc_mlp_set_params(model, psc.mlp_flatten(p))
    y = psc.psc_mlp_predict(model, x)
    y0, _ = omlp.forward(p, x)
    assert normwise(y, y0) < 1e-5


def test_forward_applies_feature_scaling(model):
    p = workloads.mlp_init(4, F)
    x, _ = _data(5, 200)
    mean = np.linspace(-1, 1, F).astype(np.float32)
    std = np.linspace(0.5, 2.0, F).astype(np.float32)
    psc.psc_mlp_set_params(model, psc.mlp_flatten(p))
    psc.psc_mlp_set_norm(model, mean, std)
    y = psc.psc_mlp_predict(model, x)
    y0, _ = omlp.forward(p, (x.astype(np.float64) - mean) / std)
    assert normwise(y, y0) < 1e-5


@pytest.mark.parametrize("n", [17, 256])
def test_gradients_match_oracle(model, n):
    p = workloads.mlp_init(6, F)
    x, t = _data(7, n)
    psc.psc_mlp_set_params(model, psc.mlp_flatten(p))
    g, loss = psc.psc_mlp_grad(model, x, t)
    y0, cache = omlp.forward(p, x)
    g0 = omlp.backward(p, cache, y0, t)
    assert loss == pytest.approx(omlp.loss(y0, t), rel=1e-5)
    gg = psc.mlp_unflatten(g)
    for k in omlp.NAMES:
        assert normwise(gg[k], g0[k].reshape(gg[k].shape)) < 1e-4, k
    # parameters unchanged by a gradient evaluation
    assert np.array_equal(psc.psc_mlp_get_params(model), psc.mlp_flatten(p))


def test_adam_steps_match_oracle(model):
    """Two passes of mini-batches 64, 64, 64, 8 in sample order (no shuffle) against FP64 Adam."""
    p = workloads.mlp_init(8, F)
    x, t = _data(9, 200)
    lr = 1e-2
    psc.psc_mlp_set_params(model, psc.mlp_flatten(p))
    psc.psc_mlp_train(model, x, t, epochs=2, batch=64, lr=lr, shuffle_seed=0)
    got = psc.mlp_unflatten(psc.psc_mlp_get_params(model))
    ref = {k: np.asarray(v, np.float64) for k, v in p.items()}
    m, v = omlp.zeros_like(ref), omlp.zeros_like(ref)
    step, small = 0, {k: np.zeros(ref[k].shape, bool) for k in omlp.NAMES}
    for _ in range(2):
        for b0 in range(0, 200, 64):
            xb, tb = x[b0:b0 + 64], t[b0:b0 + 64]
            y, cache = omlp.forward(ref, xb)
            g = omlp.backward(ref, cache, y, tb)
            for k in omlp.NAMES:   # gradients near zero: the sign of Adam's first step is rounding-decided
                small[k] |= np.abs(g[k]) < 1e-4 * np.sqrt(np.mean(g[k] ** 2)) + 1e-12
            step += 1
            ref, m, v = omlp.adam_step(ref, g, m, v, step, lr=lr)
    for k in omlp.NAMES:
        d = np.abs(got[k].astype(np.float64) - ref[k].reshape(got[k].shape))
        moved = np.abs(ref[k] - np.asarray(p[k], np.float64)).reshape(d.shape)
        sm = small[k].reshape(d.shape)
        assert np.all(d[~sm] <= 1e-3 * moved[~sm] + 1e-6), k
        assert np.all(d[sm] <= 2 * lr * step), k


def test_training_reduces_loss_and_is_deterministic(model):
    x, t = _data(10, 2000)
    p = psc.mlp_flatten(workloads.mlp_init(11, F))
    psc.psc_mlp_set_params(model, p)
    l1 = psc.psc_mlp_train(model, x, t, epochs=30, batch=128, lr=3e-3, shuffle_seed=5)
    w1 = psc.psc_mlp_get_params(model)
    assert l1[-1] < 0.2 * l1[0]
    psc.psc_mlp_set_params(model, p)
    l2 = psc.psc_mlp_train(model, x, t, epochs=30, batch=128, lr=3e-3, shuffle_seed=5)
    assert np.array_equal(l1, l2) and np.array_equal(w1, psc.psc_mlp_get_params(model))


def test_bad_arguments(model):
    with pytest.raises(psc.PscError):
        psc.psc_mlp_set_norm(model, np.zeros(F), np.zeros(F))
    with pytest.raises(psc.PscError):
        psc.psc_mlp_train(model, np.zeros((4, F)), np.zeros(4), epochs=0)


def test_samples_of_a_recorded_run():
    spec = workloads.mha_spec(512, 512, 8)
    inp = workloads.mha_inputs(0, 512, 512)
    X, t = costmodel.record_samples(spec, inp, n_streams=4, mapper="component", runs=1)
    # one sample per op: 57 kernels, an upload per isolated write (X, Wo and the 24 per-head
    # weight slices) and the read-back of Y
    assert X.shape == (57 + 26 + 1, F) and np.all(np.isfinite(t))
    kinds = X[:, :6].argmax(axis=1)
    assert np.all(X[:, :6].sum(axis=1) == 1)
    assert np.bincount(kinds, minlength=6).tolist() == [41, 8, 8, 0, 26, 1]
    assert np.all((X[:, 11] >= 0) & (X[:, 11] <= 3)) and X[:, 11].max() >= 1
    # a 512 x 64 x 512 projection: log2 M, N, K and bytes
    g = X[(kinds == 0) & (X[:, 8] == 9) & (X[:, 7] == 6)][0]
    assert g[6] == 9 and g[9] == pytest.approx(np.log2(4 * (512 * 512 + 512 * 64 + 512 * 64)))
    Xd, _ = costmodel.record_samples(spec, None, n_streams=2, runs=1)
    assert Xd.shape == (57, F)   # device-resident: kernels only
    # one row per op with the median over runs
    Xm, tm = costmodel.record_samples(spec, None, n_streams=2, runs=3, reduce="median")
    assert Xm.shape == (57, F) and np.array_equal(Xm[:, :11], Xd[:, :11]) and np.all(np.isfinite(tm))


def _collect(seeds, dim=(64, 1024), nodes=(40, 120)):
    xs, ts = [], []
    for i, sd in enumerate(seeds):
        spec = workloads.random_dag_spec(sd, n_nodes=nodes, dim=dim)
        inp = workloads.random_dag_inputs(sd, spec) if i % 3 == 0 else None
        x, t = costmodel.record_samples(spec, inp, n_streams=(1, 2, 4, 8)[i % 4], runs=2)
        xs.append(x)
        ts.append(t)
    return np.concatenate(xs), np.concatenate(ts)


@pytest.mark.timeout(600)
def test_learned_model_beats_heuristic_on_held_out_dags():
    X, t = _collect(range(0, 24))
    Xh, th = _collect(range(1000, 1006))
    cm = costmodel.fit(X, t, epochs=60, batch=256, lr=2e-3, seed=0)
    try:
        assert cm.losses[-1] < cm.losses[0]
        e_mlp = costmodel.mape(cm.predict_us(Xh), th)
        e_heu = costmodel.mape(psc.psc_cost_predict(Xh), th)
        print(f"\nheld-out op-time MAPE: mlp {e_mlp:.3f}, heuristic {e_heu:.3f} "
              f"({len(t)} training / {len(th)} held-out samples)")
        assert e_mlp < e_heu and e_mlp < 0.5
        # EFT under the learned model: a valid schedule whose results equal the coarse schedule's
        spec = workloads.random_dag_spec(1003, n_nodes=(40, 120), dim=(64, 1024))
        inp = workloads.random_dag_inputs(1003, spec)
        r = psc.SpecRunner(spec, "fine", n_streams=4, mapper="eft", cost=cm.handle)
        ok, errs, _ = validator.check_schedule(spec, r.export())
        assert ok, errs
        r.set_inputs(inp)
        r.run()
        got = {k: r.result(k) for k in r.out_names}
        r.close()
        want, _ = psc.run_spec(spec, inp, "coarse")
        for k in want:
            assert np.array_equal(got[k], want[k]), k
        # what the learned model changes in measured makespan: EFT under each model and round
        # robin on held-out random DAGs and on attention DAGs (many small kernels), device-resident,
        # median of 9 runs each.  The schedules run on AQL queues -- one hardware queue per stream:
        # HIP streams share the runtime's four hardware queues round robin in creation order, so
        # which of a schedule's streams end up on one queue (and run serially) would depend on what
        # the process created before, not on the mapping under test
        dags = [workloads.random_dag_spec(sd, n_nodes=(40, 120), dim=(64, 1024)) for sd in range(1000, 1006)]
        dags += [workloads.mha_spec(512, 512, 8), workloads.mha_spec(512, 512, 8, gemm_dtype="bf16")]
        ratios_h, ratios_rr = [], []
        for spec in dags:
            med, exps = [], []
            for kw in (dict(mapper="eft", cost=cm.handle), dict(mapper="eft", cost=None), dict(mapper="rr")):
                r = psc.SpecRunner(spec, "fine", n_streams=4, dispatch="aql", host_threads=1, timeout_ms=30000, **kw)
                try:
                    exps.append(r.export())
                    r.run(with_inputs=False, with_outputs=False)
                    med.append(float(np.median([r.run(with_inputs=False, with_outputs=False)["makespan_ms"]
                                                for _ in range(9)])))
                finally:
                    r.close()
            use = [np.bincount([o["stream"] for o in e["ops"] if o["type"] == "kernel"], minlength=4).tolist()
                   for e in exps]
            ratios_h.append(med[0] / med[1])
            ratios_rr.append(med[0] / med[2])
            print(f"  {len(spec['kernels'])} kernels: eft-mlp {med[0]:.3f} ms, eft-heuristic {med[1]:.3f}, "
                  f"rr {med[2]:.3f}; kernels per stream {use}", flush=True)
        gm_h = float(np.exp(np.mean(np.log(ratios_h))))
        gm_rr = float(np.exp(np.mean(np.log(ratios_rr))))
        print(f"makespan eft-mlp / eft-heuristic: geometric mean {gm_h:.3f} (min {min(ratios_h):.3f}, "
              f"max {max(ratios_h):.3f}); eft-mlp / rr {gm_rr:.3f}", flush=True)
        # the learned model predicts op times better; whether it shortens these schedules is
        # within run-to-run noise (the design notes give the measured ratios) -- what is asserted
        # is that it makes them no worse
        assert gm_h < 1.08 and gm_rr < 1.08, (ratios_h, ratios_rr)
    finally:
        cm.close()


def test_save_load_resumes_training(tmp_path):
    """Two passes of Adam equal one pass, save, load into a fresh model, one more pass -- bit for
    bit: the file carries the parameters, both moments, the step count and the feature scaling."""
    p = workloads.mlp_init(21, F)
    x, t = _data(22, 300)
    mean = np.linspace(-0.5, 0.5, F).astype(np.float32)
    std = np.linspace(0.5, 1.5, F).astype(np.float32)
    a, b, c = (psc.psc_mlp_create(0) for _ in range(3))
    try:
        for mm in (a, b):
            psc.psc_mlp_set_norm(mm, mean, std)
            psc.psc_mlp_set_params(mm, psc.mlp_flatten(p))
        psc.psc_mlp_train(a, x, t, epochs=2, batch=64, lr=1e-2, shuffle_seed=0)
        psc.psc_mlp_train(b, x, t, epochs=1, batch=64, lr=1e-2, shuffle_seed=0)
        path = str(tmp_path / "model.bin")
        psc.psc_mlp_save(b, path)
        assert psc.psc_mlp_file_check(path) == 5          # ceil(300 / 64) Adam steps
        psc.psc_mlp_load(c, path)
        np.testing.assert_array_equal(psc.psc_mlp_predict(c, x), psc.psc_mlp_predict(b, x))
        psc.psc_mlp_train(c, x, t, epochs=1, batch=64, lr=1e-2, shuffle_seed=0)
        np.testing.assert_array_equal(psc.psc_mlp_get_params(c), psc.psc_mlp_get_params(a))
    finally:
        for mm in (a, b, c):
            psc.psc_mlp_destroy(mm)


def test_damaged_model_file_changes_nothing_and_falls_back(tmp_path):
    p = workloads.mlp_init(23, F)
    m = psc.psc_mlp_create(0)
    try:
        psc.psc_mlp_set_params(m, psc.mlp_flatten(p))
        path = str(tmp_path / "model.bin")
        psc.psc_mlp_save(m, path)
        raw = bytearray(open(path, "rb").read())
        raw[4321] ^= 0x01
        bad = str(tmp_path / "bad.bin")
        open(bad, "wb").write(bytes(raw))
        psc.psc_mlp_set_params(m, psc.mlp_flatten(workloads.mlp_init(24, F)))
        before = psc.psc_mlp_get_params(m)
        with pytest.raises(psc.PscError) as e:
            psc.psc_mlp_load(m, bad)
        assert e.value.status == psc.PSC_ERR_IO
        np.testing.assert_array_equal(psc.psc_mlp_get_params(m), before)
        model, why = costmodel.load(bad)
        assert model is None and "checksum" in why
        # the heuristic schedules the DAG instead, and the result is still right
        spec = workloads.mha_spec(128, 128, 2)
        inp = workloads.mha_inputs(0, 128, 128)
        out, _ = psc.run_spec(spec, inp, "fine", n_streams=2, mapper="eft", cost=None)
        assert normwise(out["Y0"], oracle_outputs(spec, inp)["Y0"]) < 1e-4
        good, why = costmodel.load(path)
        assert why is None
        np.testing.assert_array_equal(psc.psc_mlp_get_params(good.handle), psc.mlp_flatten(p))
        good.close()
    finally:
        psc.psc_mlp_destroy(m)
