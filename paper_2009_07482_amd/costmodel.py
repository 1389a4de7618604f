"""Learned cost model workflow: record op timings, fit the MLP on the GPU, use it for EFT mapping.

The paper names machine-learning assisted scheduling as future work (Sec. VII).  Samples come
from the runtime itself: a schedule run with ``record_ops`` yields one (features, ln us) row per
op that did work (``psc_sched_samples``); ``fit`` z-scores the features, initialises the
perceptron and trains it with the library's GPU kernels; the resulting handle goes into
``psc_sched_opts.cost`` with the EFT mapper.
"""
import numpy as np

import paper_2009_07482_amd as psc


def record_samples(spec, inputs=None, n_streams=4, mapper="rr", runs=2, device=0, reduce=None):
    """Run ``spec`` ``runs`` times (after one warm-up) with per-op timing; returns (X, t).

    With ``inputs`` (host arrays by name) the host copies run and are sampled too; without, the
    data stays on the device and only kernels are sampled.  ``reduce=None`` returns every run's
    rows; ``reduce="median"`` one row per op with the median of its ``runs`` log-durations (single
    event-timed runs under concurrency vary by ~0.23 in ln us between repeats).
    """
    r = psc.SpecRunner(spec, "fine", n_streams=n_streams, mapper=mapper, record_ops=True,
                       host_threads=1, device=device)
    try:
        if inputs is not None:
            r.set_inputs(inputs)
        with_io = inputs is not None
        r.run(with_inputs=with_io, with_outputs=with_io)
        xs, ts = [], []
        for _ in range(runs):
            r.run(with_inputs=with_io, with_outputs=with_io)
            x, t = r.samples()
            xs.append(x)
            ts.append(t)
        if reduce == "median":
            # the same ops do work in every run, in op order; only the busy-stream count may differ
            assert all(len(x) == len(xs[0]) and np.array_equal(x[:, :11], xs[0][:, :11]) for x in xs)
            X = xs[0].copy()
            X[:, 11] = np.median(np.stack([x[:, 11] for x in xs]), axis=0)
            return X, np.median(np.stack(ts), axis=0)
        return np.concatenate(xs), np.concatenate(ts)
    finally:
        r.close()


class CostModel:
    """An MLP cost model living on one GPU (owns a psc_mlp handle)."""

    def __init__(self, handle, mean, std, losses):
        self.handle = handle
        self.mean, self.std, self.losses = mean, std, losses

    def predict_us(self, X):
        return psc.psc_cost_predict(X, self.handle)

    def save(self, path):
        """Parameters, Adam state and feature scaling to ``path`` (psc_mlp_save)."""
        psc.psc_mlp_save(self.handle, path)

    def close(self):
        if self.handle is not None:
            psc.psc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(X, t, epochs=60, batch=256, lr=1e-3, seed=0, device=0):
    """Train the cost model on samples (X [n, 12], t = ln us [n]) and return a CostModel."""
    import workloads
    X = np.ascontiguousarray(X, np.float32)
    t = np.ascontiguousarray(t, np.float32)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0).astype(np.float32)
    params = workloads.mlp_init(seed, psc.PSC_FEATURES)
    params["b3"] = np.array([t.mean()], np.float32)   # start at the mean log duration
    h = psc.psc_mlp_create(device)
    try:
        psc.psc_mlp_set_norm(h, mean, std)
        psc.psc_mlp_set_params(h, psc.mlp_flatten(params))
        losses = psc.psc_mlp_train(h, X, t, epochs=epochs, batch=batch, lr=lr, shuffle_seed=seed + 1)
    except Exception:
        psc.psc_mlp_destroy(h)
        raise
    return CostModel(h, mean, std, losses)


def load(path, device=0):
    """(CostModel, None) for a cost-model file that loads, else (None, reason): a missing,
    truncated, altered or non-finite file is refused whole by the library, and the caller then
    schedules with the roofline heuristic (``cost=None``)."""
    try:
        psc.psc_mlp_file_check(path)
    except psc.PscError as e:
        return None, str(e)
    h = psc.psc_mlp_create(device)
    try:
        psc.psc_mlp_load(h, path)
    except psc.PscError as e:
        psc.psc_mlp_destroy(h)
        return None, str(e)
    return CostModel(h, None, None, None), None


def mape(pred_us, t_log_us):
    """Mean absolute percentage error of predicted durations against measured ln-durations."""
    meas = np.exp(np.asarray(t_log_us, np.float64))
    return float(np.mean(np.abs(np.asarray(pred_us, np.float64) - meas) / meas))
