// Command-queue setup (setup_cq of Sec. IV-B, Algorithm 1) for one GPU.
//
// Every policy produces a kernel order, which is a topological order (Def. 5), and a stream per
// kernel.  Ops are then emitted per kernel following the enq rules of Sec. III: the kernel's
// isolated writes before its ndrange on its stream, its isolated reads right after it.  All
// kernels share one device here, so the dependent copies of inter edges are not needed: a
// consumer reads the producer's output where it lies.  Cross-stream precedences (rules (i)-(iii))
// become waits on the producing op; a vector clock per op drops waits already implied by stream
// order or by other waits.
#include <algorithm>
#include <cmath>
#include <queue>

#include "core.hpp"

namespace psc {

namespace {

constexpr double kCUs = 256.0;

float lg2(double v) { return v > 1.0 ? float(std::log2(v)) : 0.0f; }

struct HeuristicCost final : CostModel {
  // Roofline-style estimate from the features alone: a kernel occupies min(1, workgroups / CUs)
  // of the chip and runs at that share of the matrix-core or HBM peak, plus a fixed dispatch
  // latency; a copy runs at a host-link rate.  Each other stream in flight adds 15%.
  void predict_us(const float *feat, int64_t n, double *us) override {
    for (int64_t r = 0; r < n; ++r) {
      const float *f = feat + r * kFeatures;
      const double M = std::exp2(double(f[6])), N = std::exp2(double(f[7])), K = std::exp2(double(f[8]));
      const double bytes = std::exp2(double(f[9]));
      const bool bf16 = f[10] > 0.5f;
      double t;
      if (f[4] > 0.5f || f[5] > 0.5f) {
        t = 4.0 + bytes / 50.0e9 * 1e6;
      } else if (f[0] > 0.5f) {
        const double flops = 2.0 * M * N * K;
        const double peak = bf16 ? 1.2e15 : 9.0e13;
        const double tiles = std::ceil(M / 64.0) * std::ceil(N / 64.0);
        const double share = std::min(1.0, tiles / kCUs);
        t = 3.0 + std::max(flops / (peak * share), bytes / 4.0e12) * 1e6;
      } else {
        const double blocks = std::ceil(M * N / 4096.0);
        t = 3.0 + bytes / (4.0e12 * std::min(1.0, blocks / kCUs)) * 1e6;
      }
      us[r] = t * (1.0 + 0.15 * std::max(0.0f, f[11]));
    }
  }
};

// List scheduling on the cost model: kernels by descending bottom-level rank (ties: lower id),
// each placed on the stream where it can start first (ties: earliest predicted finish, then lower
// stream).  A kernel's duration on a candidate stream is
// the prediction for the number of other streams still busy at its start, so all predictions are
// made up front: one batch of feature rows, kernels x (0 .. S-1 streams in flight) plus the
// uploads of the isolated inputs.
void map_eft(const Dag &g, int32_t S, CostModel &cost, std::vector<int32_t> &order,
             std::vector<int32_t> &stream_of) {
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  const int32_t nb = static_cast<int32_t>(g.bufs.size());
  std::vector<float> feat(size_t(nk * S + nb) * kFeatures, 0.0f);
  for (int32_t k = 0; k < nk; ++k)
    for (int32_t j = 0; j < S; ++j) kernel_features(g, k, j, &feat[size_t(k * S + j) * kFeatures]);
  std::vector<char> is_h2d(nb, 0);
  for (int32_t b : g.h2d_bufs) is_h2d[b] = 1;
  for (int32_t b = 0; b < nb; ++b)
    if (is_h2d[b]) copy_features(g, b, true, 0, &feat[size_t(nk * S + b) * kFeatures]);
  std::vector<double> pred(size_t(nk * S + nb), 0.0);
  cost.predict_us(feat.data(), int64_t(pred.size()), pred.data());
  // a learned model can return non-finite or negative times (an untrained or corrupt network);
  // every comparison below would then fail silently, so the roofline heuristic takes over
  bool usable = true;
  for (double v : pred) usable = usable && std::isfinite(v) && v >= 0.0;
  if (!usable) make_heuristic_cost()->predict_us(feat.data(), int64_t(pred.size()), pred.data());
  auto w = [&](int32_t k, int32_t j) { return pred[size_t(k * S + std::min(j, S - 1))]; };
  auto up_us = [&](int32_t b) { return pred[size_t(nk * S + b)]; };
  // bottom-level rank over a reverse topological order, with the uncontended durations
  std::vector<int32_t> topo = g.bfs_order();
  std::vector<double> bl(nk, 0.0);
  for (auto it = topo.rbegin(); it != topo.rend(); ++it) {
    double m = 0;
    for (int32_t s : g.succ[*it]) m = std::max(m, bl[s]);
    bl[*it] = w(*it, 0) + m;
  }
  using Item = std::pair<double, int32_t>;  // (-rank, id)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> ready;
  std::vector<int32_t> indeg(nk);
  for (int32_t k = 0; k < nk; ++k) {
    indeg[k] = static_cast<int32_t>(g.pred[k].size());
    if (!indeg[k]) ready.push({-bl[k], k});
  }
  std::vector<double> avail(S, 0.0), finish(nk, 0.0);
  std::vector<char> uploaded(nb, 0);
  order.clear();
  while (!ready.empty()) {
    const int32_t k = ready.top().second;
    ready.pop();
    double dep_ready = 0;
    for (int32_t p : g.pred[k]) dep_ready = std::max(dep_ready, finish[p]);
    double up = 0;
    for (int32_t b : g.iso_in[k])
      if (!uploaded[b]) up += up_us(b);
    // the stream where the kernel can start first; among equal starts the earliest predicted
    // finish under the contention at that start.  (Comparing contended finish times alone is
    // myopic: a model that has learned how much a kernel stretches beside busy streams would
    // make every kernel wait for a free stream -- serialise -- without counting what waiting
    // costs the rest of the schedule.)  The chosen stream then stays busy for the contended time.
    int32_t best = 0;
    double best_st = 1e300, best_f = 1e300;
    for (int32_t s = 0; s < S; ++s) {
      const double st = std::max(avail[s] + up, dep_ready);
      int32_t busy = 0;
      for (int32_t q = 0; q < S; ++q) busy += q != s && avail[q] > st;
      const double f = st + w(k, busy);
      if (st < best_st - 1e-9 || (st < best_st + 1e-9 && f < best_f - 1e-9)) {
        best_st = st;
        best_f = f;
        best = s;
      }
    }
    for (int32_t b : g.iso_in[k]) uploaded[b] = 1;
    stream_of[k] = best;
    avail[best] = finish[k] = best_f;
    order.push_back(k);
    for (int32_t s : g.succ[k])
      if (--indeg[s] == 0) ready.push({-bl[s], s});
  }
}

}  // namespace

std::unique_ptr<CostModel> make_heuristic_cost() { return std::make_unique<HeuristicCost>(); }

void kernel_features(const Dag &g, int32_t kernel, int32_t in_flight, float *f) {
  const Kernel &ker = g.kers[kernel];
  const Buffer &o = g.bufs[ker.outs[0]];
  const Buffer &a = g.bufs[ker.ins[0]];
  for (int i = 0; i < kFeatures; ++i) f[i] = 0.0f;
  const int kind = ker.kind == PSC_GEMM ? 0 : ker.kind == PSC_TRANSPOSE ? 1 : ker.kind == PSC_SOFTMAX ? 2 : 3;
  f[kind] = 1.0f;
  f[6] = lg2(double(o.rows));
  f[7] = lg2(double(o.cols));
  f[8] = ker.kind == PSC_GEMM ? lg2(double(a.cols)) : 0.0f;
  double bytes = double(o.rows) * o.cols * elem_size(o.dtype);
  for (int32_t b : ker.ins) bytes += double(g.bufs[b].rows) * g.bufs[b].cols * elem_size(g.bufs[b].dtype);
  f[9] = lg2(bytes);
  f[10] = a.dtype == PSC_BF16 ? 1.0f : 0.0f;
  f[11] = float(in_flight);
}

void copy_features(const Dag &g, int32_t buffer, bool h2d, int32_t in_flight, float *f) {
  const Buffer &b = g.bufs[buffer];
  for (int i = 0; i < kFeatures; ++i) f[i] = 0.0f;
  f[h2d ? 4 : 5] = 1.0f;
  f[6] = lg2(double(b.rows));
  f[7] = lg2(double(b.cols));
  f[9] = lg2(double(b.rows) * b.cols * elem_size(b.dtype));
  f[10] = b.dtype == PSC_BF16 ? 1.0f : 0.0f;
  f[11] = float(in_flight);
}

// The buffer an isolated write is uploaded as: itself, or (copy_roots) its root when no kernel
// writes any part of that root, so one dense copy serves every window of it.
std::vector<int32_t> upload_buffers(const Dag &g, bool copy_roots) {
  std::vector<int32_t> as(g.bufs.size());
  for (size_t b = 0; b < g.bufs.size(); ++b) as[b] = int32_t(b);
  if (copy_roots) {
    std::vector<char> written(g.bufs.size(), 0);
    for (const Kernel &k : g.kers)
      for (int32_t b : k.outs) written[g.bufs[b].root] = 1;
    for (size_t b = 0; b < g.bufs.size(); ++b)
      if (!written[g.bufs[b].root]) as[b] = g.bufs[b].root;
  }
  return as;
}

namespace {

// PSC_DEVICE: every H2D first on queue 0, then each kernel on a queue of its own waiting for its
// predecessor kernels and its inputs' H2D, then every D2H on queue 0 waiting for its producer.
SchedPlan build_device_plan(const Dag &g, bool copy_roots) {
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  const std::vector<int32_t> upload_as = upload_buffers(g, copy_roots);
  SchedPlan plan;
  plan.device = true;
  plan.n_streams = plan.total_streams = 1 + nk;
  const std::vector<int32_t> order = g.bfs_order();
  std::vector<int32_t> h2d_op(g.bufs.size(), -1);
  int32_t pos0 = 0;
  auto emit = [&](int32_t type, int32_t kernel, int32_t buffer, int32_t stream, int32_t pos,
                  std::vector<int32_t> waits) {
    Op op;
    op.type = type;
    op.kernel = kernel;
    op.buffer = buffer;
    op.stream = stream;
    op.pos = pos;
    op.host_order = static_cast<int32_t>(plan.ops.size());
    std::sort(waits.begin(), waits.end());
    waits.erase(std::unique(waits.begin(), waits.end()), waits.end());
    for (int32_t w : waits) plan.ops[w].recorded = true;
    op.waits = std::move(waits);
    plan.ops.push_back(std::move(op));
    return static_cast<int32_t>(plan.ops.size() - 1);
  };
  for (int32_t k : order)
    for (int32_t b : g.iso_in[k])
      if (h2d_op[upload_as[b]] < 0) h2d_op[upload_as[b]] = emit(PSC_OP_H2D, -1, upload_as[b], 0, pos0++, {});
  plan.kernel_op.assign(nk, -1);
  for (int32_t k : order) {
    std::vector<int32_t> w;
    for (int32_t p : g.pred[k]) w.push_back(plan.kernel_op[p]);
    for (int32_t b : g.iso_in[k]) w.push_back(h2d_op[upload_as[b]]);
    plan.kernel_op[k] = emit(PSC_OP_KERNEL, k, -1, 1 + k, 0, w);
  }
  for (int32_t k : order)
    for (int32_t b : g.iso_out[k]) emit(PSC_OP_D2H, -1, b, 0, pos0++, {plan.kernel_op[k]});
  return plan;
}

}  // namespace

// PSC_EAGER / PSC_HEFT (the dynamic coarse-grained baselines of Sec. V, Experiments 2 and 3):
// every kernel its own task component.  The op list is the coarse one (each kernel with its
// uploads before and its read-backs after it); which stream -- device queue -- runs it, and when,
// is decided at run time.  Here: predicted durations and the bottom-level ranks that order the
// ready queue.
SchedPlan build_dynamic_plan(const Dag &g, int policy, const psc_sched_opts &o) {
  psc_sched_opts one = o;
  one.copy_stream = 0;
  SchedPlan plan = build_plan(g, PSC_COARSE, one);
  plan.dynamic = true;
  plan.heft = policy == PSC_HEFT;
  plan.n_streams = plan.total_streams = o.n_streams;
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  std::vector<float> feat(size_t(std::max(1, nk)) * kFeatures, 0.0f);
  for (int32_t k = 0; k < nk; ++k) kernel_features(g, k, 0, &feat[size_t(k) * kFeatures]);
  plan.dyn_us.assign(nk, 0.0);
  auto cost = o.cost ? mlp_cost_model(o.cost) : make_heuristic_cost();
  if (nk) cost->predict_us(feat.data(), nk, plan.dyn_us.data());
  bool usable = true;
  for (double v : plan.dyn_us) usable = usable && std::isfinite(v) && v >= 0.0;
  if (!usable && nk) make_heuristic_cost()->predict_us(feat.data(), nk, plan.dyn_us.data());
  plan.dyn_rank.assign(nk, 0.0);
  const std::vector<int32_t> topo = g.bfs_order();
  for (auto it = topo.rbegin(); it != topo.rend(); ++it) {
    double m = 0;
    for (int32_t q : g.succ[*it]) m = std::max(m, plan.dyn_rank[q]);
    plan.dyn_rank[*it] = plan.dyn_us[*it] + m;
  }
  return plan;
}

SchedPlan build_plan(const Dag &g, int policy, const psc_sched_opts &o) {
  if (policy == PSC_DEVICE) return build_device_plan(g, o.copy_roots != 0);
  if (policy == PSC_EAGER || policy == PSC_HEFT) return build_dynamic_plan(g, policy, o);
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  SchedPlan plan;
  const int32_t S = policy == PSC_COARSE ? 1 : o.n_streams;
  plan.n_streams = S;
  const bool cs = policy != PSC_COARSE && o.copy_stream;
  bool any_d2h = false;
  for (const auto &v : g.iso_out) any_d2h = any_d2h || !v.empty();
  // with copy streams: uploads on stream S, read-backs on stream S + 1 (the two directions use
  // different DMA engines, and a read-back never holds up a later kernel of its producer's stream)
  const int32_t copy_s = cs ? S : -1;
  const int32_t read_s = cs && any_d2h ? S + 1 : -1;
  plan.total_streams = S + (cs ? 1 : 0) + (read_s >= 0 ? 1 : 0);

  std::vector<int32_t> order, stream_of(nk, 0);
  if (policy == PSC_COARSE) {
    order = g.bfs_order();
  } else if (o.mapper == PSC_MAP_RR) {
    order = g.bfs_order();
    for (int32_t i = 0; i < nk; ++i) stream_of[order[i]] = i % S;
  } else if (o.mapper == PSC_MAP_COMPONENT) {
    order = g.bfs_order();
    for (int32_t k = 0; k < nk; ++k) stream_of[k] = g.kers[k].component % S;
  } else if (o.mapper == PSC_MAP_EFT) {
    auto cost = o.cost ? mlp_cost_model(o.cost) : make_heuristic_cost();
    map_eft(g, S, *cost, order, stream_of);
  } else {
    fail(PSC_ERR_ARG, "unknown mapper");
  }

  // out-of-order queues: kernels by DAG level (longest path from a root), the mapper's order
  // within a level, so that a queue's wait for one kernel's producers holds back only kernels of
  // later levels -- every kernel of a level can be in flight together
  const bool ooo = policy == PSC_FINE && o.out_of_order;
  plan.out_of_order = ooo;
  if (ooo) {
    std::vector<int32_t> level(nk, 0);
    for (int32_t k : g.bfs_order())
      for (int32_t q : g.succ[k]) level[q] = std::max(level[q], level[k] + 1);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return level[a] < level[b]; });
  }

  const std::vector<int32_t> upload_as = upload_buffers(g, o.copy_roots != 0);

  // emit ops with their dependencies (ids of earlier ops)
  std::vector<std::vector<int32_t>> deps;
  std::vector<int32_t> h2d_op(g.bufs.size(), -1);
  plan.kernel_op.assign(nk, -1);
  std::vector<int32_t> pos(plan.total_streams, 0);
  auto emit = [&](int32_t type, int32_t kernel, int32_t buffer, int32_t stream,
                  std::vector<int32_t> d) {
    Op op;
    op.type = type;
    op.kernel = kernel;
    op.buffer = buffer;
    op.stream = stream;
    op.pos = pos[stream]++;
    op.host_order = static_cast<int32_t>(plan.ops.size());
    plan.ops.push_back(std::move(op));
    deps.push_back(std::move(d));
    return static_cast<int32_t>(plan.ops.size() - 1);
  };
  if (cs)
    for (int32_t k : order)
      for (int32_t b : g.iso_in[k])
        if (h2d_op[upload_as[b]] < 0) h2d_op[upload_as[b]] = emit(PSC_OP_H2D, -1, upload_as[b], copy_s, {});
  for (int32_t k : order) {
    const int32_t s = stream_of[k];
    if (!cs)
      for (int32_t b : g.iso_in[k])
        if (h2d_op[upload_as[b]] < 0) h2d_op[upload_as[b]] = emit(PSC_OP_H2D, -1, upload_as[b], s, {});
    std::vector<int32_t> d;
    for (int32_t p : g.pred[k]) d.push_back(plan.kernel_op[p]);
    for (int32_t b : g.iso_in[k]) d.push_back(h2d_op[upload_as[b]]);
    const int32_t kop = emit(PSC_OP_KERNEL, k, -1, s, d);
    plan.kernel_op[k] = kop;
    for (int32_t b : g.iso_out[k]) emit(PSC_OP_D2H, -1, b, read_s >= 0 ? read_s : s, {kop});
  }

  const int32_t T = plan.total_streams;
  const size_t n = plan.ops.size();
  if (ooo) {
    // stream order implies nothing: every direct precedence is a wait
    for (size_t i = 0; i < n; ++i) {
      std::vector<int32_t> d = deps[i];
      std::sort(d.begin(), d.end());
      d.erase(std::unique(d.begin(), d.end()), d.end());
      for (int32_t dep : d) plan.ops[dep].recorded = true;
      plan.ops[i].waits = std::move(d);
    }
    return plan;
  }
  // waits: vector clocks over streams; vc[i][t] = last position on stream t known to precede op i
  std::vector<int32_t> vc(n * T, -1);
  std::vector<int32_t> last_on(T, -1);
  std::vector<int32_t> cur(T);
  for (size_t i = 0; i < n; ++i) {
    Op &op = plan.ops[i];
    const int32_t prev = last_on[op.stream];
    if (prev >= 0)
      std::copy(vc.begin() + prev * T, vc.begin() + (prev + 1) * T, cur.begin());
    else
      std::fill(cur.begin(), cur.end(), -1);
    std::vector<int32_t> d = deps[i];
    std::sort(d.begin(), d.end(), std::greater<int32_t>());  // later ops first
    d.erase(std::unique(d.begin(), d.end()), d.end());
    for (int32_t dep : d) {
      const Op &p = plan.ops[dep];
      if (p.stream == op.stream) continue;  // stream order covers it
      if (cur[p.stream] >= p.pos) continue;  // implied by an earlier wait
      op.waits.push_back(dep);
      plan.ops[dep].recorded = true;
      for (int32_t t = 0; t < T; ++t) cur[t] = std::max(cur[t], vc[dep * T + t]);
    }
    std::sort(op.waits.begin(), op.waits.end());
    cur[op.stream] = op.pos;
    std::copy(cur.begin(), cur.end(), vc.begin() + i * T);
    last_on[op.stream] = static_cast<int32_t>(i);
  }
  return plan;
}

}  // namespace psc
