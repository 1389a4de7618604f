// Stream/event dispatcher (the dispatch step of Algorithm 1, Sec. IV-B) on HIP.
//
// prepare(): one device arena for every unbound root buffer, the schedule's streams (default
// priority, non-blocking), one event per op that another stream waits for, and a prepared launch
// per kernel.  run(): record a start event, make every stream wait for it, enqueue the ops in host
// order -- each wait is a hipStreamWaitEvent on the producing op's event, which HIP requires to
// have been recorded (enqueued) earlier, so host order is topological -- then join every stream
// into stream 0, record the end event and wait for it.  In graph mode the same enqueue sequence
// is built once as an explicit hipGraph (a node per op, an edge per precedence) and replayed with
// one hipGraphLaunch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstring>
#include <queue>
#include <string>

#include "aql.hpp"
#include "core.hpp"
#include "dispatch.hpp"
#include "kernels.hpp"
#include "persistent.hpp"

namespace psc {

#define PSC_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) fail(PSC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct CopyDesc {  // one resolved host copy
  bool active = false;
  void *dst = nullptr;
  const void *src = nullptr;
  size_t dpitch = 0, spitch = 0, width = 0, height = 0;
  hipMemcpyKind kind = hipMemcpyHostToDevice;
};

// State the dynamic schedulers share with their completion callbacks (Algorithm 1's F, A and the
// finished-kernel status), guarded by one lock.
struct DynState {
  std::mutex mu;
  std::condition_variable cv;
  const Dag *g = nullptr;
  const SchedPlan *plan = nullptr;
  std::vector<int32_t> indeg;                   // unfinished predecessors per kernel
  std::vector<std::pair<double, int32_t>> heap;  // ready kernels: (rank, -kernel), a max-heap
  std::vector<char> available;                  // per stream (device queue)
  int32_t finished = 0;
  uint64_t updates = 0;                          // callbacks seen
  struct Arg {
    DynState *st;
    int32_t kernel, stream;
  };
  std::vector<Arg> args;                         // per kernel, the callback's user argument

  void push_ready(int32_t k) {
    heap.push_back({plan->dyn_rank[k], -k});
    std::push_heap(heap.begin(), heap.end());
  }
};

// cb of Algorithm 1: the kernel finished (its stream reached the callback); its successors whose
// predecessors have all finished join the ready queue and its stream is available again.  Runs on
// the HIP runtime's callback thread and makes no HIP call.
void dyn_callback(void *p) {
  auto *a = static_cast<DynState::Arg *>(p);
  DynState &st = *a->st;
  {
    std::lock_guard<std::mutex> lk(st.mu);
    for (int32_t q : st.g->succ[a->kernel])
      if (--st.indeg[q] == 0) st.push_ready(q);
    st.available[a->stream] = 1;
    ++st.finished;
    ++st.updates;
  }
  st.cv.notify_one();
}

// The host copies of a PSC_DEVICE plan the executor runs as nodes of its own (after the
// kernels: node n_kernels + i), in plan op order: each isolated upload, with the kernels that
// wait for it, and each read-back, with the kernel that produces it.
struct ExecCopy {
  int32_t op = -1, buffer = -1;
  bool h2d = true;
  std::vector<int32_t> kernels;
  int32_t rows = 0, rows_per_task = 1;
  int64_t width = 0;  // bytes per row
};

struct Device {
  int device = 0;
  void *arena = nullptr;
  std::vector<char *> base;  // per buffer id (roots only): device storage
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> op_ev;
  std::vector<hipEvent_t> join_ev;
  hipEvent_t start = nullptr, end = nullptr;
  bool in_flight = false;          // a timed-out run may still execute (wait for `end` first)
  std::vector<hipEvent_t> t0, t1;  // per-op timing (record_ops)
  std::vector<Launch> launch;      // per kernel id
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void *> graph_key;
  std::vector<psc_op_time> times;
  std::vector<char> active;        // per op in the recorded run: it did work
  bool have_times = false;
  // component completion marks (mark_components): slot k = after END kernel k, slot nk = start
  uint64_t *marks = nullptr;
  Launch mark_start;
  std::vector<Launch> mark_after;  // per kernel; .func == nullptr unless an END kernel
  bool have_marks = false;
  std::unique_ptr<Dispatcher> disp;
  std::unique_ptr<AqlSchedule> aql;  // PSC_DISPATCH_AQL: queues, signals, argument records
  std::unique_ptr<struct DynState> dyn;  // PSC_EAGER / PSC_HEFT: the run-time scheduler's state
  // PSC_DEVICE executor
  void *exec_mem = nullptr;
  ExecArgs ea{};
  int exec_instance = 0;       // compiled executor instance (tile-function groups) for this DAG
  void *exec_mem_copy = nullptr;      // the plan with the host copies (ea_copy)
  ExecArgs ea_copy{};
  const ExecArgs *ea_run = &ea;       // the plan the last run used
  std::vector<ExecCopy> exec_copies;  // host copies run as executor nodes (after the kernels)
  std::vector<char> exec_dma;         // per plan op: this run copied it by DMA instead
  ExecNode *h_copy_nodes = nullptr;   // page-locked: their records, rewritten before every run
  uint32_t *h_err = nullptr;  // page-locked word receiving the executor's error flag
  double clock_mhz = 100.0;   // device wall clock rate

  ~Device() {
    if (in_flight && end) (void)hipEventSynchronize(end);  // a timed-out run still executing
    aql.reset();                                           // (waits for its own run the same way)
    disp.reset();
    if (exec_mem) (void)hipFree(exec_mem);
    if (exec_mem_copy) (void)hipFree(exec_mem_copy);
    if (marks) (void)hipFree(marks);
    if (h_err) (void)hipHostFree(h_err);
    if (h_copy_nodes) (void)hipHostFree(h_copy_nodes);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : op_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : join_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : t0)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : t1)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {start, end})
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : streams)
      if (s) (void)hipStreamDestroy(s);
    if (arena) (void)hipFree(arena);
  }
};

namespace {

char *buffer_ptr(const Dag &g, const Device &d, int32_t b) {
  const Buffer &x = g.bufs[b];
  const Buffer &r = g.bufs[x.root];
  return d.base[x.root] + (x.r0 * r.cols + x.c0) * elem_size(r.dtype);
}
int64_t buffer_ld(const Dag &g, int32_t b) { return g.bufs[g.bufs[b].root].cols; }

void build_launch(const Dag &g, const Device &d, int32_t k, Launch &L) {
  const Kernel &ker = g.kers[k];
  auto P = [&](int32_t b) { return buffer_ptr(g, d, b); };
  auto LD = [&](int32_t b) { return buffer_ld(g, b); };
  bool ok = false;
  switch (ker.kind) {
    case PSC_GEMM: {
      const Buffer &a = g.bufs[ker.ins[0]], &b = g.bufs[ker.ins[1]], &c = g.bufs[ker.outs[0]];
      GemmArgs ga{};
      ga.A = P(ker.ins[0]);
      ga.B = P(ker.ins[1]);
      ga.C = P(ker.outs[0]);
      ga.lda = LD(ker.ins[0]);
      ga.ldb = LD(ker.ins[1]);
      ga.ldc = LD(ker.outs[0]);
      ga.M = int32_t(a.rows);
      ga.N = int32_t(b.cols);
      ga.K = int32_t(a.cols);
      ga.alpha = ker.alpha;
      ok = make_gemm(L, ga, a.dtype, c.dtype, ker.tile);
      break;
    }
    case PSC_SOFTMAX: {
      const Buffer &x = g.bufs[ker.ins[0]], &y = g.bufs[ker.outs[0]];
      SoftmaxArgs sa{P(ker.ins[0]), P(ker.outs[0]), LD(ker.ins[0]), LD(ker.outs[0]), int32_t(x.rows), int32_t(x.cols)};
      ok = make_softmax(L, sa, x.dtype, y.dtype);
      break;
    }
    case PSC_TRANSPOSE: {
      const Buffer &x = g.bufs[ker.ins[0]];
      TransArgs ta{P(ker.ins[0]), P(ker.outs[0]), LD(ker.ins[0]), LD(ker.outs[0]), int32_t(x.rows), int32_t(x.cols)};
      ok = make_transpose(L, ta, x.dtype, ker.tile);
      break;
    }
    case PSC_ADD: {
      const Buffer &x = g.bufs[ker.ins[0]], &c = g.bufs[ker.outs[0]];
      AddArgs aa{P(ker.ins[0]), P(ker.ins[1]), P(ker.outs[0]), LD(ker.ins[0]), LD(ker.ins[1]), LD(ker.outs[0]),
                 int32_t(x.rows), int32_t(x.cols)};
      ok = make_add(L, aa, x.dtype, c.dtype);
      break;
    }
  }
  if (!ok) fail(PSC_ERR_UNSUPPORTED, "no kernel instance for '" + ker.name + "'");
}

void launch(const Launch &L, hipStream_t s) {
  if (L.empty) return;
  void *args[] = {const_cast<unsigned char *>(L.args)};
  PSC_HIP(hipLaunchKernel(L.func, L.grid, L.block, args, L.shmem, s));
}

}  // namespace

namespace {

int in_dtype_of(const Dag &g, const Kernel &k) { return g.bufs[k.ins[0]].dtype; }

// Predicted duration of one executor task (microseconds) for the host's list schedule: a CU's
// share of the matrix-core peak (at half efficiency) or of the memory bandwidth, plus a fixed
// per-task overhead.
double exec_task_us(const Dag &g, const Kernel &ker, const ExecNode &nd) {
  constexpr double kOverhead = 0.6, kCuBw = 40e9;
  if (nd.variant == 0) return 0.1;
  const Buffer &a = g.bufs[ker.ins[0]], &o = g.bufs[ker.outs[0]];
  const double ea = double(elem_size(a.dtype)), eo = double(elem_size(o.dtype));
  if (ker.kind == PSC_GEMM) {
    const double K = double(a.cols), bm = nd.tile_m, bn = nd.tile_n;
    const double flops = 2.0 * bm * bn * K;
    const double cu_flops = (a.dtype == PSC_BF16 ? 2.5e15 : 157.3e12) / 256.0 * 0.5;
    const double bytes = (bm * K + K * bn) * ea + bm * bn * eo;
    // GEMM tasks measured about twice this roofline figure inside the executor (one workgroup per
    // CU, no other wavefronts to hide their memory latency); with the factor the attention DAG's
    // makespan is 9% shorter (x3 and x4 were worse than x2)
    return kOverhead + 2.0 * std::max(flops / cu_flops, bytes / kCuBw) * 1e6;
  }
  const double elems = double(nd.tile_m) * double(nd.tile_n);
  const double per = ker.kind == PSC_ADD ? 2.0 * ea + eo : ea + eo;
  return kOverhead + elems * per / kCuBw * 1e6;
}

// The executor's plan: node descriptions, predecessor lists and the per-workgroup task lists (a
// list schedule: kernels in descending bottom-level order among those whose predecessors are
// placed, each task on the workgroup predicted to be free first).  Host only.
struct ExecPlan {
  std::vector<ExecNode> nodes;
  std::vector<int32_t> pred;
  std::vector<ExecTask> tasks;
  std::vector<int32_t> work_off;
};

// The executor's node descriptions when tiles are sized for `tile_workers` workgroups: each
// kernel's tile is chosen for the workgroups it can expect, half of them divided by the kernels
// at its depth (the longest path from a root) -- kernels of neighbouring depths run side by side
// in the list schedule, so a depth's kernels seldom have all workgroups to themselves (measured
// on the 512 attention DAG: 0.110 ms against 0.116-0.119 with all of them and 0.128 with a
// quarter).  A run holding more than one workgroup per CU sizes them for one per CU: the second
// workgroup hides the first's latency rather than adding CUs to split a kernel over (measured:
// 8-10% shorter on the 512 attention DAG at two per CU, ~2% on the 12-layer DAG, the same at one
// per CU).
std::vector<ExecNode> exec_nodes(const Dag &g, const std::vector<Launch> &launch, int32_t tile_workers) {
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  std::vector<ExecNode> nodes(nk);
  std::vector<int32_t> depth(nk, 0), width;
  for (int32_t k : g.bfs_order())
    for (int32_t q : g.succ[k]) depth[q] = std::max(depth[q], depth[k] + 1);
  for (int32_t k = 0; k < nk; ++k) {
    if (depth[k] >= int32_t(width.size())) width.resize(depth[k] + 1, 0);
    ++width[depth[k]];
  }
  const int32_t Wmax = std::max(1, tile_workers / 2);
  for (int32_t k = 0; k < nk; ++k) {
    const Kernel &ker = g.kers[k];
    const int want = std::max(1, Wmax / std::max(1, width[depth[k]]));
    nodes[k] = make_exec_node(ker.kind, launch[k].args, in_dtype_of(g, ker), g.bufs[ker.outs[0]].dtype,
                              launch[k].tile, want);
  }
  return nodes;
}

std::vector<ExecCopy> exec_copies(const Dag &g, const SchedPlan &plan) {
  std::vector<ExecCopy> c;
  std::vector<int32_t> idx(plan.ops.size(), -1);
  for (size_t o = 0; o < plan.ops.size(); ++o) {
    const Op &op = plan.ops[o];
    if (op.type == PSC_OP_KERNEL) continue;
    idx[o] = static_cast<int32_t>(c.size());
    ExecCopy x;
    x.op = static_cast<int32_t>(o);
    x.buffer = op.buffer;
    x.h2d = op.type == PSC_OP_H2D;
    const Buffer &b = g.bufs[op.buffer];
    x.rows = b.rows;
    x.width = int64_t(b.cols) * elem_size(b.dtype);
    // tasks of about 64 KiB
    x.rows_per_task = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(b.rows, 65536 / std::max<int64_t>(1, x.width))));
    c.push_back(std::move(x));
  }
  for (size_t o = 0; o < plan.ops.size(); ++o) {
    const Op &op = plan.ops[o];
    for (int32_t w : op.waits) {
      if (op.type == PSC_OP_KERNEL && idx[w] >= 0 && c[idx[w]].h2d) c[idx[w]].kernels.push_back(op.kernel);
      if (op.type == PSC_OP_D2H && plan.ops[w].type == PSC_OP_KERNEL) c[idx[o]].kernels.push_back(plan.ops[w].kernel);
    }
  }
  return c;
}

// Copy tasks run on at most this many workgroups of their own (W / 16 of the grid).
constexpr int32_t kCopyWorkers = 32;

ExecNode make_copy_node(const ExecCopy &x) {
  ExecNode n{};
  if (x.rows == 0 || x.width == 0) {
    n.variant = 0;
    n.n_tiles = 1;
    return n;
  }
  n.variant = kCopyVariant;
  n.n_tiles = (x.rows + x.rows_per_task - 1) / x.rows_per_task;
  n.tile_m = x.rows_per_task;
  n.tile_n = static_cast<int32_t>(std::min<int64_t>(x.width, INT32_MAX));
  return n;
}

// List schedule of the kernels' tiles onto W workgroups (lists[0 .. W)): kernels in descending
// bottom-level order among those whose predecessors are placed, each tile on the workgroup
// predicted to finish it first.  Returns every kernel's bottom level.
std::vector<double> schedule_kernels(const Dag &g, const std::vector<ExecNode> &nodes, int32_t W,
                                     std::vector<std::vector<ExecTask>> &lists) {
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  std::vector<double> cost(nk), bl(nk, 0.0), finish(nk, 0.0);
  for (int32_t k = 0; k < nk; ++k) cost[k] = exec_task_us(g, g.kers[k], nodes[k]);
  const std::vector<int32_t> topo = g.bfs_order();
  for (auto it = topo.rbegin(); it != topo.rend(); ++it) {
    double m = 0;
    for (int32_t q : g.succ[*it]) m = std::max(m, bl[q]);
    bl[*it] = cost[*it] * std::ceil(double(nodes[*it].n_tiles) / W) + m;
  }
  using Item = std::pair<double, int32_t>;  // (-rank, kernel)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> ready;
  std::vector<int32_t> indeg(nk);
  for (int32_t k = 0; k < nk; ++k)
    if (!(indeg[k] = static_cast<int32_t>(g.pred[k].size()))) ready.push({-bl[k], k});
  // Tiles are placed one at a time on the workgroup predicted to finish them first.  A tile that
  // continues its kernel's run on a workgroup costs its compute only; starting a kernel on a
  // workgroup also costs publishing the run (a release, ~2 us) and, for a kernel with
  // predecessors, the acquire (~2 us).  A kernel may use at most W / (kernels ready when it is
  // placed) workgroups, so kernels that could run side by side (the heads of an attention layer,
  // the instances of a batch) share the GPU instead of each spreading over all of it and paying
  // a fence pair on every workgroup.
  constexpr double kRelease = 2.1, kAcquire = 1.8;
  std::vector<double> free_time(W, 0.0);
  using Free = std::pair<double, int32_t>;  // (time the workgroup is free, workgroup); lazy entries
  std::priority_queue<Free, std::vector<Free>, std::greater<Free>> free_at;
  for (int32_t w = 0; w < W; ++w) free_at.push({0.0, w});
  std::vector<int32_t> used;
  while (!ready.empty()) {
    const int32_t k = ready.top().second;
    const int32_t cap = std::max<int32_t>(1, (W + int32_t(ready.size()) - 1) / int32_t(ready.size()));
    ready.pop();
    double rt = 0;
    for (int32_t p : g.pred[k]) rt = std::max(rt, finish[p]);
    const double sw = kRelease + (g.pred[k].empty() ? 0.0 : kAcquire);
    used.clear();
    for (int32_t t = 0; t < nodes[k].n_tiles; ++t) {
      // continue on the earliest-free workgroup already running this kernel ...
      int32_t wc = -1;
      for (int32_t w : used)
        if (wc < 0 || free_time[w] < free_time[wc]) wc = w;
      double end_c = wc >= 0 ? std::max(free_time[wc], rt) + cost[k] : 1e300;
      // ... or start on the earliest-free workgroup, while under the cap
      int32_t wn = -1;
      double end_n = 1e300;
      if (int32_t(used.size()) < cap) {
        while (free_at.top().first != free_time[free_at.top().second]) free_at.pop();  // stale
        wn = free_at.top().second;
        end_n = std::max(free_time[wn], rt) + sw + cost[k];
      }
      const bool cont = end_c <= end_n;
      const int32_t w = cont ? wc : wn;
      const double end = cont ? end_c : end_n;
      if (!cont) used.push_back(w);
      free_time[w] = end;
      free_at.push({end, w});
      finish[k] = std::max(finish[k], end);
      lists[w].push_back(ExecTask{k, t, 0, 0});
    }
    for (int32_t q : g.succ[k])
      if (--indeg[q] == 0) ready.push({-bl[q], q});
  }
  return bl;
}

// The executor's plan: node descriptions, predecessor lists and the per-workgroup task lists.
// Without copies: the kernels' list schedule on every workgroup.  With copies (the executor
// runs the uploads and read-backs itself): the last CW = W / 16 (at most 32) workgroups run
// only copy tasks -- every upload, the first needed first (by its readers' bottom level), then
// every read-back -- dealt round robin, while the others run the kernels' list schedule; a
// kernel also waits for its inputs' uploads, a read-back for its writer.  Each list is a
// subsequence of one order in which every task comes after its predecessors' (uploads, kernels
// in placement order, read-backs), so with all workgroups resident every wait ends.  Host only.
ExecPlan plan_executor(const Dag &g, const std::vector<Launch> &launch, int32_t max_workers,
                       int32_t tile_workers, const std::vector<ExecCopy> &copies) {
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  const int32_t nc = static_cast<int32_t>(copies.size());
  ExecPlan ep;
  ep.nodes = exec_nodes(g, launch, tile_workers);
  std::vector<std::vector<int32_t>> P(nk);
  for (int32_t k = 0; k < nk; ++k) P[k] = g.pred[k];
  for (int32_t c = 0; c < nc; ++c) {
    ep.nodes.push_back(make_copy_node(copies[c]));
    P.emplace_back();
    for (int32_t k : copies[c].kernels) {
      if (copies[c].h2d) P[k].push_back(nk + c);
      else P[nk + c].push_back(k);
    }
  }
  uint64_t total = 0;
  for (size_t v = 0; v < ep.nodes.size(); ++v) {
    ep.nodes[v].n_pred = static_cast<int32_t>(P[v].size());
    ep.nodes[v].pred_off = static_cast<int32_t>(ep.pred.size());
    ep.pred.insert(ep.pred.end(), P[v].begin(), P[v].end());
    total += uint64_t(ep.nodes[v].n_tiles);
  }
  if (total >= (uint64_t(1) << 31)) fail(PSC_ERR_UNSUPPORTED, "too many executor tasks");
  const int32_t W = static_cast<int32_t>(std::max<uint64_t>(1, std::min<uint64_t>(total, uint64_t(std::max(1, max_workers)))));
  const int32_t CW = nc == 0 || W < 2 ? 0 : std::min(kCopyWorkers, std::max(1, W / 16));
  const int32_t WK = W - CW;  // workgroups running kernels
  std::vector<std::vector<ExecTask>> lists(W);
  const std::vector<double> bl = schedule_kernels(g, ep.nodes, WK, lists);
  if (nc) {
    std::vector<int32_t> ups, downs;
    std::vector<double> pri(nc, 0.0);
    for (int32_t c = 0; c < nc; ++c) {
      (copies[c].h2d ? ups : downs).push_back(c);
      for (int32_t k : copies[c].kernels) pri[c] = std::max(pri[c], bl[k]);
    }
    std::stable_sort(ups.begin(), ups.end(), [&](int32_t x, int32_t y) { return pri[x] > pri[y]; });
    std::stable_sort(downs.begin(), downs.end(), [&](int32_t x, int32_t y) { return pri[x] > pri[y]; });
    std::vector<ExecTask> seq;
    for (int32_t c : ups)
      for (int32_t t = 0; t < ep.nodes[nk + c].n_tiles; ++t) seq.push_back(ExecTask{nk + c, t, 0, 0});
    const size_t n_up = seq.size();
    for (int32_t c : downs)
      for (int32_t t = 0; t < ep.nodes[nk + c].n_tiles; ++t) seq.push_back(ExecTask{nk + c, t, 0, 0});
    if (CW > 0) {
      for (size_t i = 0; i < seq.size(); ++i) lists[WK + int32_t(i % CW)].push_back(seq[i]);
    } else {  // one workgroup: uploads, kernels, read-backs
      std::vector<ExecTask> one(seq.begin(), seq.begin() + n_up);
      one.insert(one.end(), lists[0].begin(), lists[0].end());
      one.insert(one.end(), seq.begin() + n_up, seq.end());
      lists[0] = std::move(one);
    }
  }
  ep.work_off.assign(W + 1, 0);
  ep.tasks.reserve(total);
  for (int32_t w = 0; w < W; ++w) {
    auto &L = lists[w];
    int32_t run = 0;
    for (size_t i = 0; i < L.size(); ++i) {  // publish at the end of each run of one node's tiles
      run = (i > 0 && L[i - 1].node == L[i].node) ? run + 1 : 1;
      if (i + 1 == L.size() || L[i + 1].node != L[i].node) L[i].signal = run;
    }
    ep.tasks.insert(ep.tasks.end(), L.begin(), L.end());
    ep.work_off[w + 1] = static_cast<int32_t>(ep.tasks.size());
  }
  return ep;
}

// The executor instance for a DAG: among the compiled instances with at most per_cu_cap
// workgroups per CU (0: any), by decreasing resident workgroups, the first whose tile-function
// groups cover every node variant the DAG gets at that worker count (the tile choice depends on
// the worker count, capped at one per CU: *tile_workers); the last instance covers all.
int pick_exec_instance(const Dag &g, const std::vector<Launch> &launch, int device, int32_t per_cu_cap,
                       int32_t *workers, int32_t *tile_workers) {
  const int n = exec_num_instances();
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  std::vector<std::pair<int32_t, int>> cand;  // (-workers, instance): more workers first, then order
  for (int i = 0; i < n; ++i) {
    const int32_t w = exec_max_workers(device, i);
    if (per_cu_cap > 0 && w > per_cu_cap * cus && i != n - 1) continue;
    cand.push_back({-(per_cu_cap > 0 ? std::min(w, per_cu_cap * cus) : w), i});
  }
  std::sort(cand.begin(), cand.end());
  for (const auto &c : cand) {
    uint32_t need = 0;
    for (const ExecNode &nd : exec_nodes(g, launch, std::min(-c.first, cus))) need |= exec_variant_group(nd.variant);
    if ((need & ~exec_instance_groups(c.second)) == 0) {
      *workers = -c.first;
      *tile_workers = std::min(*workers, cus);
      return c.second;
    }
  }
  *workers = exec_max_workers(device, n - 1);
  if (per_cu_cap > 0) *workers = std::min(*workers, per_cu_cap * cus);
  *tile_workers = std::min(*workers, cus);
  return n - 1;
}

// One executor plan in device memory (its own allocation, freed with the schedule).
void upload_exec_plan(const ExecPlan &ep, Device &d, void *&mem, ExecArgs &a) {
  const int32_t nn = static_cast<int32_t>(ep.nodes.size());
  const int32_t W = static_cast<int32_t>(ep.work_off.size()) - 1;
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_nodes = 0, o_pred = o_nodes + up(sizeof(ExecNode) * std::max(1, nn));
  const size_t o_tasks = o_pred + up(4 * std::max<size_t>(1, ep.pred.size()));
  const size_t o_off = o_tasks + up(sizeof(ExecTask) * std::max<size_t>(1, ep.tasks.size()));
  const size_t o_done = o_off + up(4 * size_t(W + 1));
  const size_t o_ctl = o_done + up(4 * std::max(1, nn));
  const size_t o_tf = o_ctl + 256;
  const size_t o_tl = o_tf + up(8 * std::max(1, nn));
  const size_t o_ts = o_tl + up(8 * std::max(1, nn));
  const size_t bytes = o_ts + 256;
  hipError_t e = hipMalloc(&mem, bytes);
  if (e != hipSuccess) fail(PSC_ERR_OOM, std::string("hipMalloc (executor state): ") + hipGetErrorString(e));
  char *base = static_cast<char *>(mem);
  PSC_HIP(hipMemcpy(base + o_nodes, ep.nodes.data(), sizeof(ExecNode) * nn, hipMemcpyHostToDevice));
  if (!ep.pred.empty()) PSC_HIP(hipMemcpy(base + o_pred, ep.pred.data(), 4 * ep.pred.size(), hipMemcpyHostToDevice));
  PSC_HIP(hipMemcpy(base + o_tasks, ep.tasks.data(), sizeof(ExecTask) * ep.tasks.size(), hipMemcpyHostToDevice));
  PSC_HIP(hipMemcpy(base + o_off, ep.work_off.data(), 4 * ep.work_off.size(), hipMemcpyHostToDevice));
  a.nodes = reinterpret_cast<const ExecNode *>(base + o_nodes);
  a.pred = reinterpret_cast<const int32_t *>(base + o_pred);
  a.tasks = reinterpret_cast<const ExecTask *>(base + o_tasks);
  a.work_off = reinterpret_cast<const int32_t *>(base + o_off);
  a.done = reinterpret_cast<uint32_t *>(base + o_done);
  a.ctl = reinterpret_cast<uint32_t *>(base + o_ctl);
  a.t_first = reinterpret_cast<uint64_t *>(base + o_tf);
  a.t_last = reinterpret_cast<uint64_t *>(base + o_tl);
  a.t_start = reinterpret_cast<uint64_t *>(base + o_ts);
  a.n_nodes = nn;
  a.n_workers = W;
  a.host_err = d.h_err;
  // one wait may last 5 s of device time (the clock runs at clock_mhz)
  a.max_wait = uint64_t(5.0e6 * d.clock_mhz);
}

// Two plans: the kernels alone (device-resident runs, and runs whose host memory the device
// cannot address), and the kernels with the host copies run by the executor.
void prepare_executor(const Dag &g, const SchedPlan &plan, int32_t per_cu_cap, Device &d) {
  int32_t max_workers = 1, tile_workers = 1;
  d.exec_instance = pick_exec_instance(g, d.launch, d.device, per_cu_cap, &max_workers, &tile_workers);
  d.exec_copies = exec_copies(g, plan);
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d.device) == hipSuccess && khz > 0)
    d.clock_mhz = khz / 1000.0;
  else
    (void)hipGetLastError();  // keep the default rate; leave no sticky error behind
  PSC_HIP(hipHostMalloc(reinterpret_cast<void **>(&d.h_err), 16, hipHostMallocDefault));
  *d.h_err = 0;
  upload_exec_plan(plan_executor(g, d.launch, max_workers, tile_workers, {}), d, d.exec_mem, d.ea);
  const size_t nc = d.exec_copies.size();
  if (nc) {
    const ExecPlan ep = plan_executor(g, d.launch, max_workers, tile_workers, d.exec_copies);
    upload_exec_plan(ep, d, d.exec_mem_copy, d.ea_copy);
    PSC_HIP(hipHostMalloc(reinterpret_cast<void **>(&d.h_copy_nodes), sizeof(ExecNode) * nc, hipHostMallocDefault));
    for (size_t c = 0; c < nc; ++c) d.h_copy_nodes[c] = ep.nodes[ep.nodes.size() - nc + c];  // counts, predecessors
  }
}

}  // namespace

void prepare(psc_sched &s) {
  if (s.dev) return;
  const Dag &g = s.dag->g;
  auto d = std::make_unique<Device>();
  d->device = s.opts.device;
  PSC_HIP(hipSetDevice(d->device));
  // arena for unbound roots, 256-byte aligned slots
  std::vector<size_t> off(g.bufs.size(), 0);
  size_t total = 0;
  for (size_t b = 0; b < g.bufs.size(); ++b) {
    const Buffer &x = g.bufs[b];
    if (x.parent >= 0 || x.bound) continue;
    off[b] = total;
    total += (size_t(x.rows) * x.cols * elem_size(x.dtype) + 255) & ~size_t(255);
  }
  if (total) {
    hipError_t e = hipMalloc(&d->arena, total);
    if (e != hipSuccess) fail(PSC_ERR_OOM, "hipMalloc of " + std::to_string(total) + " bytes: " + hipGetErrorString(e));
  }
  d->base.assign(g.bufs.size(), nullptr);
  for (size_t b = 0; b < g.bufs.size(); ++b) {
    const Buffer &x = g.bufs[b];
    if (x.parent >= 0) continue;
    d->base[b] = x.bound ? static_cast<char *>(x.bound) : static_cast<char *>(d->arena) + off[b];
  }
  const bool dev_mode = s.plan.device;
  d->streams.assign(dev_mode ? 1 : s.plan.total_streams, nullptr);
  for (auto &st : d->streams) PSC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  const bool aql_mode = !dev_mode && s.opts.dispatch == PSC_DISPATCH_AQL;
  d->op_ev.assign(s.plan.ops.size(), nullptr);
  if (!dev_mode && !aql_mode)
    for (size_t i = 0; i < s.plan.ops.size(); ++i)
      if (s.plan.ops[i].recorded || (s.plan.dynamic && s.plan.ops[i].type == PSC_OP_H2D))
        PSC_HIP(hipEventCreateWithFlags(&d->op_ev[i], hipEventDisableTiming));
  d->join_ev.assign(d->streams.size(), nullptr);
  for (auto &e : d->join_ev) PSC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  PSC_HIP(hipEventCreate(&d->start));
  PSC_HIP(hipEventCreate(&d->end));
  if (s.opts.record_ops && !dev_mode && !aql_mode) {
    d->t0.assign(s.plan.ops.size(), nullptr);
    d->t1.assign(s.plan.ops.size(), nullptr);
    for (auto &e : d->t0) PSC_HIP(hipEventCreate(&e));
    for (auto &e : d->t1) PSC_HIP(hipEventCreate(&e));
  }
  d->launch.assign(g.kers.size(), Launch{});
  for (size_t k = 0; k < g.kers.size(); ++k) build_launch(g, *d, int32_t(k), d->launch[k]);
  if (s.opts.mark_components && !dev_mode) {
    const size_t nk = g.kers.size();
    PSC_HIP(hipMalloc(&d->marks, 8 * (nk + 1)));
    make_mark(d->mark_start, d->marks + nk);
    d->mark_after.assign(nk, Launch{});
    for (size_t k = 0; k < nk; ++k) {
      bool end = true;
      for (int32_t q : g.succ[k]) end = end && g.kers[q].component != g.kers[k].component;
      if (end) make_mark(d->mark_after[k], d->marks + k);
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d->device) == hipSuccess && khz > 0)
      d->clock_mhz = khz / 1000.0;
    else
      (void)hipGetLastError();
  }
  if (dev_mode) {
    prepare_executor(g, s.plan, s.opts.exec_per_cu, *d);
  } else if (s.plan.dynamic) {
    d->dyn = std::make_unique<DynState>();
  } else {
    const int32_t nt = s.opts.host_threads > 0 ? s.opts.host_threads : s.plan.total_streams;
    d->disp = std::make_unique<Dispatcher>(s.plan, nt);
    if (aql_mode)
      d->aql = std::make_unique<AqlSchedule>(d->device, s.plan, d->launch, d->mark_after,
                                             d->marks ? &d->mark_start : nullptr, s.opts.record_ops != 0);
  }
  s.dev = std::move(d);
}

namespace {

// Resolve host copies: for every copy op, the io entry whose buffer covers the op's buffer.
std::vector<CopyDesc> resolve_io(const psc_sched &s, const psc_host_io *io, int32_t n_io) {
  const Dag &g = s.dag->g;
  const Device &d = *s.dev;
  std::vector<int32_t> io_buf(n_io, -1);
  for (int32_t i = 0; i < n_io; ++i) {
    if (!io[i].name) fail(PSC_ERR_ARG, "psc_host_io entry with NULL name");
    auto it = g.buf_by_name.find(io[i].name);
    if (it == g.buf_by_name.end()) fail(PSC_ERR_NAME, std::string("unknown buffer '") + io[i].name + "'");
    const Buffer &b = g.bufs[it->second];
    const size_t want = size_t(b.rows) * b.cols * elem_size(b.dtype);
    if (io[i].bytes != want)
      fail(PSC_ERR_ARG, "host buffer for '" + b.name + "' has " + std::to_string(io[i].bytes) +
                            " bytes, expected " + std::to_string(want));
    if (!io[i].host_ptr && want) fail(PSC_ERR_ARG, "NULL host pointer for '" + b.name + "'");
    io_buf[i] = it->second;
  }
  std::vector<CopyDesc> cd(s.plan.ops.size());
  std::vector<char> used(n_io, 0);
  for (size_t o = 0; o < s.plan.ops.size(); ++o) {
    const Op &op = s.plan.ops[o];
    if (op.type == PSC_OP_KERNEL) continue;
    const Buffer &b = g.bufs[op.buffer];
    for (int32_t i = 0; i < n_io; ++i) {
      const Buffer &e = g.bufs[io_buf[i]];
      if (!e.region().covers(b.region())) continue;
      const int64_t es = elem_size(b.dtype);
      char *host = static_cast<char *>(io[i].host_ptr) + ((b.r0 - e.r0) * e.cols + (b.c0 - e.c0)) * es;
      char *dev = buffer_ptr(g, d, op.buffer);
      CopyDesc &c = cd[o];
      c.active = b.rows > 0 && b.cols > 0;
      c.width = size_t(b.cols) * es;
      c.height = size_t(b.rows);
      const size_t dev_pitch = size_t(buffer_ld(g, op.buffer)) * es;
      const size_t host_pitch = size_t(e.cols) * es;
      if (op.type == PSC_OP_H2D) {
        c.dst = dev; c.dpitch = dev_pitch; c.src = host; c.spitch = host_pitch; c.kind = hipMemcpyHostToDevice;
      } else {
        c.dst = host; c.dpitch = host_pitch; c.src = dev; c.spitch = dev_pitch; c.kind = hipMemcpyDeviceToHost;
      }
      used[i] = 1;
      break;
    }
  }
  for (int32_t i = 0; i < n_io; ++i)
    if (!used[i]) fail(PSC_ERR_NAME, std::string("'") + io[i].name + "' covers no isolated write or read of the schedule");
  return cd;
}

void do_copy(const CopyDesc &c, hipStream_t st) {
  if (!c.active) return;
  if (c.dpitch == c.width && c.spitch == c.width)
    PSC_HIP(hipMemcpyAsync(c.dst, c.src, c.width * c.height, c.kind, st));
  else
    PSC_HIP(hipMemcpy2DAsync(c.dst, c.dpitch, c.src, c.spitch, c.width, c.height, c.kind, st));
}

struct HipBackend final : Backend {
  psc_sched &s;
  Device &d;
  const std::vector<CopyDesc> &cd;
  bool timed;
  HipBackend(psc_sched &s_, const std::vector<CopyDesc> &cd_, bool timed_)
      : s(s_), d(*s_.dev), cd(cd_), timed(timed_) {}
  hipStream_t st(int32_t op) const { return d.streams[s.plan.ops[op].stream]; }
  void wait(int32_t op, int32_t awaited) override { PSC_HIP(hipStreamWaitEvent(st(op), d.op_ev[awaited], 0)); }
  void exec(int32_t o) override {
    const Op &op = s.plan.ops[o];
    if (timed) PSC_HIP(hipEventRecord(d.t0[o], st(o)));
    if (op.type == PSC_OP_KERNEL) launch(d.launch[op.kernel], st(o));
    else do_copy(cd[o], st(o));
    if (timed) PSC_HIP(hipEventRecord(d.t1[o], st(o)));
    if (op.type == PSC_OP_KERNEL && d.marks && d.mark_after[op.kernel].func) launch(d.mark_after[op.kernel], st(o));
  }
  void record(int32_t o) override { PSC_HIP(hipEventRecord(d.op_ev[o], st(o))); }
  void stream_done(int32_t stream) override {
    if (stream != 0) PSC_HIP(hipEventRecord(d.join_ev[stream], d.streams[stream]));
  }
};

// The same dispatch sequence written as AQL packets (waits become barrier-AND packets; records
// are implicit: every op completes its own signal).
struct AqlBackend final : Backend {
  AqlSchedule &a;
  explicit AqlBackend(AqlSchedule &a_) : a(a_) {}
  void wait(int32_t op, int32_t awaited) override { a.wait(op, awaited); }
  void exec(int32_t op) override { a.exec(op); }
  void record(int32_t) override {}
  void stream_done(int32_t) override {}
};

void fork_streams(Device &d, hipEvent_t ev) {
  for (size_t i = 1; i < d.streams.size(); ++i) PSC_HIP(hipStreamWaitEvent(d.streams[i], ev, 0));
}

void join_streams(Device &d) {  // join events were recorded by the dispatch threads
  for (size_t i = 1; i < d.streams.size(); ++i) PSC_HIP(hipStreamWaitEvent(d.streams[0], d.join_ev[i], 0));
}

}  // namespace

namespace {

// The schedule as an explicit graph: one node per op; its dependencies are the previous op on the
// same stream and the ops it waits for, so the graph has exactly the schedule's precedences.
void build_graph(psc_sched &s, const std::vector<CopyDesc> &cd) {
  Device &d = *s.dev;
  PSC_HIP(hipGraphCreate(&d.graph, 0));
  const size_t n = s.plan.ops.size();
  std::vector<hipGraphNode_t> node(n, nullptr), last(s.plan.total_streams, nullptr);
  std::vector<hipGraphNode_t> deps;
  auto kernel_node = [&](const Launch &L, const hipGraphNode_t *dp, size_t nd) {
    hipKernelNodeParams kp{};
    void *args[] = {const_cast<unsigned char *>(L.args)};
    kp.func = const_cast<void *>(L.func);
    kp.gridDim = L.grid;
    kp.blockDim = L.block;
    kp.sharedMemBytes = L.shmem;
    kp.kernelParams = args;
    hipGraphNode_t x = nullptr;
    PSC_HIP(hipGraphAddKernelNode(&x, d.graph, dp, nd, &kp));
    return x;
  };
  hipGraphNode_t start_mark = d.marks ? kernel_node(d.mark_start, nullptr, 0) : nullptr;
  for (size_t o = 0; o < n; ++o) {
    const Op &op = s.plan.ops[o];
    deps.clear();
    if (last[op.stream]) deps.push_back(last[op.stream]);
    for (int32_t w : op.waits) deps.push_back(node[w]);
    if (deps.empty() && start_mark) deps.push_back(start_mark);
    hipGraphNode_t nd = nullptr;
    const hipGraphNode_t *dp = deps.empty() ? nullptr : deps.data();
    if (op.type == PSC_OP_KERNEL && !d.launch[op.kernel].empty) {
      nd = kernel_node(d.launch[op.kernel], dp, deps.size());
    } else if (op.type != PSC_OP_KERNEL && cd[o].active) {
      const CopyDesc &c = cd[o];
      if (c.dpitch == c.width && c.spitch == c.width) {
        PSC_HIP(hipGraphAddMemcpyNode1D(&nd, d.graph, dp, deps.size(), c.dst, c.src, c.width * c.height, c.kind));
      } else {
        hipMemcpy3DParms mp{};
        mp.srcPtr = make_hipPitchedPtr(const_cast<void *>(c.src), c.spitch, c.width, c.height);
        mp.dstPtr = make_hipPitchedPtr(c.dst, c.dpitch, c.width, c.height);
        mp.extent = make_hipExtent(c.width, c.height, 1);
        mp.kind = c.kind;
        PSC_HIP(hipGraphAddMemcpyNode(&nd, d.graph, dp, deps.size(), &mp));
      }
    } else {
      PSC_HIP(hipGraphAddEmptyNode(&nd, d.graph, dp, deps.size()));
    }
    node[o] = nd;
    last[op.stream] = nd;
    if (op.type == PSC_OP_KERNEL && d.marks && d.mark_after[op.kernel].func) kernel_node(d.mark_after[op.kernel], &nd, 1);
  }
  PSC_HIP(hipGraphInstantiate(&d.exec, d.graph, nullptr, nullptr, 0));
}

}  // namespace

namespace {

// Failure injection: enqueue the host-order prefix before the failing op on its streams (waits
// of a prefix op only name earlier ops), wait for it, then fail as a launch error would.
[[noreturn]] void run_fault_prefix(psc_sched &s, const std::vector<CopyDesc> &cd) {
  Device &d = *s.dev;
  const int32_t k = s.opts.fault_inject_op - 1;
  HipBackend backend(s, cd, false);
  PSC_HIP(hipEventRecord(d.start, d.streams[0]));
  fork_streams(d, d.start);
  for (int32_t o = 0; o < k; ++o) {
    const Op &op = s.plan.ops[o];
    for (int32_t w : op.waits) backend.wait(o, w);
    backend.exec(o);
    if (op.recorded) backend.record(o);
  }
  for (hipStream_t st : d.streams) PSC_HIP(hipStreamSynchronize(st));
  const Op &f = s.plan.ops[k];
  const std::string what = f.type == PSC_OP_KERNEL ? "kernel '" + s.dag->g.kers[f.kernel].name + "'"
                                                   : std::string(f.type == PSC_OP_H2D ? "H2D of '" : "D2H of '") +
                                                         s.dag->g.bufs[f.buffer].name + "'";
  fail(PSC_ERR_HIP, "injected fault: op " + std::to_string(k) + " (" + what + ") was not launched; the " +
                        std::to_string(k) + " ops before it in host order ran and have finished");
}

// Waits for the run's end event, at most timeout_ms when that is set.
void wait_end(psc_sched &s) {
  Device &d = *s.dev;
  if (s.opts.timeout_ms <= 0) {
    PSC_HIP(hipEventSynchronize(d.end));
    return;
  }
  const auto limit = std::chrono::steady_clock::now() + std::chrono::milliseconds(s.opts.timeout_ms);
  for (;;) {
    const hipError_t q = hipEventQuery(d.end);
    if (q == hipSuccess) return;
    if (q != hipErrorNotReady) PSC_HIP(q);
    if (std::chrono::steady_clock::now() >= limit) {
      d.in_flight = true;
      fail(PSC_ERR_TIMEOUT, "run not finished within timeout_ms = " + std::to_string(s.opts.timeout_ms) +
                                " (still executing; the next psc_run or psc_sched_destroy waits for it)");
    }
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

namespace {

// The scheduling loop of Algorithm 1 for PSC_EAGER / PSC_HEFT on one GPU: select a ready kernel
// and a stream (a device with one command queue), enqueue its uploads, the kernel, its
// read-backs and the callback, and sleep until a callback updates the ready queue or the
// available streams.  Afterwards the plan's ops carry the structure this run had.
void run_dynamic(psc_sched &s, const std::vector<CopyDesc> &cd, bool timed) {
  Device &d = *s.dev;
  const Dag &g = s.dag->g;
  SchedPlan &plan = s.plan;
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  const int32_t S = plan.total_streams;
  DynState &st = *d.dyn;
  // ops of each kernel in the coarse op list: its uploads before it, its read-backs after it
  std::vector<std::vector<int32_t>> ups(nk), reads(nk);
  {
    std::vector<int32_t> pending_up;
    int32_t last_kernel = -1;
    for (size_t o = 0; o < plan.ops.size(); ++o) {
      const Op &op = plan.ops[o];
      if (op.type == PSC_OP_H2D) {
        pending_up.push_back(int32_t(o));
      } else if (op.type == PSC_OP_KERNEL) {
        ups[op.kernel] = pending_up;
        pending_up.clear();
        last_kernel = op.kernel;
      } else if (last_kernel >= 0) {
        reads[last_kernel].push_back(int32_t(o));
      }
    }
  }
  // an upload is issued by whichever of its buffer's readers is dispatched first
  std::vector<int32_t> upload_of(g.bufs.size(), -1);
  for (int32_t k = 0; k < nk; ++k)
    for (int32_t o : ups[k]) upload_of[plan.ops[o].buffer] = o;
  const std::vector<int32_t> upload_as = upload_buffers(g, s.opts.copy_roots != 0);
  std::vector<int32_t> up_stream(plan.ops.size(), -1);
  st.g = &g;
  st.plan = &plan;
  st.indeg.assign(nk, 0);
  st.heap.clear();
  st.available.assign(S, 1);
  st.finished = 0;
  st.updates = 0;
  st.args.assign(nk, DynState::Arg{&st, 0, 0});
  for (int32_t k = 0; k < nk; ++k) {
    st.indeg[k] = static_cast<int32_t>(g.pred[k].size());
    st.args[k].kernel = k;
  }
  for (int32_t k = 0; k < nk; ++k)
    if (!st.indeg[k]) st.push_ready(k);
  std::vector<int32_t> stream_of(nk, -1), pos(S, 0);
  std::vector<double> busy_until(S, 0.0);  // HEFT: predicted time each stream's kernel ends (us)
  std::vector<std::vector<int32_t>> new_waits(plan.ops.size());
  std::vector<int32_t> new_stream(plan.ops.size(), 0), new_pos(plan.ops.size(), 0), new_order(plan.ops.size(), 0);
  int32_t order = 0;
  hipStream_t s0 = d.streams[0];
  PSC_HIP(hipEventRecord(d.start, s0));
  fork_streams(d, d.start);
  const auto t0 = std::chrono::steady_clock::now();
  auto now_us = [&] { return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count(); };
  auto timed_op = [&](int32_t o, hipStream_t q, auto &&body) {
    if (timed) PSC_HIP(hipEventRecord(d.t0[o], q));
    body();
    if (timed) PSC_HIP(hipEventRecord(d.t1[o], q));
  };
  try {
    std::unique_lock<std::mutex> lk(st.mu);
    while (st.finished < nk) {
      while (!st.heap.empty()) {
        const int32_t k = -st.heap.front().second;
        int32_t q = -1;
        if (!plan.heft) {  // eager: any available stream
          for (int32_t x = 0; x < S && q < 0; ++x)
            if (st.available[x]) q = x;
        } else {           // HEFT: earliest predicted finish over every stream; wait for it if busy
          const double now = now_us();
          double best = 1e300;
          int32_t arg = 0;
          for (int32_t x = 0; x < S; ++x) {
            const double f = std::max(now, st.available[x] ? now : busy_until[x]) + plan.dyn_us[k];
            if (f < best - 1e-9) { best = f; arg = x; }
          }
          if (st.available[arg]) q = arg;
        }
        if (q < 0) break;
        std::pop_heap(st.heap.begin(), st.heap.end());
        st.heap.pop_back();
        st.available[q] = 0;
        st.args[k].stream = q;
        lk.unlock();
        // dispatch (uploads, kernel, read-backs, callback) outside the lock
        hipStream_t hs = d.streams[q];
        const int32_t kop = plan.kernel_op[k];
        for (int32_t b : g.iso_in[k]) {
          const int32_t uo = upload_of[upload_as[b]];
          if (uo < 0) continue;
          if (up_stream[uo] < 0) {
            timed_op(uo, hs, [&] { do_copy(cd[uo], hs); });
            PSC_HIP(hipEventRecord(d.op_ev[uo], hs));
            up_stream[uo] = q;
            new_stream[uo] = q, new_pos[uo] = pos[q]++, new_order[uo] = order++;
          } else if (up_stream[uo] != q) {
            PSC_HIP(hipStreamWaitEvent(hs, d.op_ev[uo], 0));
            new_waits[kop].push_back(uo);
          }
        }
        for (int32_t p : g.pred[k])
          if (stream_of[p] != q) new_waits[kop].push_back(plan.kernel_op[p]);
        timed_op(kop, hs, [&] { launch(d.launch[k], hs); });
        new_stream[kop] = q, new_pos[kop] = pos[q]++, new_order[kop] = order++;
        for (int32_t ro : reads[k]) {
          timed_op(ro, hs, [&] { do_copy(cd[ro], hs); });
          new_stream[ro] = q, new_pos[ro] = pos[q]++, new_order[ro] = order++;
        }
        stream_of[k] = q;
        busy_until[q] = now_us() + plan.dyn_us[k];
        PSC_HIP(hipLaunchHostFunc(hs, dyn_callback, &st.args[k]));
        lk.lock();
      }
      if (st.finished >= nk) break;
      const uint64_t seen = st.updates;
      // sleep_till_cb_update; a kernel in flight always ends, so a minute with no callback
      // means the runtime lost one: fail rather than wait for ever
      if (!st.cv.wait_for(lk, std::chrono::seconds(60), [&] { return st.updates != seen; }))
        fail(PSC_ERR_TIMEOUT, "dynamic schedule: no completion callback for 60 s (" +
                                  std::to_string(st.finished) + " of " + std::to_string(nk) + " kernels finished)");
    }
  } catch (...) {
    // callbacks of what was dispatched still reference the state: let them all run first
    for (hipStream_t x : d.streams) (void)hipStreamSynchronize(x);
    throw;
  }
  for (int32_t x = 1; x < S; ++x) PSC_HIP(hipEventRecord(d.join_ev[x], d.streams[x]));
  join_streams(d);
  PSC_HIP(hipEventRecord(d.end, s0));
  for (size_t o = 0; o < plan.ops.size(); ++o) {
    Op &op = plan.ops[o];
    op.stream = new_stream[o];
    op.pos = new_pos[o];
    op.host_order = new_order[o];
    std::sort(new_waits[o].begin(), new_waits[o].end());
    new_waits[o].erase(std::unique(new_waits[o].begin(), new_waits[o].end()), new_waits[o].end());
    op.waits = new_waits[o];
  }
  plan.realized = true;
}

}  // namespace

void run(psc_sched &s, const psc_host_io *io, int32_t n_io, psc_run_stats *stats) {
  prepare(s);
  Device &d = *s.dev;
  PSC_HIP(hipSetDevice(d.device));
  if (d.in_flight) {  // the previous run timed out: its work must end before buffers are reused
    if (d.aql) (void)d.aql->wait_end(0);
    else PSC_HIP(hipEventSynchronize(d.end));
    d.in_flight = false;
  }
  const std::vector<CopyDesc> cd = resolve_io(s, io, n_io);
  if (s.opts.fault_inject_op > 0) run_fault_prefix(s, cd);
  const bool timed = s.opts.record_ops != 0;
  hipStream_t s0 = d.streams[0];
  double host_ms = 0;
  if (s.plan.device) {
    const auto h0 = std::chrono::steady_clock::now();
    // The executor runs each upload and read-back whose host memory the device can address
    // itself (page-locked memory mapped at the same address), as tasks of its copy plan beside
    // the kernels; the others are DMA copies before (uploads) or after (read-backs) it, their
    // nodes empty.  With no copy for the executor the kernels-only plan runs.
    std::vector<char> &dma = d.exec_dma;
    dma.assign(s.plan.ops.size(), 0);
    const size_t nc = d.exec_copies.size();
    size_t n_exec = 0;
    for (size_t c = 0; c < nc; ++c) {
      const ExecCopy &x = d.exec_copies[c];
      const CopyDesc &cp = cd[x.op];
      ExecNode &n = d.h_copy_nodes[c];
      n.variant = 0;
      if (!cp.active || x.rows == 0 || x.width == 0) continue;
      const void *host = x.h2d ? cp.src : cp.dst;
      hipPointerAttribute_t at{};
      const bool mapped = hipPointerGetAttributes(&at, host) == hipSuccess && at.type == hipMemoryTypeHost &&
                          at.devicePointer == host;
      if (!mapped) {
        (void)hipGetLastError();  // an unregistered pointer is an expected outcome, not an error
        dma[x.op] = 1;
        continue;
      }
      CopyArgs a{};
      a.src = static_cast<const unsigned char *>(cp.src);
      a.dst = static_cast<unsigned char *>(cp.dst);
      a.spitch = int64_t(cp.spitch);
      a.dpitch = int64_t(cp.dpitch);
      a.width = int64_t(cp.width);
      a.rows = x.rows;
      a.rows_per_task = x.rows_per_task;
      n.variant = kCopyVariant;
      memcpy(n.args, &a, sizeof(a));
      ++n_exec;
    }
    if (n_exec == 0)  // kernels-only plan: every active copy by DMA
      for (size_t c = 0; c < nc; ++c) dma[d.exec_copies[c].op] = cd[d.exec_copies[c].op].active;
    d.ea_run = n_exec ? &d.ea_copy : &d.ea;
    const ExecArgs &ea = *d.ea_run;
    PSC_HIP(hipEventRecord(d.start, s0));
    if (n_exec)
      PSC_HIP(hipMemcpyAsync(const_cast<ExecNode *>(ea.nodes) + (ea.n_nodes - int32_t(nc)), d.h_copy_nodes,
                             sizeof(ExecNode) * nc, hipMemcpyHostToDevice, s0));
    for (size_t o = 0; o < s.plan.ops.size(); ++o)
      if (s.plan.ops[o].type == PSC_OP_H2D && dma[o]) do_copy(cd[o], s0);
    *d.h_err = 0;  // the previous run has completed: psc_run waits for its end
    PSC_HIP(launch_exec_reset(ea, s0));
    PSC_HIP(launch_exec(ea, d.exec_instance, s0));
    for (size_t o = 0; o < s.plan.ops.size(); ++o)
      if (s.plan.ops[o].type == PSC_OP_D2H && dma[o]) do_copy(cd[o], s0);
    PSC_HIP(hipEventRecord(d.end, s0));
    host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  } else if (s.plan.dynamic) {
    const auto h0 = std::chrono::steady_clock::now();
    run_dynamic(s, cd, timed);
    host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  } else if (d.aql) {
    std::vector<AqlCopy> ac(cd.size());
    for (size_t o = 0; o < cd.size(); ++o) {
      const CopyDesc &c = cd[o];
      ac[o] = AqlCopy{c.active, c.kind == hipMemcpyHostToDevice, c.dst, c.src, c.dpitch, c.spitch, c.width, c.height};
    }
    const auto h0 = std::chrono::steady_clock::now();
    d.aql->begin(ac);
    AqlBackend backend(*d.aql);
    try {
      d.disp->run(backend);
    } catch (...) {
      // nothing may wait forever on an op that was never enqueued: complete those, join, drain
      d.aql->release_undispatched();
      d.aql->end();
      (void)d.aql->wait_end(0);
      throw;
    }
    d.aql->end();
    host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  } else if (s.opts.use_graph) {
    std::vector<const void *> key;
    for (const CopyDesc &c : cd) key.push_back(c.active ? (c.kind == hipMemcpyHostToDevice ? c.src : c.dst) : nullptr);
    if (!d.exec || key != d.graph_key) {
      if (d.exec) { PSC_HIP(hipGraphExecDestroy(d.exec)); d.exec = nullptr; }
      if (d.graph) { PSC_HIP(hipGraphDestroy(d.graph)); d.graph = nullptr; }
      build_graph(s, cd);
      d.graph_key = key;
    }
    const auto h0 = std::chrono::steady_clock::now();
    PSC_HIP(hipEventRecord(d.start, s0));
    PSC_HIP(hipGraphLaunch(d.exec, s0));
    PSC_HIP(hipEventRecord(d.end, s0));
    host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  } else {
    const auto h0 = std::chrono::steady_clock::now();
    if (d.marks) launch(d.mark_start, s0);
    PSC_HIP(hipEventRecord(d.start, s0));
    fork_streams(d, d.start);
    HipBackend backend(s, cd, timed);
    d.disp->run(backend);
    join_streams(d);
    PSC_HIP(hipEventRecord(d.end, s0));
    host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  }
  float ms = 0;
  if (d.aql) {
    if (!d.aql->wait_end(s.opts.timeout_ms)) {
      d.in_flight = true;
      fail(PSC_ERR_TIMEOUT, "run not finished within timeout_ms = " + std::to_string(s.opts.timeout_ms) +
                                " (still executing; the next psc_run or psc_sched_destroy waits for it)");
    }
    ms = float(d.aql->makespan_ms());
  } else {
    wait_end(s);
    PSC_HIP(hipEventElapsedTime(&ms, d.start, d.end));
  }
  d.have_marks = d.marks != nullptr || s.plan.device;
  if (s.plan.device && *d.h_err)
    fail(PSC_ERR_HIP, std::string("device executor stopped (flag ") + std::to_string(*d.h_err) + "): " +
                          (*d.h_err == 2 ? "a task's tile function is not in the executor instance"
                                         : "a wait for a predecessor kernel exceeded its bound"));
  if (timed && s.plan.device) {
    const ExecArgs &ea = *d.ea_run;
    const int32_t nk = ea.n_nodes;
    std::vector<uint64_t> tf(nk), tl(nk);
    uint64_t t0 = 0;
    PSC_HIP(hipMemcpy(tf.data(), ea.t_first, 8 * nk, hipMemcpyDeviceToHost));
    PSC_HIP(hipMemcpy(tl.data(), ea.t_last, 8 * nk, hipMemcpyDeviceToHost));
    PSC_HIP(hipMemcpy(&t0, ea.t_start, 8, hipMemcpyDeviceToHost));
    d.times.assign(s.plan.ops.size(), psc_op_time{0, 0, 0.f, 0.f});
    d.active.assign(s.plan.ops.size(), 0);
    std::vector<int32_t> node_of(s.plan.ops.size(), -1);  // executor node of each op
    if (d.ea_run == &d.ea_copy) {
      const int32_t nkern = nk - int32_t(d.exec_copies.size());
      for (size_t c = 0; c < d.exec_copies.size(); ++c)
        if (!d.exec_dma[d.exec_copies[c].op] && cd[d.exec_copies[c].op].active)
          node_of[d.exec_copies[c].op] = nkern + int32_t(c);
    }
    for (size_t o = 0; o < s.plan.ops.size(); ++o) {
      const Op &op = s.plan.ops[o];
      d.times[o].op = int32_t(o);
      d.times[o].stream = op.stream;
      if (op.type == PSC_OP_KERNEL) node_of[o] = d.launch[op.kernel].empty ? -1 : op.kernel;
      d.active[o] = node_of[o] >= 0;
      if (node_of[o] >= 0) {  // copies by DMA keep no device times
        d.times[o].start_us = float(double(int64_t(tf[node_of[o]] - t0)) / d.clock_mhz);
        d.times[o].end_us = float(double(int64_t(tl[node_of[o]] - t0)) / d.clock_mhz);
      }
    }
    d.have_times = true;
  } else if (timed && d.aql) {
    std::vector<float> a, b;
    d.aql->op_times(a, b);
    d.times.resize(s.plan.ops.size());
    d.active.assign(s.plan.ops.size(), 0);
    for (size_t o = 0; o < s.plan.ops.size(); ++o) {
      const Op &op = s.plan.ops[o];
      d.times[o] = psc_op_time{int32_t(o), op.stream, a[o], b[o]};
      d.active[o] = op.type == PSC_OP_KERNEL ? !d.launch[op.kernel].empty : cd[o].active;
    }
    d.have_times = true;
  } else if (timed) {
    d.times.resize(s.plan.ops.size());
    d.active.assign(s.plan.ops.size(), 0);
    for (size_t o = 0; o < s.plan.ops.size(); ++o) {
      float a = 0, b = 0;
      PSC_HIP(hipEventElapsedTime(&a, d.start, d.t0[o]));
      PSC_HIP(hipEventElapsedTime(&b, d.start, d.t1[o]));
      d.times[o] = psc_op_time{int32_t(o), s.plan.ops[o].stream, a * 1000.f, b * 1000.f};
      const Op &op = s.plan.ops[o];
      d.active[o] = op.type == PSC_OP_KERNEL ? !d.launch[op.kernel].empty : cd[o].active;
    }
    d.have_times = true;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->makespan_ms = ms;
    stats->host_enqueue_ms = host_ms;
    stats->n_ops = int32_t(s.plan.ops.size());
    for (const Op &op : s.plan.ops) {
      stats->n_kernels += op.type == PSC_OP_KERNEL;
      stats->n_h2d += op.type == PSC_OP_H2D;
      stats->n_d2h += op.type == PSC_OP_D2H;
      stats->n_waits += int32_t(op.waits.size());
    }
    stats->n_streams = s.plan.total_streams;
    stats->graph = s.opts.use_graph != 0;
    stats->aql_packets = d.aql ? d.aql->packets_last_run() : 0;
  }
}

void op_times(const psc_sched &s, psc_op_time *out, int32_t cap, int32_t *n) {
  if (!s.dev || !s.dev->have_times) fail(PSC_ERR_STATE, "no recorded run (set record_ops and call psc_run)");
  const auto &t = s.dev->times;
  if (n) *n = int32_t(t.size());
  if (out) {
    if (cap < int32_t(t.size())) fail(PSC_ERR_ARG, "capacity too small");
    std::copy(t.begin(), t.end(), out);
  }
}

// Cost-model samples of the recorded run.  Ops on one stream run one after another, so for each
// other stream a binary search over its ops' start times finds the op (if any) whose interval
// contains this op's start.
void samples(const psc_sched &s, float *feat, float *log_us, int32_t cap, int32_t *n) {
  if (!s.dev || !s.dev->have_times) fail(PSC_ERR_STATE, "no recorded run (set record_ops and call psc_run)");
  const Device &d = *s.dev;
  const Dag &g = s.dag->g;
  const auto &t = d.times;
  const int32_t S = s.plan.total_streams;
  std::vector<std::vector<int32_t>> on(S);  // active ops per stream by start time
  for (size_t o = 0; o < t.size(); ++o)
    if (d.active[o] && t[o].end_us > t[o].start_us) on[s.plan.ops[o].stream].push_back(int32_t(o));
  for (auto &v : on)
    std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return t[a].start_us < t[b].start_us; });
  int32_t cnt = 0;
  for (size_t o = 0; o < t.size(); ++o) cnt += d.active[o] && t[o].end_us > t[o].start_us;
  *n = cnt;
  if (!feat && !log_us) return;
  if (cap < cnt) fail(PSC_ERR_ARG, "capacity too small");
  int32_t i = 0;
  for (size_t o = 0; o < t.size(); ++o) {
    if (!(d.active[o] && t[o].end_us > t[o].start_us)) continue;
    const Op &op = s.plan.ops[o];
    const float st = t[o].start_us;
    int32_t busy = 0;
    for (int32_t q = 0; q < S; ++q) {
      if (q == op.stream || on[q].empty()) continue;
      // last op on q starting at or before st
      auto it = std::upper_bound(on[q].begin(), on[q].end(), st,
                                 [&](float v, int32_t b) { return v < t[b].start_us; });
      if (it == on[q].begin()) continue;
      busy += t[*(it - 1)].end_us > st;
    }
    if (feat) {
      float *f = feat + size_t(i) * kFeatures;
      if (op.type == PSC_OP_KERNEL) kernel_features(g, op.kernel, busy, f);
      else copy_features(g, op.buffer, op.type == PSC_OP_H2D, busy, f);
    }
    if (log_us) log_us[i] = float(std::log(double(t[o].end_us) - double(t[o].start_us)));
    ++i;
  }
}

// Host-only: the device executor's task lists for `workers` workgroups, from launches built on a
// stand-in arena address (never dereferenced).
void device_tasks(const psc_sched &s, int32_t workers, int32_t *tasks, int32_t cap, int32_t *n_tasks,
                  int32_t *work_off) {
  const Dag &g = s.dag->g;
  Device d;
  d.base.assign(g.bufs.size(), nullptr);
  uintptr_t at = uintptr_t(1) << 32;
  for (size_t b = 0; b < g.bufs.size(); ++b) {
    const Buffer &x = g.bufs[b];
    if (x.parent >= 0) continue;
    d.base[b] = reinterpret_cast<char *>(at);
    at += (size_t(x.rows) * x.cols * elem_size(x.dtype) + 255) & ~size_t(255);
  }
  std::vector<Launch> launch(g.kers.size());
  for (size_t k = 0; k < g.kers.size(); ++k) build_launch(g, d, int32_t(k), launch[k]);
  const ExecPlan ep = plan_executor(g, launch, workers, workers, exec_copies(g, build_plan(g, PSC_DEVICE, s.opts)));
  *n_tasks = static_cast<int32_t>(ep.tasks.size());
  if (!tasks && !work_off) return;
  if (cap < *n_tasks) fail(PSC_ERR_ARG, "capacity too small");
  if (tasks)
    for (size_t i = 0; i < ep.tasks.size(); ++i) {
      tasks[3 * i] = ep.tasks[i].node;
      tasks[3 * i + 1] = ep.tasks[i].tile;
      tasks[3 * i + 2] = ep.tasks[i].signal;
    }
  if (work_off)  // workgroups beyond the task count get empty lists
    for (int32_t w = 0; w <= workers; ++w) work_off[w] = ep.work_off[std::min<size_t>(w, ep.work_off.size() - 1)];
}

// Host-only: every kernel launch of the schedule (built on stand-in addresses) is known to the
// AQL dispatcher's code object table; returns the number of distinct kernels, or -1 and a reason.
int32_t aql_check(const psc_sched &s, char *why, int32_t why_cap) {
  const Dag &g = s.dag->g;
  Device d;
  d.base.assign(g.bufs.size(), nullptr);
  uintptr_t at = uintptr_t(1) << 32;
  for (size_t b = 0; b < g.bufs.size(); ++b) {
    const Buffer &x = g.bufs[b];
    if (x.parent >= 0) continue;
    d.base[b] = reinterpret_cast<char *>(at);
    at += (size_t(x.rows) * x.cols * elem_size(x.dtype) + 255) & ~size_t(255);
  }
  std::vector<Launch> ls(g.kers.size() + 1);
  for (size_t k = 0; k < g.kers.size(); ++k) build_launch(g, d, int32_t(k), ls[k]);
  make_mark(ls.back(), reinterpret_cast<uint64_t *>(at));
  std::vector<const void *> seen;
  for (const Launch &L : ls) {
    if (L.empty) continue;
    std::string reason;
    if (!aql_launch_supported(L, &reason)) {
      if (why && why_cap > 0) {
        std::strncpy(why, reason.c_str(), size_t(why_cap - 1));
        why[why_cap - 1] = 0;
      }
      return -1;
    }
    if (std::find(seen.begin(), seen.end(), L.func) == seen.end()) seen.push_back(L.func);
  }
  if (why && why_cap > 0) why[0] = 0;
  return int32_t(seen.size());
}

void component_times(const psc_sched &s, float *done_us, int32_t cap, int32_t *n) {
  const Dag &g = s.dag->g;
  const int32_t nk = static_cast<int32_t>(g.kers.size());
  int32_t nc = 0;
  for (const Kernel &k : g.kers) nc = std::max(nc, k.component + 1);
  *n = nc;
  if (!done_us) return;
  if (cap < nc) fail(PSC_ERR_ARG, "capacity too small");
  if (!s.dev || !s.dev->have_marks)
    fail(PSC_ERR_STATE, "no marked run (set mark_components, or use PSC_DEVICE, and call psc_run)");
  const Device &d = *s.dev;
  PSC_HIP(hipSetDevice(d.device));
  std::vector<uint64_t> at(nk + 1, 0);  // completion clock per END kernel, start at [nk]
  std::vector<char> end(nk, 0);
  for (int32_t k = 0; k < nk; ++k) {
    end[k] = 1;
    for (int32_t q : g.succ[k]) end[k] = end[k] && g.kers[q].component != g.kers[k].component;
  }
  if (s.plan.device) {
    PSC_HIP(hipMemcpy(at.data(), d.ea_run->t_last, 8 * size_t(nk), hipMemcpyDeviceToHost));  // kernels first
    PSC_HIP(hipMemcpy(&at[nk], d.ea_run->t_start, 8, hipMemcpyDeviceToHost));
  } else {
    PSC_HIP(hipMemcpy(at.data(), d.marks, 8 * size_t(nk + 1), hipMemcpyDeviceToHost));
  }
  std::vector<double> done(nc, -1.0);
  for (int32_t k = 0; k < nk; ++k)
    if (end[k]) {
      const double us = double(int64_t(at[k] - at[nk])) / d.clock_mhz;
      double &c = done[g.kers[k].component];
      c = std::max(c, us);
    }
  for (int32_t c = 0; c < nc; ++c) done_us[c] = float(done[c]);
}

void device_info(int device, char *name, int name_cap, char *arch, int arch_cap, int *cus, int *clock_mhz,
                 int64_t *mem) {
  hipDeviceProp_t pr{};
  PSC_HIP(hipGetDeviceProperties(&pr, device));
  auto put = [](char *dst, int cap, const char *src) {
    if (!dst || cap <= 0) return;
    std::strncpy(dst, src, size_t(cap - 1));
    dst[cap - 1] = 0;
  };
  put(name, name_cap, pr.name);
  put(arch, arch_cap, pr.gcnArchName);
  if (cus) *cus = pr.multiProcessorCount;
  if (clock_mhz) *clock_mhz = pr.clockRate / 1000;
  if (mem) *mem = int64_t(pr.totalGlobalMem);
}

void device_ptr(const psc_sched &s, const char *name, void **dptr, int64_t *ld) {
  if (!s.dev) fail(PSC_ERR_STATE, "schedule not prepared");
  const Dag &g = s.dag->g;
  auto it = g.buf_by_name.find(name);
  if (it == g.buf_by_name.end()) fail(PSC_ERR_NAME, std::string("unknown buffer '") + name + "'");
  if (dptr) *dptr = buffer_ptr(g, *s.dev, it->second);
  if (ld) *ld = buffer_ld(g, it->second);
}

void sched_read(const psc_sched &s, const char *name, void *host, size_t bytes) {
  if (!s.dev) fail(PSC_ERR_STATE, "schedule not prepared");
  const Dag &g = s.dag->g;
  auto it = g.buf_by_name.find(name);
  if (it == g.buf_by_name.end()) fail(PSC_ERR_NAME, std::string("unknown buffer '") + name + "'");
  const Buffer &b = g.bufs[it->second];
  const size_t es = size_t(elem_size(b.dtype)), row = size_t(b.cols) * es;
  if (bytes != row * size_t(b.rows))
    fail(PSC_ERR_SHAPE, std::string("buffer '") + name + "' holds " + std::to_string(row * size_t(b.rows)) +
                            " bytes, not " + std::to_string(bytes));
  if (!bytes) return;
  PSC_HIP(hipSetDevice(s.dev->device));
  PSC_HIP(hipDeviceSynchronize());   // whatever is in flight on the schedule's streams lands first
  PSC_HIP(hipMemcpy2D(host, row, buffer_ptr(g, *s.dev, it->second), size_t(buffer_ld(g, it->second)) * es, row,
                      size_t(b.rows), hipMemcpyDeviceToHost));
}

// Seeded values (uniform in [-1, 1)) in the device storage of every root buffer that holds an
// isolated write, so that a schedule can be timed on realistic data without host inputs.
void fill_inputs(psc_sched &s) {
  if (!s.dev) prepare(s);
  const Dag &g = s.dag->g;
  Device &d = *s.dev;
  PSC_HIP(hipSetDevice(d.device));
  std::vector<char> done(g.bufs.size(), 0);
  uint32_t seed = 11u;
  for (int32_t b : g.h2d_bufs) {
    const int32_t r = g.bufs[b].root;
    if (done[r]) continue;
    done[r] = 1;
    const Buffer &rb = g.bufs[r];
    Launch L;
    make_fill(L, buffer_ptr(g, d, r), (rb.rows * rb.cols * elem_size(rb.dtype)) & ~int64_t(3), rb.dtype == PSC_BF16,
              seed++);
    if (!L.empty) launch(L, nullptr);
  }
  PSC_HIP(hipDeviceSynchronize());
}

// Autotuner: times every GEMM tile configuration on device buffers of the given shape (seeded
// values uniform in [-1, 1)) with back-to-back launches between HIP events, records the fastest in the tile cache and
// returns it.  us_per_tile[t] (t < cap) receives each configuration's mean time (0 for t = 0).
int autotune_gemm(int device, int M, int N, int K, int ab, int c, int iters, float *best_us, float *us_per_tile,
                  int cap) {
  PSC_HIP(hipSetDevice(device));
  const size_t ea = ab == PSC_BF16 ? 2 : 4, ec = c == PSC_BF16 ? 2 : 4;
  void *A = nullptr, *B = nullptr, *C = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = 0;
  float best_t = 0;
  auto cleanup = [&] {
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (C) (void)hipFree(C);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
  };
  try {
    PSC_HIP(hipMalloc(&A, std::max<size_t>(16, size_t(M) * K * ea)));
    PSC_HIP(hipMalloc(&B, std::max<size_t>(16, size_t(K) * N * ea)));
    PSC_HIP(hipMalloc(&C, std::max<size_t>(16, size_t(M) * N * ec)));
    PSC_HIP(hipMemset(A, 0, std::max<size_t>(16, size_t(M) * K * ea)));
    PSC_HIP(hipMemset(B, 0, std::max<size_t>(16, size_t(K) * N * ea)));
    PSC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    {
      Launch fa, fb;
      make_fill(fa, A, int64_t(M) * K * ea, ab == PSC_BF16, 1u);
      make_fill(fb, B, int64_t(K) * N * ea, ab == PSC_BF16, 2u);
      launch(fa, st);
      launch(fb, st);
    }
    PSC_HIP(hipEventCreate(&e0));
    PSC_HIP(hipEventCreate(&e1));
    for (int t = 1; t < gemm_num_tiles(); ++t) {
      GemmArgs g{};
      g.A = A; g.B = B; g.C = C;
      g.lda = K; g.ldb = N; g.ldc = N;
      g.M = M; g.N = N; g.K = K; g.alpha = 1.0f;
      Launch L;
      // a configuration that resolves to another one for this shape and dtype (BF16-only tiles
      // with FP32 operands, whole-tile configurations on a shape they do not fit) is not timed:
      // the cache must name the tile a launch actually uses
      if (!make_gemm(L, g, ab, c, t) || L.tile != t) continue;
      for (int w = 0; w < 3; ++w) launch(L, st);
      PSC_HIP(hipEventRecord(e0, st));
      for (int i = 0; i < iters; ++i) launch(L, st);
      PSC_HIP(hipEventRecord(e1, st));
      PSC_HIP(hipEventSynchronize(e1));
      float ms = 0;
      PSC_HIP(hipEventElapsedTime(&ms, e0, e1));
      const float us = ms * 1000.f / float(std::max(1, iters));
      if (us_per_tile && t < cap) us_per_tile[t] = us;
      if (best == 0 || us < best_t) { best = t; best_t = us; }
    }
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
  if (us_per_tile && cap > 0) us_per_tile[0] = 0.f;
  if (best) tile_cache_set(M, N, K, ab, c, best);
  if (best_us) *best_us = best_t;
  return best;
}

int sched_kernel_tile(const psc_sched &s, int32_t kernel) {
  if (!s.dev) fail(PSC_ERR_STATE, "schedule not prepared");
  return s.dev->launch[kernel].tile;
}

void sched_executor_info(const psc_sched &s, int32_t *workers, int32_t *per_cu, uint32_t *groups) {
  if (!s.dev) fail(PSC_ERR_STATE, "schedule not prepared");
  if (!s.plan.device) fail(PSC_ERR_STATE, "not a PSC_DEVICE schedule");
  const Device &d = *s.dev;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d.device) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  if (workers) *workers = d.ea.n_workers;
  if (per_cu) {
    *per_cu = exec_max_workers(d.device, d.exec_instance) / cus;
    if (s.opts.exec_per_cu > 0) *per_cu = std::min(*per_cu, s.opts.exec_per_cu);
  }
  if (groups) *groups = exec_instance_groups(d.exec_instance);
}

void *host_alloc(size_t bytes) {
  void *p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes ? bytes : 1, hipHostMallocDefault);
  if (e != hipSuccess) fail(PSC_ERR_OOM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  return p;
}

void host_free(void *p) {
  if (p) PSC_HIP(hipHostFree(p));
}

void device_sync(int device) {
  PSC_HIP(hipSetDevice(device));
  PSC_HIP(hipDeviceSynchronize());
}

float kernel_time(psc_sched &s, int32_t kernel, int32_t iters) {
  prepare(s);
  Device &d = *s.dev;
  PSC_HIP(hipSetDevice(d.device));
  const Op &op = s.plan.ops[s.plan.kernel_op[kernel]];
  hipStream_t st = d.streams[s.plan.device ? 0 : op.stream];
  PSC_HIP(hipEventRecord(d.start, st));
  for (int32_t i = 0; i < iters; ++i) launch(d.launch[kernel], st);
  PSC_HIP(hipEventRecord(d.end, st));
  wait_end(s);
  float ms = 0;
  PSC_HIP(hipEventElapsedTime(&ms, d.start, d.end));
  return ms * 1000.f / float(std::max(1, iters));
}

}  // namespace psc

psc_sched::psc_sched() = default;
psc_sched::~psc_sched() = default;
