// extern "C" entry points declared in include/psc.h.  Each call converts internal errors into a
// psc_status and a thread-local message; no exception crosses the boundary.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <tuple>
#include <memory>
#include <new>
#include <string>

#include <mutex>
#include <random>
#include <thread>

#include "core.hpp"
#include "dispatch.hpp"
#include "mlp.hpp"
#include "persist.hpp"

namespace psc {
void prepare(psc_sched &s);
void run(psc_sched &s, const psc_host_io *io, int32_t n_io, psc_run_stats *stats);
void op_times(const psc_sched &s, psc_op_time *out, int32_t cap, int32_t *n);
void samples(const psc_sched &s, float *feat, float *log_us, int32_t cap, int32_t *n);
void component_times(const psc_sched &s, float *done_us, int32_t cap, int32_t *n);
int32_t aql_check(const psc_sched &s, char *why, int32_t why_cap);
void device_tasks(const psc_sched &s, int32_t workers, int32_t *tasks, int32_t cap, int32_t *n_tasks,
                  int32_t *work_off);
void device_ptr(const psc_sched &s, const char *name, void **dptr, int64_t *ld);
void sched_read(const psc_sched &s, const char *name, void *host, size_t bytes);
void fill_inputs(psc_sched &s);
void prepare(psc_sched &s);
float kernel_time(psc_sched &s, int32_t kernel, int32_t iters);
void *host_alloc(size_t bytes);
void host_free(void *p);
void device_sync(int device);
void device_info(int device, char *name, int name_cap, char *arch, int arch_cap, int *cus, int *clock_mhz,
                 int64_t *mem);
int autotune_gemm(int device, int M, int N, int K, int ab, int c, int iters, float *best_us, float *us_per_tile,
                  int cap);
int sched_kernel_tile(const psc_sched &s, int32_t kernel);
void sched_executor_info(const psc_sched &s, int32_t *workers, int32_t *per_cu, uint32_t *groups);
void tile_cache_set(int M, int N, int K, int ab, int c, int tile);
int tile_cache_get(int M, int N, int K, int ab, int c);
void tile_cache_clear();
size_t tile_cache_size();
int gemm_num_tiles();
psc_dag *dag_from_json(const char *json, const char *const *sym_names, const int64_t *sym_values, int32_t n_sym,
                       psc_spec_info *info);
}  // namespace psc

namespace {

thread_local std::string g_err;

template <typename F>
psc_status guard(F &&f) {
  try {
    f();
    g_err.clear();
    return PSC_OK;
  } catch (const psc::Error &e) {
    g_err = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return PSC_ERR_OOM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return PSC_ERR_ARG;
  } catch (...) {
    g_err = "unknown error";
    return PSC_ERR_ARG;
  }
}

void need(bool cond, psc_status st, const char *msg) {
  if (!cond) psc::fail(st, msg);
}
void need(bool cond, psc_status st, const std::string &msg) { need(cond, st, msg.c_str()); }

void not_frozen(const psc::Dag &g) {
  if (g.frozen) psc::fail(PSC_ERR_STATE, "the DAG is frozen: it has been scheduled");
}

int32_t find_buffer(const psc::Dag &g, const char *name) {
  need(name != nullptr, PSC_ERR_ARG, "NULL buffer name");
  auto it = g.buf_by_name.find(name);
  if (it == g.buf_by_name.end()) psc::fail(PSC_ERR_NAME, std::string("unknown buffer '") + name + "'");
  return it->second;
}

psc_sched_opts default_opts() {
  psc_sched_opts o;
  std::memset(&o, 0, sizeof(o));
  o.n_streams = 4;
  o.mapper = PSC_MAP_RR;
  return o;
}

}  // namespace

extern "C" {

psc_status psc_dag_create(psc_dag **out) {
  return guard([&] {
    need(out != nullptr, PSC_ERR_ARG, "NULL out");
    *out = new psc_dag();
  });
}

psc_status psc_dag_destroy(psc_dag *dag) {
  return guard([&] {
    if (!dag) return;
    if (dag->g.live_scheds) psc::fail(PSC_ERR_STATE, "destroy every schedule of this DAG first");
    delete dag;
  });
}

psc_status psc_add_buffer(psc_dag *dag, const char *name, int32_t dtype, int64_t rows, int64_t cols,
                          const char *view_of, int64_t row_off, int64_t col_off) {
  return guard([&] {
    need(dag && name, PSC_ERR_ARG, "NULL argument");
    psc::Dag &g = dag->g;
    not_frozen(g);
    need(dtype == PSC_F32 || dtype == PSC_BF16, PSC_ERR_ARG, "dtype must be PSC_F32 or PSC_BF16");
    need(rows >= 0 && cols >= 0 && rows < (int64_t(1) << 31) && cols < (int64_t(1) << 31), PSC_ERR_ARG,
         "rows and cols must be in [0, 2^31)");
    need(std::strlen(name) > 0, PSC_ERR_NAME, "empty buffer name");
    if (g.buf_by_name.count(name)) psc::fail(PSC_ERR_NAME, std::string("duplicate buffer '") + name + "'");
    psc::Buffer b;
    b.name = name;
    b.dtype = dtype;
    b.rows = rows;
    b.cols = cols;
    const int32_t id = static_cast<int32_t>(g.bufs.size());
    if (view_of) {
      const int32_t p = find_buffer(g, view_of);
      const psc::Buffer &pb = g.bufs[p];
      need(row_off >= 0 && col_off >= 0 && row_off + rows <= pb.rows && col_off + cols <= pb.cols,
           PSC_ERR_SHAPE, "view window lies outside its parent");
      need(pb.dtype == dtype, PSC_ERR_SHAPE, "a view must have its parent's dtype");
      b.parent = p;
      b.root = pb.root;
      b.r0 = pb.r0 + row_off;
      b.c0 = pb.c0 + col_off;
    } else {
      need(row_off == 0 && col_off == 0, PSC_ERR_ARG, "offsets need view_of");
      b.root = id;
    }
    g.bufs.push_back(b);
    g.buf_by_name[b.name] = id;
  });
}

psc_status psc_add_kernel(psc_dag *dag, const char *name, int32_t kind, const char *const *inputs, int32_t n_in,
                          const char *const *outputs, int32_t n_out, const psc_kernel_params *params,
                          int32_t *kernel_id) {
  return guard([&] {
    need(dag && name, PSC_ERR_ARG, "NULL argument");
    psc::Dag &g = dag->g;
    not_frozen(g);
    need(kind >= PSC_GEMM && kind <= PSC_ADD, PSC_ERR_ARG, "unknown kernel kind");
    const int want_in = (kind == PSC_GEMM || kind == PSC_ADD) ? 2 : 1;
    if (n_in != want_in || n_out != 1)
      psc::fail(PSC_ERR_ARG, std::string("kernel '") + name + "': wrong number of inputs or outputs for its kind");
    need(inputs && outputs, PSC_ERR_ARG, "NULL operand list");
    need(std::strlen(name) > 0, PSC_ERR_NAME, "empty kernel name");
    if (g.ker_by_name.count(name)) psc::fail(PSC_ERR_NAME, std::string("duplicate kernel '") + name + "'");
    psc::Kernel k;
    k.name = name;
    k.kind = kind;
    for (int32_t i = 0; i < n_in; ++i) k.ins.push_back(find_buffer(g, inputs[i]));
    for (int32_t i = 0; i < n_out; ++i) k.outs.push_back(find_buffer(g, outputs[i]));
    if (params) {
      if (params->alpha_set || params->alpha != 0.0f) k.alpha = params->alpha;
      k.tile = params->tile;
    }
    const int32_t id = static_cast<int32_t>(g.kers.size());
    g.kers.push_back(k);
    g.ker_by_name[k.name] = id;
    if (kernel_id) *kernel_id = id;
  });
}

psc_status psc_add_edge(psc_dag *dag, int32_t src_kernel, const char *src_output, int32_t dst_kernel,
                        const char *dst_input) {
  return guard([&] {
    need(dag && src_output && dst_input, PSC_ERR_ARG, "NULL argument");
    psc::Dag &g = dag->g;
    not_frozen(g);
    const int32_t nk = static_cast<int32_t>(g.kers.size());
    need(src_kernel >= 0 && src_kernel < nk && dst_kernel >= 0 && dst_kernel < nk, PSC_ERR_ARG, "kernel id out of range");
    const int32_t sb = find_buffer(g, src_output), db = find_buffer(g, dst_input);
    const auto &so = g.kers[src_kernel].outs;
    const auto &di = g.kers[dst_kernel].ins;
    if (std::find(so.begin(), so.end(), sb) == so.end())
      psc::fail(PSC_ERR_NAME, std::string("'") + src_output + "' is not an output of kernel '" + g.kers[src_kernel].name + "'");
    if (std::find(di.begin(), di.end(), db) == di.end())
      psc::fail(PSC_ERR_NAME, std::string("'") + dst_input + "' is not an input of kernel '" + g.kers[dst_kernel].name + "'");
    if (!g.bufs[sb].region().overlaps(g.bufs[db].region()))
      psc::fail(PSC_ERR_SHAPE, std::string("edge joins '") + src_output + "' and '" + dst_input + "', which share no storage");
    g.edges.push_back({src_kernel, sb, dst_kernel, db});
  });
}

psc_status psc_dag_from_json(const char *json, const char *const *sym_names, const int64_t *sym_values,
                             int32_t n_sym, psc_dag **out, psc_spec_info *info) {
  psc_dag *made = nullptr;
  const psc_status st = guard([&] {
    need(out != nullptr, PSC_ERR_ARG, "NULL out");
    psc_spec_info tmp;
    made = psc::dag_from_json(json, sym_names, sym_values, n_sym, &tmp);
    *out = made;
    if (info) *info = tmp;
  });
  return st;
}

psc_status psc_buffer_desc(const psc_dag *dag, int32_t id, char *name, int32_t name_cap, int32_t *dtype,
                           int64_t *rows, int64_t *cols, int32_t *parent, int64_t *row_off, int64_t *col_off) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    const psc::Dag &g = dag->g;
    need(id >= 0 && id < int32_t(g.bufs.size()), PSC_ERR_ARG, "buffer id out of range");
    const psc::Buffer &b = g.bufs[id];
    if (name && name_cap > 0) {
      const size_t n = std::min(b.name.size(), size_t(name_cap - 1));
      std::memcpy(name, b.name.data(), n);
      name[n] = 0;
    }
    if (dtype) *dtype = b.dtype;
    if (rows) *rows = b.rows;
    if (cols) *cols = b.cols;
    if (parent) *parent = b.parent;
    const psc::Buffer *p = b.parent >= 0 ? &g.bufs[b.parent] : nullptr;
    if (row_off) *row_off = p ? b.r0 - p->r0 : 0;
    if (col_off) *col_off = p ? b.c0 - p->c0 : 0;
  });
}

psc_status psc_kernel_desc(const psc_dag *dag, int32_t id, char *name, int32_t name_cap, int32_t *kind,
                           int32_t *inputs, int32_t *n_in, int32_t *output, float *alpha, int32_t *component) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    const psc::Dag &g = dag->g;
    need(id >= 0 && id < int32_t(g.kers.size()), PSC_ERR_ARG, "kernel id out of range");
    const psc::Kernel &k = g.kers[id];
    if (name && name_cap > 0) {
      const size_t n = std::min(k.name.size(), size_t(name_cap - 1));
      std::memcpy(name, k.name.data(), n);
      name[n] = 0;
    }
    if (kind) *kind = k.kind;
    if (inputs)
      for (size_t i = 0; i < k.ins.size() && i < 2; ++i) inputs[i] = k.ins[i];
    if (n_in) *n_in = int32_t(k.ins.size());
    if (output) *output = k.outs.empty() ? -1 : k.outs[0];
    if (alpha) *alpha = k.alpha;
    if (component) *component = k.component;
  });
}

psc_status psc_edge_desc(const psc_dag *dag, int32_t e, int32_t *src_kernel, int32_t *src_buffer,
                         int32_t *dst_kernel, int32_t *dst_buffer) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    const psc::Dag &g = dag->g;
    need(e >= 0 && e < int32_t(g.edges.size()), PSC_ERR_ARG, "edge id out of range");
    const psc::Edge &x = g.edges[e];
    if (src_kernel) *src_kernel = x.src;
    if (src_buffer) *src_buffer = x.src_buf;
    if (dst_kernel) *dst_kernel = x.dst;
    if (dst_buffer) *dst_buffer = x.dst_buf;
  });
}

psc_status psc_set_component(psc_dag *dag, int32_t kernel, int32_t component) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    not_frozen(dag->g);
    need(kernel >= 0 && kernel < int32_t(dag->g.kers.size()), PSC_ERR_ARG, "kernel id out of range");
    need(component >= 0, PSC_ERR_ARG, "component must be >= 0");
    dag->g.kers[kernel].component = component;
  });
}

psc_status psc_bind_device(psc_dag *dag, const char *name, void *dptr, size_t bytes) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    psc::Dag &g = dag->g;
    not_frozen(g);
    const int32_t b = find_buffer(g, name);
    psc::Buffer &x = g.bufs[b];
    if (x.parent >= 0) psc::fail(PSC_ERR_NAME, std::string("'") + name + "' is a view; bind its root");
    need(dptr != nullptr, PSC_ERR_ARG, "NULL device pointer");
    need(bytes >= size_t(x.rows) * x.cols * psc::elem_size(x.dtype), PSC_ERR_ARG, "device memory too small");
    x.bound = dptr;
    x.bound_bytes = bytes;
  });
}

psc_status psc_dag_info(const psc_dag *dag, int32_t *n_kernels, int32_t *n_buffers, int32_t *n_edges) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    if (n_kernels) *n_kernels = int32_t(dag->g.kers.size());
    if (n_buffers) *n_buffers = int32_t(dag->g.bufs.size());
    if (n_edges) *n_edges = int32_t(dag->g.edges.size());
  });
}

psc_status psc_buffer_id(const psc_dag *dag, const char *name, int32_t *id) {
  return guard([&] {
    need(dag && id, PSC_ERR_ARG, "NULL argument");
    *id = find_buffer(dag->g, name);
  });
}

psc_status psc_dag_classify(psc_dag *dag, int32_t component, int32_t *kclass, int32_t *edge_inter) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    dag->g.validate();
    dag->g.classify(component, kclass, edge_inter);
  });
}

}  // extern "C"

namespace {

std::unique_ptr<psc_sched> new_sched(psc_dag *dag, int32_t policy, const psc_sched_opts *opts) {
  need(policy >= PSC_COARSE && policy <= PSC_HEFT, PSC_ERR_ARG,
       "policy must be PSC_COARSE, PSC_FINE, PSC_DEVICE, PSC_EAGER or PSC_HEFT");
  psc_sched_opts o = opts ? *opts : default_opts();
  const bool dynamic = policy == PSC_EAGER || policy == PSC_HEFT;
  if (policy != PSC_FINE && !dynamic) o.n_streams = 1;
  if (dynamic) {
    need(!o.use_graph, PSC_ERR_ARG, "dynamic schedules decide at run time; use_graph does not apply");
    need(o.dispatch == PSC_DISPATCH_HIP, PSC_ERR_UNSUPPORTED, "dynamic schedules use PSC_DISPATCH_HIP");
    need(!o.fault_inject_op && !o.timeout_ms && !o.mark_components, PSC_ERR_UNSUPPORTED,
         "fault_inject_op, timeout_ms and mark_components apply to static schedules");
  }
  need(!(policy == PSC_DEVICE && o.use_graph), PSC_ERR_ARG, "PSC_DEVICE runs one kernel; use_graph does not apply");
  need(o.n_streams >= 1 && o.n_streams <= 64, PSC_ERR_ARG, "n_streams must be in [1, 64]");
  need(o.mapper >= PSC_MAP_RR && o.mapper <= PSC_MAP_COMPONENT, PSC_ERR_ARG, "unknown mapper");
  need(!(o.use_graph && o.record_ops), PSC_ERR_ARG, "record_ops cannot be combined with use_graph");
  need(o.device >= 0, PSC_ERR_ARG, "negative device");
  need(o.mark_components == 0 || o.mark_components == 1, PSC_ERR_ARG, "mark_components must be 0 or 1");
  need(o.timeout_ms >= 0, PSC_ERR_ARG, "negative timeout_ms");
  need(o.fault_inject_op >= 0, PSC_ERR_ARG, "negative fault_inject_op");
  need(!(policy == PSC_DEVICE && o.fault_inject_op), PSC_ERR_ARG, "fault_inject_op does not apply to PSC_DEVICE");
  need(o.dispatch == PSC_DISPATCH_HIP || o.dispatch == PSC_DISPATCH_AQL, PSC_ERR_ARG, "unknown dispatch");
  need(o.out_of_order == 0 || o.out_of_order == 1, PSC_ERR_ARG, "out_of_order must be 0 or 1");
  need(o.copy_roots == 0 || o.copy_roots == 1, PSC_ERR_ARG, "copy_roots must be 0 or 1");
  need(o.exec_per_cu >= 0, PSC_ERR_ARG, "exec_per_cu must be >= 0");
  if (o.out_of_order)
    need(policy == PSC_FINE && o.dispatch == PSC_DISPATCH_AQL, PSC_ERR_UNSUPPORTED,
         "out-of-order queues need PSC_FINE with PSC_DISPATCH_AQL (HIP streams are in order)");
  if (o.dispatch == PSC_DISPATCH_AQL) {
    need(policy != PSC_DEVICE, PSC_ERR_ARG, "PSC_DEVICE runs one kernel; dispatch does not apply");
    need(!o.use_graph, PSC_ERR_ARG, "use_graph applies to PSC_DISPATCH_HIP only");
    need(!o.fault_inject_op, PSC_ERR_UNSUPPORTED, "fault_inject_op applies to PSC_DISPATCH_HIP only");
  }
  psc::Dag &g = dag->g;
  if (!g.validated || !g.frozen) g.validate();
  g.frozen = true;
  auto s = std::make_unique<psc_sched>();
  s->dag = dag;
  s->opts = o;
  s->policy = policy;
  s->plan = psc::build_plan(g, policy, o);
  need(size_t(o.fault_inject_op) <= s->plan.ops.size(), PSC_ERR_ARG,
       "fault_inject_op " + std::to_string(o.fault_inject_op) + " beyond the schedule's " +
           std::to_string(s->plan.ops.size()) + " ops");
  return s;
}

// Disjoint union of DAGs: names prefixed with "<i>/", ids and components offset.
std::unique_ptr<psc_dag> dag_union(psc_dag *const *dags, int32_t n) {
  auto u = std::make_unique<psc_dag>();
  psc::Dag &m = u->g;
  int32_t comp_off = 0;
  for (int32_t i = 0; i < n; ++i) {
    need(dags[i] != nullptr, PSC_ERR_ARG, "NULL DAG at batch position " + std::to_string(i));
    const psc::Dag &g = dags[i]->g;
    const int32_t boff = int32_t(m.bufs.size()), koff = int32_t(m.kers.size());
    const std::string pre = std::to_string(i) + "/";
    for (psc::Buffer b : g.bufs) {
      b.name = pre + b.name;
      if (b.parent >= 0) b.parent += boff;
      b.root += boff;
      m.buf_by_name[b.name] = int32_t(m.bufs.size());
      m.bufs.push_back(std::move(b));
    }
    int32_t n_comp = 0;
    for (psc::Kernel k : g.kers) {
      k.name = pre + k.name;
      for (int32_t &x : k.ins) x += boff;
      for (int32_t &x : k.outs) x += boff;
      n_comp = std::max(n_comp, k.component + 1);
      k.component += comp_off;
      m.ker_by_name[k.name] = int32_t(m.kers.size());
      m.kers.push_back(std::move(k));
    }
    for (psc::Edge e : g.edges) {
      e.src += koff;
      e.dst += koff;
      e.src_buf += boff;
      e.dst_buf += boff;
      m.edges.push_back(e);
    }
    comp_off += n_comp;
  }
  return u;
}

}  // namespace

extern "C" {

psc_status psc_schedule(psc_dag *dag, int32_t policy, const psc_sched_opts *opts, psc_sched **out) {
  return guard([&] {
    need(dag && out, PSC_ERR_ARG, "NULL argument");
    auto s = new_sched(dag, policy, opts);
    ++dag->g.live_scheds;
    *out = s.release();
  });
}

psc_status psc_schedule_batch(psc_dag *const *dags, int32_t n, int32_t policy, const psc_sched_opts *opts,
                              psc_sched **out) {
  return guard([&] {
    need(dags && out, PSC_ERR_ARG, "NULL argument");
    need(n >= 1, PSC_ERR_ARG, "a batch needs at least one DAG");
    auto u = dag_union(dags, n);
    auto s = new_sched(u.get(), policy, opts);
    ++u->g.live_scheds;
    s->owned_dag = std::move(u);
    *out = s.release();
  });
}

psc_status psc_sched_export(const psc_sched *sched, psc_op *ops, int32_t cap, int32_t *n_ops, int32_t *waits,
                            int32_t waits_cap, int32_t *n_waits) {
  return guard([&] {
    need(sched != nullptr, PSC_ERR_ARG, "NULL schedule");
    need(!sched->plan.dynamic || sched->plan.realized, PSC_ERR_STATE,
         "a dynamic schedule's queue structure exists after its first psc_run");
    const auto &P = sched->plan.ops;
    int32_t nw = 0;
    for (const auto &op : P) nw += int32_t(op.waits.size());
    if (n_ops) *n_ops = int32_t(P.size());
    if (n_waits) *n_waits = nw;
    if (ops && waits) {
      need(cap >= int32_t(P.size()) && waits_cap >= nw, PSC_ERR_ARG, "capacity too small");
      int32_t off = 0;
      for (size_t i = 0; i < P.size(); ++i) {
        const auto &op = P[i];
        ops[i] = psc_op{int32_t(i), op.type, op.kernel, op.buffer, op.stream, op.pos, op.host_order,
                        int32_t(op.waits.size()), off};
        for (int32_t w : op.waits) waits[off++] = w;
      }
    }
  });
}

psc_status psc_sched_streams(const psc_sched *sched, int32_t *n_streams) {
  return guard([&] {
    need(sched && n_streams, PSC_ERR_ARG, "NULL argument");
    *n_streams = sched->plan.total_streams;
  });
}

psc_status psc_sched_prepare(psc_sched *sched) {
  return guard([&] {
    need(sched != nullptr, PSC_ERR_ARG, "NULL schedule");
    psc::prepare(*sched);
  });
}

psc_status psc_run(psc_sched *sched, const psc_host_io *io, int32_t n_io, psc_run_stats *stats) {
  return guard([&] {
    need(sched != nullptr, PSC_ERR_ARG, "NULL schedule");
    need(n_io >= 0 && (n_io == 0 || io), PSC_ERR_ARG, "bad io list");
    psc::run(*sched, io, n_io, stats);
  });
}

psc_status psc_sched_op_times(const psc_sched *sched, psc_op_time *out, int32_t cap, int32_t *n) {
  return guard([&] {
    need(sched != nullptr, PSC_ERR_ARG, "NULL schedule");
    psc::op_times(*sched, out, cap, n);
  });
}

psc_status psc_device_info(int32_t device, char *name, int32_t name_cap, char *arch, int32_t arch_cap,
                           int32_t *compute_units, int32_t *clock_mhz, int64_t *memory_bytes) {
  return guard([&] {
    need(device >= 0, PSC_ERR_ARG, "negative device");
    psc::device_info(device, name, name_cap, arch, arch_cap, compute_units, clock_mhz, memory_bytes);
  });
}

psc_status psc_sched_device_tasks(const psc_sched *sched, int32_t workers, int32_t *tasks, int32_t cap,
                                  int32_t *n_tasks, int32_t *work_off) {
  return guard([&] {
    need(sched && n_tasks, PSC_ERR_ARG, "NULL argument");
    need(workers >= 1, PSC_ERR_ARG, "workers must be >= 1");
    psc::device_tasks(*sched, workers, tasks, cap, n_tasks, work_off);
  });
}

psc_status psc_sched_aql_check(const psc_sched *sched, int32_t *n_kernels, char *why, int32_t why_cap) {
  return guard([&] {
    need(sched != nullptr, PSC_ERR_ARG, "NULL schedule");
    const int32_t k = psc::aql_check(*sched, why, why_cap);
    if (n_kernels) *n_kernels = k;
  });
}

psc_status psc_sched_component_times(const psc_sched *sched, float *done_us, int32_t cap, int32_t *n) {
  return guard([&] {
    need(sched && n, PSC_ERR_ARG, "NULL argument");
    psc::component_times(*sched, done_us, cap, n);
  });
}

psc_status psc_sched_samples(const psc_sched *sched, float *features, float *log_us, int32_t cap, int32_t *n) {
  return guard([&] {
    need(sched && n, PSC_ERR_ARG, "NULL argument");
    psc::samples(*sched, features, log_us, cap, n);
  });
}

psc_status psc_mlp_create(int32_t device, psc_mlp **out) {
  return guard([&] {
    need(out != nullptr, PSC_ERR_ARG, "NULL out");
    *out = psc::mlp_create(device);
  });
}

psc_status psc_mlp_destroy(psc_mlp *m) {
  return guard([&] { delete m; });
}

psc_status psc_mlp_set_params(psc_mlp *m, const float *params, int64_t n) {
  return guard([&] {
    need(m && params, PSC_ERR_ARG, "NULL argument");
    need(n == psc::kMlpP, PSC_ERR_ARG, "parameter count must be PSC_MLP_PARAMS");
    psc::mlp_set_params(*m, params);
  });
}

psc_status psc_mlp_get_params(psc_mlp *m, float *params, int64_t n) {
  return guard([&] {
    need(m && params, PSC_ERR_ARG, "NULL argument");
    need(n == psc::kMlpP, PSC_ERR_ARG, "parameter count must be PSC_MLP_PARAMS");
    psc::mlp_get_params(*m, params);
  });
}

psc_status psc_mlp_set_norm(psc_mlp *m, const float *mean, const float *std_dev) {
  return guard([&] {
    need(m && mean && std_dev, PSC_ERR_ARG, "NULL argument");
    psc::mlp_set_norm(*m, mean, std_dev);
  });
}

psc_status psc_mlp_predict(psc_mlp *m, const float *x, int64_t n, float *y) {
  return guard([&] {
    need(m && x && y, PSC_ERR_ARG, "NULL argument");
    psc::mlp_predict(*m, x, n, y);
  });
}

psc_status psc_mlp_grad(psc_mlp *m, const float *x, const float *t, int64_t n, float *grads, double *loss) {
  return guard([&] {
    need(m && x && t, PSC_ERR_ARG, "NULL argument");
    const double l = psc::mlp_grad(*m, x, t, n, grads);
    if (loss) *loss = l;
  });
}

psc_status psc_mlp_grad_static(psc_mlp *m, const float *x, const float *t, int64_t n, float *grads, double *loss) {
  return guard([&] {
    need(m && x && t, PSC_ERR_ARG, "NULL argument");
    static_assert(PSC_MLP_STATIC_MAX == psc::kMlpStaticMax, "scratch size");
    const double l = psc::mlp_grad_static(*m, x, t, n, grads);
    if (loss) *loss = l;
  });
}

psc_status psc_mlp_save(psc_mlp *m, const char *path) {
  return guard([&] {
    need(m && path, PSC_ERR_ARG, "NULL argument");
    psc::MlpState st;
    psc::mlp_get_state(*m, st);
    psc::mlp_file_write(path, st);
  });
}

psc_status psc_mlp_load(psc_mlp *m, const char *path) {
  return guard([&] {
    need(m && path, PSC_ERR_ARG, "NULL argument");
    const psc::MlpState st = psc::mlp_file_read(path);   // everything checked before any change
    psc::mlp_put_state(*m, st);
  });
}

psc_status psc_mlp_file_check(const char *path, int64_t *step) {
  return guard([&] {
    need(path != nullptr, PSC_ERR_ARG, "NULL path");
    const psc::MlpState st = psc::mlp_file_read(path);
    if (step) *step = st.step;
  });
}

psc_status psc_mlp_train(psc_mlp *m, const float *x, const float *t, int64_t n, const psc_mlp_train_opts *opts,
                         float *epoch_loss) {
  return guard([&] {
    need(m && x && t && opts, PSC_ERR_ARG, "NULL argument");
    psc::MlpTrainOpts o;
    o.epochs = opts->epochs;
    o.batch = opts->batch;
    o.lr = opts->lr;
    o.beta1 = opts->beta1;
    o.beta2 = opts->beta2;
    o.eps = opts->eps;
    o.shuffle_seed = opts->shuffle_seed;
    psc::mlp_train(*m, x, t, n, o, epoch_loss);
  });
}

psc_status psc_kernel_features(const psc_dag *dag, int32_t kernel, int32_t in_flight, float *f) {
  return guard([&] {
    need(dag && f, PSC_ERR_ARG, "NULL argument");
    need(dag->g.validated, PSC_ERR_STATE, "DAG not validated (schedule it first)");
    need(kernel >= 0 && kernel < int32_t(dag->g.kers.size()), PSC_ERR_ARG, "kernel id out of range");
    need(in_flight >= 0, PSC_ERR_ARG, "negative in_flight");
    psc::kernel_features(dag->g, kernel, in_flight, f);
  });
}

psc_status psc_cost_predict(psc_mlp *m, const float *x, int64_t n, float *us) {
  return guard([&] {
    need(x && us, PSC_ERR_ARG, "NULL argument");
    need(n >= 0, PSC_ERR_ARG, "negative row count");
    if (n == 0) return;
    auto cost = m ? psc::mlp_cost_model(m) : psc::make_heuristic_cost();
    std::vector<double> d(n);
    cost->predict_us(x, n, d.data());
    for (int64_t i = 0; i < n; ++i) us[i] = float(d[i]);
  });
}

psc_status psc_sched_queue_order(const psc_sched *sched, int32_t *out_of_order) {
  return guard([&] {
    need(sched && out_of_order, PSC_ERR_ARG, "NULL argument");
    *out_of_order = sched->plan.out_of_order ? 1 : 0;
  });
}

psc_status psc_sched_device_ptr(const psc_sched *sched, const char *name, void **dptr, int64_t *ld) {
  return guard([&] {
    need(sched && name, PSC_ERR_ARG, "NULL argument");
    psc::device_ptr(*sched, name, dptr, ld);
  });
}

psc_status psc_sched_read(const psc_sched *sched, const char *name, void *host, size_t bytes) {
  return guard([&] {
    need(sched && name && (host || bytes == 0), PSC_ERR_ARG, "NULL argument");
    psc::sched_read(*sched, name, host, bytes);
  });
}

psc_status psc_kernel_time(psc_sched *sched, int32_t kernel, int32_t iters, float *avg_us) {
  return guard([&] {
    need(sched && avg_us, PSC_ERR_ARG, "NULL argument");
    need(kernel >= 0 && kernel < int32_t(sched->dag->g.kers.size()), PSC_ERR_ARG, "kernel id out of range");
    need(iters >= 1, PSC_ERR_ARG, "iters must be >= 1");
    *avg_us = psc::kernel_time(*sched, kernel, iters);
  });
}

psc_status psc_host_alloc(size_t bytes, void **out) {
  return guard([&] {
    need(out != nullptr, PSC_ERR_ARG, "NULL out");
    *out = psc::host_alloc(bytes);
  });
}

psc_status psc_host_free(void *ptr) {
  return guard([&] { psc::host_free(ptr); });
}

psc_status psc_device_sync(int32_t device) {
  return guard([&] {
    need(device >= 0, PSC_ERR_ARG, "negative device");
    psc::device_sync(device);
  });
}

namespace {
struct TraceBackend final : psc::Backend {
  std::mutex m;
  std::vector<int32_t> ev;
  int32_t jitter_us;
  uint32_t seed;
  explicit TraceBackend(int32_t j, uint32_t s) : jitter_us(j), seed(s) {}
  void jitter(int32_t salt) {
    if (jitter_us <= 0) return;
    thread_local std::mt19937 rng;
    thread_local bool seeded = false;
    if (!seeded) {
      rng.seed(seed ^ (uint32_t(std::hash<std::thread::id>()(std::this_thread::get_id())) + uint32_t(salt)));
      seeded = true;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(rng() % uint32_t(jitter_us + 1)));
  }
  void push(int32_t a, int32_t b, int32_t c) {
    std::lock_guard<std::mutex> lk(m);
    ev.insert(ev.end(), {a, b, c});
  }
  void wait(int32_t op, int32_t awaited) override { jitter(op); push(0, op, awaited); }
  void exec(int32_t op) override { jitter(op); push(1, op, -1); }
  void record(int32_t op) override { jitter(op); push(2, op, -1); }
  void stream_done(int32_t stream) override { push(3, -1, stream); }
};
}  // namespace

psc_status psc_sched_dispatch_trace(const psc_sched *sched, int32_t host_threads, int32_t jitter_us, uint32_t seed,
                                    int32_t *out, int32_t cap, int32_t *n) {
  return guard([&] {
    need(sched && n, PSC_ERR_ARG, "NULL argument");
    need(host_threads >= 0 && jitter_us >= 0, PSC_ERR_ARG, "negative argument");
    const int32_t nt = host_threads > 0 ? host_threads : sched->plan.total_streams;
    psc::Dispatcher disp(sched->plan, nt);
    TraceBackend tb(jitter_us, seed);
    disp.run(tb);
    *n = int32_t(tb.ev.size() / 3);
    if (out) {
      need(cap >= int32_t(tb.ev.size()), PSC_ERR_ARG, "capacity too small");
      std::copy(tb.ev.begin(), tb.ev.end(), out);
    }
  });
}

psc_status psc_gemm_tile_count(int32_t *n) {
  return guard([&] {
    need(n != nullptr, PSC_ERR_ARG, "NULL n");
    *n = psc::gemm_num_tiles();
  });
}

psc_status psc_tile_cache_set(int32_t M, int32_t N, int32_t K, int32_t ab_dtype, int32_t c_dtype, int32_t tile) {
  return guard([&] {
    need(M >= 0 && N >= 0 && K >= 0, PSC_ERR_ARG, "negative size");
    need(tile >= 0 && tile < psc::gemm_num_tiles(), PSC_ERR_ARG, "tile out of range");
    need((ab_dtype == PSC_F32 || ab_dtype == PSC_BF16) && (c_dtype == PSC_F32 || c_dtype == PSC_BF16), PSC_ERR_ARG,
         "bad dtype");
    psc::tile_cache_set(M, N, K, ab_dtype, c_dtype, tile);
  });
}

psc_status psc_tile_cache_get(int32_t M, int32_t N, int32_t K, int32_t ab_dtype, int32_t c_dtype, int32_t *tile) {
  return guard([&] {
    need(tile != nullptr, PSC_ERR_ARG, "NULL tile");
    *tile = psc::tile_cache_get(M, N, K, ab_dtype, c_dtype);
  });
}

psc_status psc_tile_cache_key(int32_t device, char *key, int32_t cap) {
  return guard([&] {
    need(key != nullptr && cap > 0, PSC_ERR_ARG, "NULL key or cap <= 0");
    const std::string k = psc::tile_cache_key(device);
    need(int32_t(k.size()) < cap, PSC_ERR_ARG, "key buffer too small (" + std::to_string(k.size() + 1) + " bytes needed)");
    std::memcpy(key, k.c_str(), k.size() + 1);
  });
}

psc_status psc_tile_cache_save(const char *path, const char *key) {
  return guard([&] {
    need(path && key, PSC_ERR_ARG, "NULL argument");
    psc::tile_cache_save(path, key);
  });
}

psc_status psc_tile_cache_load(const char *path, const char *key, int32_t *n_loaded) {
  return guard([&] {
    need(path && key, PSC_ERR_ARG, "NULL argument");
    const int n = psc::tile_cache_load(path, key);
    if (n_loaded) *n_loaded = n;
  });
}

psc_status psc_tile_cache_clear(int32_t *n_removed) {
  return guard([&] {
    if (n_removed) *n_removed = int32_t(psc::tile_cache_size());
    psc::tile_cache_clear();
  });
}

psc_status psc_autotune_gemm(int32_t device, int32_t M, int32_t N, int32_t K, int32_t ab_dtype, int32_t c_dtype,
                             int32_t iters, int32_t *best_tile, float *best_us, float *us_per_tile, int32_t cap) {
  return guard([&] {
    need(M > 0 && N > 0 && K >= 0, PSC_ERR_ARG, "M and N must be positive, K >= 0");
    need(iters >= 1, PSC_ERR_ARG, "iters must be >= 1");
    need((ab_dtype == PSC_F32 || ab_dtype == PSC_BF16) && (c_dtype == PSC_F32 || c_dtype == PSC_BF16), PSC_ERR_ARG,
         "bad dtype");
    const int t = psc::autotune_gemm(device, M, N, K, ab_dtype, c_dtype, iters, best_us, us_per_tile, cap);
    if (best_tile) *best_tile = t;
  });
}

psc_status psc_autotune_dag(psc_dag *dag, int32_t device, int32_t iters, int32_t *n_tuned) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    need(iters >= 1, PSC_ERR_ARG, "iters must be >= 1");
    const psc::Dag &g = dag->g;
    std::map<std::tuple<int, int, int, int, int>, int> seen;
    for (const psc::Kernel &k : g.kers) {
      if (k.kind != PSC_GEMM || k.tile > 0) continue;
      const psc::Buffer &a = g.bufs[k.ins[0]], &b = g.bufs[k.ins[1]], &c = g.bufs[k.outs[0]];
      if (a.rows == 0 || b.cols == 0) continue;
      seen[{int(a.rows), int(b.cols), int(a.cols), a.dtype, c.dtype}] = 1;
    }
    for (const auto &kv : seen) {
      const auto &[M, N, K, ab, c] = kv.first;
      psc::autotune_gemm(device, M, N, K, ab, c, iters, nullptr, nullptr, 0);
    }
    if (n_tuned) *n_tuned = int32_t(seen.size());
  });
}

psc_status psc_autotune_dag_in_schedule(psc_dag *dag, int32_t policy, const psc_sched_opts *opts, int32_t top_k,
                                        int32_t max_classes, int32_t iters, int32_t *n_changed) {
  return guard([&] {
    need(dag != nullptr, PSC_ERR_ARG, "NULL dag");
    need(top_k >= 1 && iters >= 1 && max_classes >= 1, PSC_ERR_ARG, "top_k, max_classes and iters must be >= 1");
    const psc::Dag &g = dag->g;
    const int device = opts ? opts->device : 0;
    // GEMM classes and how many kernels of the DAG each has
    std::map<std::tuple<int, int, int, int, int>, int> count;
    for (const psc::Kernel &k : g.kers) {
      if (k.kind != PSC_GEMM || k.tile > 0) continue;
      const psc::Buffer &a = g.bufs[k.ins[0]], &b = g.bufs[k.ins[1]], &c = g.bufs[k.outs[0]];
      if (a.rows == 0 || b.cols == 0) continue;
      ++count[{int(a.rows), int(b.cols), int(a.cols), a.dtype, c.dtype}];
    }
    struct Cls {
      std::tuple<int, int, int, int, int> key;
      double weight;               // isolated best time x kernels of the class
      std::vector<int> candidates; // tiles by isolated time, fastest first
    };
    std::vector<Cls> cls;
    const int nt = psc::gemm_num_tiles();
    for (const auto &kv : count) {
      const auto &[M, N, K, ab, c] = kv.first;
      std::vector<float> us(nt, 0.f);
      float best_us = 0;
      psc::autotune_gemm(device, M, N, K, ab, c, iters, &best_us, us.data(), nt);   // caches the fastest
      std::vector<int> order;
      for (int t = 1; t < nt; ++t)
        if (us[t] > 0) order.push_back(t);
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return us[x] < us[y]; });
      if (int(order.size()) > top_k) order.resize(top_k);
      cls.push_back({kv.first, double(best_us) * kv.second, order});
    }
    std::stable_sort(cls.begin(), cls.end(), [](const Cls &x, const Cls &y) { return x.weight > y.weight; });
    if (int32_t(cls.size()) > max_classes) cls.resize(max_classes);   // the rest keep the isolated choice
    auto makespan = [&]() {
      psc_sched *s = nullptr;
      psc_status st = psc_schedule(dag, policy, opts, &s);
      if (st != PSC_OK) psc::fail(st, psc_last_error());
      std::vector<double> mk;
      try {
        psc::fill_inputs(*s);
        psc_run_stats rs{};
        psc::run(*s, nullptr, 0, &rs);
        for (int32_t it = 0; it < iters; ++it) {
          psc::run(*s, nullptr, 0, &rs);
          mk.push_back(rs.makespan_ms);
        }
      } catch (...) {
        psc_sched_destroy(s);
        throw;
      }
      psc_sched_destroy(s);
      std::nth_element(mk.begin(), mk.begin() + mk.size() / 2, mk.end());
      return mk[mk.size() / 2];
    };
    int32_t changed = 0;
    // coordinate descent, heaviest class first: each class's candidates timed in the schedule
    // with every other class at its current choice
    for (const Cls &c : cls) {
      if (c.candidates.size() < 2) continue;
      const auto &[M, N, K, ab, cd] = c.key;
      int best_t = c.candidates[0];
      double best_ms = -1;
      for (int t : c.candidates) {
        psc::tile_cache_set(M, N, K, ab, cd, t);
        const double ms = makespan();
        if (best_ms < 0 || ms < best_ms) {
          best_ms = ms;
          best_t = t;
        }
      }
      psc::tile_cache_set(M, N, K, ab, cd, best_t);
      changed += best_t != c.candidates[0];
    }
    if (n_changed) *n_changed = changed;
  });
}

psc_status psc_autotune_schedule(psc_dag *dag, int32_t policy, const psc_sched_opts *candidates, int32_t n,
                                 int32_t iters, int32_t *best, float *ms_per_run) {
  return guard([&] {
    need(dag && candidates && best, PSC_ERR_ARG, "NULL argument");
    need(n >= 1 && iters >= 1, PSC_ERR_ARG, "need at least one candidate and one iteration");
    int32_t bi = -1;
    double bt = 0;
    for (int32_t i = 0; i < n; ++i) {
      psc_sched *s = nullptr;
      double ms = -1;
      if (psc_schedule(dag, policy, &candidates[i], &s) == PSC_OK) {
        try {
          psc::run(*s, nullptr, 0, nullptr);
          psc::run(*s, nullptr, 0, nullptr);
          const auto t0 = std::chrono::steady_clock::now();
          for (int32_t it = 0; it < iters; ++it) psc::run(*s, nullptr, 0, nullptr);
          ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / iters;
        } catch (...) {
          psc_sched_destroy(s);
          throw;
        }
        psc_sched_destroy(s);
      }
      if (ms_per_run) ms_per_run[i] = float(ms);
      if (ms >= 0 && (bi < 0 || ms < bt)) {
        bi = i;
        bt = ms;
      }
    }
    need(bi >= 0, PSC_ERR_ARG, "no candidate schedule could be built");
    *best = bi;
  });
}

psc_status psc_sched_kernel_tile(const psc_sched *sched, int32_t kernel, int32_t *tile) {
  return guard([&] {
    need(sched && tile, PSC_ERR_ARG, "NULL argument");
    need(kernel >= 0 && kernel < int32_t(sched->dag->g.kers.size()), PSC_ERR_ARG, "kernel id out of range");
    need(sched->dag->g.kers[kernel].kind == PSC_GEMM, PSC_ERR_ARG, "not a GEMM kernel");
    *tile = psc::sched_kernel_tile(*sched, kernel);
  });
}

psc_status psc_sched_executor_info(const psc_sched *sched, int32_t *workers, int32_t *per_cu, uint32_t *groups) {
  return guard([&] {
    need(sched, PSC_ERR_ARG, "NULL argument");
    psc::sched_executor_info(*sched, workers, per_cu, groups);
  });
}

psc_status psc_sched_destroy(psc_sched *sched) {
  return guard([&] {
    if (!sched) return;
    --sched->dag->g.live_scheds;
    delete sched;
  });
}

const char *psc_last_error(void) { return g_err.c_str(); }

int32_t psc_abi_version(void) { return PSC_ABI_VERSION; }

}  // extern "C"
