// DAG validation and classification (Sec. III).
//
// validate() checks operand shapes per kernel kind, builds the kernel dependency graph from the
// edges of E, rejects cycles, derives the isolated writes (inputs no edge feeds) and isolated
// reads (outputs that feed no edge), and proves that every pair of kernels touching overlapping
// storage, one of them writing, is ordered by a path of edges -- the condition under which every
// topological order (every valid schedule, Def. 5) computes the same result.
#include <algorithm>
#include <deque>
#include <queue>
#include <sstream>

#include "core.hpp"

namespace psc {

[[noreturn]] void fail(psc_status st, const std::string &msg) { throw Error{st, msg}; }

namespace {

const char *kind_name(int k) {
  switch (k) {
    case PSC_GEMM: return "gemm";
    case PSC_TRANSPOSE: return "transpose";
    case PSC_SOFTMAX: return "softmax";
    case PSC_ADD: return "add";
  }
  return "?";
}

void check_kernel_shapes(const Dag &g, const Kernel &k) {
  auto B = [&](int32_t id) -> const Buffer & { return g.bufs[id]; };
  auto shape_err = [&](const std::string &m) {
    fail(PSC_ERR_SHAPE, "kernel '" + k.name + "' (" + kind_name(k.kind) + "): " + m);
  };
  auto dims = [&](const Buffer &b) {
    std::ostringstream s;
    s << b.name << " " << b.rows << "x" << b.cols;
    return s.str();
  };
  switch (k.kind) {
    case PSC_GEMM: {
      const Buffer &a = B(k.ins[0]), &b = B(k.ins[1]), &c = B(k.outs[0]);
      if (a.cols != b.rows) shape_err("A.cols != B.rows (" + dims(a) + ", " + dims(b) + ")");
      if (c.rows != a.rows || c.cols != b.cols)
        shape_err("C must be A.rows x B.cols (" + dims(c) + ")");
      if (a.dtype != b.dtype) shape_err("A and B must share a dtype");
      break;
    }
    case PSC_TRANSPOSE: {
      const Buffer &a = B(k.ins[0]), &b = B(k.outs[0]);
      if (b.rows != a.cols || b.cols != a.rows) shape_err("output must be the input's transpose shape");
      if (a.dtype != b.dtype) shape_err("input and output dtypes differ");
      break;
    }
    case PSC_SOFTMAX: {
      const Buffer &a = B(k.ins[0]), &b = B(k.outs[0]);
      if (a.rows != b.rows || a.cols != b.cols) shape_err("output shape must equal input shape");
      break;
    }
    case PSC_ADD: {
      const Buffer &a = B(k.ins[0]), &b = B(k.ins[1]), &c = B(k.outs[0]);
      if (a.rows != b.rows || a.cols != b.cols || c.rows != a.rows || c.cols != a.cols)
        shape_err("A, B and C must have one shape");
      if (a.dtype != b.dtype) shape_err("A and B must share a dtype");
      break;
    }
    default:
      fail(PSC_ERR_ARG, "kernel '" + k.name + "': unknown kind");
  }
}

// Does every cell of `target` lie in the union of `parts`?  (Grid decomposition by cut lines.)
bool union_covers(const Region &target, const std::vector<Region> &parts) {
  if (target.rows == 0 || target.cols == 0) return true;
  std::vector<int64_t> rc{target.r0, target.r0 + target.rows}, cc{target.c0, target.c0 + target.cols};
  for (const Region &p : parts) {
    if (!p.overlaps(target)) continue;
    rc.push_back(std::clamp(p.r0, target.r0, target.r0 + target.rows));
    rc.push_back(std::clamp(p.r0 + p.rows, target.r0, target.r0 + target.rows));
    cc.push_back(std::clamp(p.c0, target.c0, target.c0 + target.cols));
    cc.push_back(std::clamp(p.c0 + p.cols, target.c0, target.c0 + target.cols));
  }
  std::sort(rc.begin(), rc.end());
  rc.erase(std::unique(rc.begin(), rc.end()), rc.end());
  std::sort(cc.begin(), cc.end());
  cc.erase(std::unique(cc.begin(), cc.end()), cc.end());
  for (size_t i = 0; i + 1 < rc.size(); ++i)
    for (size_t j = 0; j + 1 < cc.size(); ++j) {
      Region cell{target.root, rc[i], cc[j], rc[i + 1] - rc[i], cc[j + 1] - cc[j]};
      bool hit = false;
      for (const Region &p : parts)
        if (p.covers(cell)) { hit = true; break; }
      if (!hit) return false;
    }
  return true;
}

}  // namespace

void Dag::validate() {
  const int32_t nk = static_cast<int32_t>(kers.size());
  for (const Kernel &k : kers) check_kernel_shapes(*this, k);

  // kernel graph from E
  pred.assign(nk, {});
  succ.assign(nk, {});
  for (const Edge &e : edges) {
    pred[e.dst].push_back(e.src);
    succ[e.src].push_back(e.dst);
  }
  for (int32_t k = 0; k < nk; ++k) {
    for (auto *v : {&pred[k], &succ[k]}) {
      std::sort(v->begin(), v->end());
      v->erase(std::unique(v->begin(), v->end()), v->end());
    }
    if (std::binary_search(pred[k].begin(), pred[k].end(), k))
      fail(PSC_ERR_CYCLE, "kernel '" + kers[k].name + "' feeds itself");
  }
  // cycle check (Kahn) and topological index
  std::vector<int32_t> indeg(nk), topo_idx(nk, -1);
  for (int32_t k = 0; k < nk; ++k) indeg[k] = static_cast<int32_t>(pred[k].size());
  std::deque<int32_t> q;
  for (int32_t k = 0; k < nk; ++k)
    if (!indeg[k]) q.push_back(k);
  int32_t seen = 0;
  while (!q.empty()) {
    int32_t k = q.front();
    q.pop_front();
    topo_idx[k] = seen++;
    for (int32_t s : succ[k])
      if (--indeg[s] == 0) q.push_back(s);
  }
  if (seen != nk) fail(PSC_ERR_CYCLE, "the edges form a cycle");

  // storage accesses per root buffer
  struct Access { int32_t kernel, buf; bool write; };
  std::vector<std::vector<Access>> by_root(bufs.size());
  for (int32_t k = 0; k < nk; ++k) {
    for (int32_t b : kers[k].ins) by_root[bufs[b].root].push_back({k, b, false});
    for (int32_t b : kers[k].outs) by_root[bufs[b].root].push_back({k, b, true});
    // a kernel must not read storage it writes (no in-place kernels)
    for (int32_t bi : kers[k].ins)
      for (int32_t bo : kers[k].outs)
        if (bufs[bi].region().overlaps(bufs[bo].region()))
          fail(PSC_ERR_SHAPE, "kernel '" + kers[k].name + "' reads and writes overlapping storage ('" +
                                  bufs[bi].name + "', '" + bufs[bo].name + "')");
    for (size_t i = 0; i < kers[k].outs.size(); ++i)
      for (size_t j = i + 1; j < kers[k].outs.size(); ++j)
        if (bufs[kers[k].outs[i]].region().overlaps(bufs[kers[k].outs[j]].region()))
          fail(PSC_ERR_SHAPE, "kernel '" + kers[k].name + "' has overlapping outputs");
  }

  // isolated writes and reads (Sec. III): per (kernel, input) without an incoming edge, and
  // per (kernel, output) without an outgoing edge
  std::vector<std::vector<int32_t>> in_edges(nk), out_edges(nk);
  for (size_t e = 0; e < edges.size(); ++e) {
    in_edges[edges[e].dst].push_back(static_cast<int32_t>(e));
    out_edges[edges[e].src].push_back(static_cast<int32_t>(e));
  }
  iso_in.assign(nk, {});
  iso_out.assign(nk, {});
  h2d_bufs.clear();
  std::vector<char> is_h2d(bufs.size(), 0);
  for (int32_t k = 0; k < nk; ++k) {
    for (int32_t b : kers[k].ins) {
      std::vector<Region> fed;
      for (int32_t ei : in_edges[k])
        if (edges[ei].dst_buf == b) fed.push_back(bufs[edges[ei].src_buf].region());
      const Region rb = bufs[b].region();
      if (fed.empty()) {
        for (const Access &a : by_root[rb.root])
          if (a.write && bufs[a.buf].region().overlaps(rb))
            fail(PSC_ERR_RACE, "input '" + bufs[b].name + "' of kernel '" + kers[k].name +
                                   "' overlaps output '" + bufs[a.buf].name + "' of kernel '" +
                                   kers[a.kernel].name + "' but no edge feeds it");
        if (std::find(iso_in[k].begin(), iso_in[k].end(), b) == iso_in[k].end())
          iso_in[k].push_back(b);
        if (!is_h2d[b]) {
          is_h2d[b] = 1;
          h2d_bufs.push_back(b);
        }
      } else if (!union_covers(rb, fed)) {
        fail(PSC_ERR_SHAPE, "input '" + bufs[b].name + "' of kernel '" + kers[k].name +
                                "' is only partly produced by the edges that feed it");
      }
    }
    for (int32_t b : kers[k].outs) {
      bool feeds = false;
      for (int32_t ei : out_edges[k])
        if (edges[ei].src_buf == b) { feeds = true; break; }
      if (!feeds && std::find(iso_out[k].begin(), iso_out[k].end(), b) == iso_out[k].end())
        iso_out[k].push_back(b);
    }
  }
  // distinct host-written buffers must not overlap each other
  for (size_t i = 0; i < h2d_bufs.size(); ++i)
    for (size_t j = i + 1; j < h2d_bufs.size(); ++j)
      if (bufs[h2d_bufs[i]].region().overlaps(bufs[h2d_bufs[j]].region()))
        fail(PSC_ERR_RACE, "host inputs '" + bufs[h2d_bufs[i]].name + "' and '" +
                               bufs[h2d_bufs[j]].name + "' overlap");

  // ordering of conflicting accesses: reachability along edges, searched backwards from the
  // later kernel (in topological index) over kernels no earlier than the earlier one
  std::vector<int32_t> stamp(nk, -1);
  int32_t gen = 0;
  std::vector<int32_t> stack;
  auto reaches = [&](int32_t from, int32_t to) {  // path from -> to ?
    if (topo_idx[from] >= topo_idx[to]) return false;
    ++gen;
    stack.assign(1, to);
    stamp[to] = gen;
    while (!stack.empty()) {
      int32_t v = stack.back();
      stack.pop_back();
      for (int32_t p : pred[v]) {
        if (p == from) return true;
        if (stamp[p] != gen && topo_idx[p] > topo_idx[from]) {
          stamp[p] = gen;
          stack.push_back(p);
        }
      }
    }
    return false;
  };
  for (const auto &acc : by_root) {
    for (size_t i = 0; i < acc.size(); ++i) {
      if (!acc[i].write) continue;
      const Region ri = bufs[acc[i].buf].region();
      for (size_t j = 0; j < acc.size(); ++j) {
        if (j == i || acc[j].kernel == acc[i].kernel) continue;
        if (acc[j].write && j < i) continue;
        if (!ri.overlaps(bufs[acc[j].buf].region())) continue;
        int32_t a = acc[i].kernel, b = acc[j].kernel;
        if (!reaches(a, b) && !reaches(b, a))
          fail(PSC_ERR_RACE, "kernels '" + kers[a].name + "' and '" + kers[b].name +
                                 "' access overlapping storage ('" + bufs[acc[i].buf].name + "', '" +
                                 bufs[acc[j].buf].name + "') with no edge path ordering them");
      }
    }
  }
  // an output read back to the host must not be overwritten later
  for (int32_t k = 0; k < nk; ++k)
    for (int32_t b : iso_out[k])
      for (const Access &a : by_root[bufs[b].root])
        if (a.write && a.kernel != k && bufs[a.buf].region().overlaps(bufs[b].region()) &&
            reaches(k, a.kernel))
          fail(PSC_ERR_RACE, "output '" + bufs[b].name + "' is read back to the host but kernel '" +
                                 kers[a.kernel].name + "' overwrites its storage later");
  validated = true;
}

std::vector<int32_t> Dag::bfs_order() const {
  // Breadth-first from FRONT (the roots), a kernel becoming eligible once all its predecessors
  // are processed, so the order is topological (Def. 5); ties by kernel id.
  const int32_t nk = static_cast<int32_t>(kers.size());
  std::vector<int32_t> indeg(nk), order;
  order.reserve(nk);
  for (int32_t k = 0; k < nk; ++k) indeg[k] = static_cast<int32_t>(pred[k].size());
  std::deque<int32_t> q;
  for (int32_t k = 0; k < nk; ++k)
    if (!indeg[k]) q.push_back(k);
  while (!q.empty()) {
    int32_t k = q.front();
    q.pop_front();
    order.push_back(k);
    for (int32_t s : succ[k])
      if (--indeg[s] == 0) q.push_back(s);
  }
  return order;
}

void Dag::classify(int32_t comp, int32_t *kclass, int32_t *edge_inter) const {
  // Defs. 1-3 of Sec. III with FRONT = kernels of the component without a producer inside it,
  // END = without a consumer inside it, IN = the others.
  const int32_t nk = static_cast<int32_t>(kers.size());
  if (kclass) {
    for (int32_t k = 0; k < nk; ++k) {
      kclass[k] = 0;
      if (kers[k].component != comp) continue;
      bool has_pred = false, has_succ = false;
      for (int32_t p : pred[k]) has_pred |= kers[p].component == comp;
      for (int32_t s : succ[k]) has_succ |= kers[s].component == comp;
      if (!has_pred) kclass[k] |= PSC_FRONT;
      if (!has_succ) kclass[k] |= PSC_END;
      if (has_pred && has_succ) kclass[k] |= PSC_IN;
    }
  }
  if (edge_inter)
    for (size_t e = 0; e < edges.size(); ++e)
      edge_inter[e] = kers[edges[e].src].component != kers[edges[e].dst].component;
}

}  // namespace psc
