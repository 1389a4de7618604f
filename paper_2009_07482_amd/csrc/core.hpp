// Internal data structures of the DAG executor: the buffer/kernel IR (Sec. III's
// G = <(K, B), (E_I, E_O, E)>), the command-queue structure a policy produces (Def. 4), and the
// device state a schedule owns.  Host-only; the HIP runtime parts live in runtime.cpp.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "psc.h"

namespace psc {

// Error carried from internal code to the C boundary, which turns it into a psc_status.
struct Error {
  psc_status status;
  std::string msg;
};
[[noreturn]] void fail(psc_status st, const std::string &msg);

inline int64_t elem_size(int dtype) { return dtype == PSC_BF16 ? 2 : 4; }

struct Region {  // rows x cols window at (r0, c0) of root buffer `root`
  int32_t root;
  int64_t r0, c0, rows, cols;
  bool overlaps(const Region &o) const {
    return root == o.root && rows > 0 && cols > 0 && o.rows > 0 && o.cols > 0 &&
           r0 < o.r0 + o.rows && o.r0 < r0 + rows && c0 < o.c0 + o.cols && o.c0 < c0 + cols;
  }
  bool covers(const Region &o) const {
    return root == o.root && r0 <= o.r0 && c0 <= o.c0 && o.r0 + o.rows <= r0 + rows &&
           o.c0 + o.cols <= c0 + cols;
  }
};

struct Buffer {
  std::string name;
  int32_t dtype = PSC_F32;
  int64_t rows = 0, cols = 0;
  int32_t parent = -1;  // direct parent for a view
  int32_t root = -1;    // root buffer id (itself for a root)
  int64_t r0 = 0, c0 = 0;  // absolute window offset inside the root
  void *bound = nullptr;
  size_t bound_bytes = 0;
  Region region() const { return Region{root, r0, c0, rows, cols}; }
};

struct Kernel {
  std::string name;
  int32_t kind = PSC_GEMM;
  std::vector<int32_t> ins, outs;
  float alpha = 1.0f;
  int32_t tile = 0;
  int32_t component = 0;
};

struct Edge {
  int32_t src, src_buf, dst, dst_buf;
};

struct Dag {
  std::vector<Buffer> bufs;
  std::unordered_map<std::string, int32_t> buf_by_name;
  std::vector<Kernel> kers;
  std::unordered_map<std::string, int32_t> ker_by_name;
  std::vector<Edge> edges;
  bool frozen = false;
  int32_t live_scheds = 0;

  // Derived by validate():
  bool validated = false;
  std::vector<std::vector<int32_t>> pred, succ;       // kernel adjacency, sorted, unique
  std::vector<std::vector<int32_t>> iso_in;           // per kernel: isolated-write buffer ids
  std::vector<std::vector<int32_t>> iso_out;          // per kernel: isolated-read buffer ids
  std::vector<int32_t> h2d_bufs;                      // distinct isolated-write buffers

  void validate();                                    // throws Error
  std::vector<int32_t> bfs_order() const;             // Kahn, FIFO, roots by id
  void classify(int32_t comp, int32_t *kclass, int32_t *edge_inter) const;
};

// Op of a command-queue structure.
struct Op {
  int32_t type;     // psc_op_type
  int32_t kernel;   // or -1
  int32_t buffer;   // or -1
  int32_t stream;
  int32_t pos;
  int32_t host_order;
  std::vector<int32_t> waits;  // ids of ops on other streams this op waits for
  bool recorded = false;       // some op waits on this one
};

struct SchedPlan {
  bool device = false;         // PSC_DEVICE: streams beyond 0 only describe precedences
  // PSC_EAGER / PSC_HEFT: kernels are dispatched one at a time at run time, each after its
  // predecessors' completion callbacks; the ops below hold every upload, kernel and read-back,
  // and each run rewrites their stream, pos, host_order and waits with what it did
  bool dynamic = false;
  bool heft = false;
  bool realized = false;       // a dynamic schedule has run at least once
  std::vector<double> dyn_us;    // per kernel: predicted microseconds (the cost model)
  std::vector<double> dyn_rank;  // per kernel: bottom-level rank on those predictions
  bool out_of_order = false;   // queues run kernels out of order: precedences are the waits alone
  int32_t n_streams = 1;       // compute streams
  int32_t total_streams = 1;   // + upload and read-back streams (copy_stream)
  std::vector<Op> ops;         // index = op id; host order = id order
  std::vector<int32_t> kernel_op;  // kernel id -> op id
};

// Feature vector of one op, the input of every cost model (all float32):
//   [0..5]  one-hot kind: GEMM, transpose, softmax, add, H2D, D2H
//   [6]     log2 M  (output rows; the copied buffer's rows for a copy)
//   [7]     log2 N  (output columns)
//   [8]     log2 K  (GEMM inner dimension; 0 otherwise)
//   [9]     log2 of the algorithmic bytes (every input and the output once)
//   [10]    1 if the first operand (or the copied buffer) is BF16, else 0
//   [11]    other streams with an op in flight when this op starts
constexpr int kFeatures = 12;
// Per buffer, the buffer its isolated write is uploaded as (psc_sched_opts.copy_roots).
std::vector<int32_t> upload_buffers(const Dag &g, bool copy_roots);
void kernel_features(const Dag &g, int32_t kernel, int32_t in_flight, float *f);
void copy_features(const Dag &g, int32_t buffer, bool h2d, int32_t in_flight, float *f);

// Cost model interface used by the EFT mapper: predicted microseconds of each feature row.
struct CostModel {
  virtual ~CostModel() = default;
  virtual void predict_us(const float *feat, int64_t n, double *us) = 0;
};
std::unique_ptr<CostModel> make_heuristic_cost();
std::unique_ptr<CostModel> mlp_cost_model(const psc_mlp *m);  // mlp.hip

SchedPlan build_plan(const Dag &g, int policy, const psc_sched_opts &o);

struct Device;  // HIP state, runtime.cpp

}  // namespace psc

struct psc_dag {
  psc::Dag g;
};

struct psc_sched {
  psc_dag *dag = nullptr;
  std::unique_ptr<psc_dag> owned_dag;  // a batch's union (dag points to it); outlives dev
  psc_sched_opts opts{};
  int32_t policy = PSC_FINE;
  psc::SchedPlan plan;
  std::unique_ptr<psc::Device> dev;
  psc_sched();
  ~psc_sched();
};
