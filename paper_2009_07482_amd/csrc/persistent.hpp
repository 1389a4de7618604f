// Device-side DAG executor (policy PSC_DEVICE): one persistent kernel runs every kernel of the DAG
// as tiles pulled from a device work queue, releasing a kernel's tiles when all its predecessors
// have completed.  Host-side interface used by the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kernels.hpp"

namespace psc {

// One DAG kernel as the executor sees it (device memory, read-only during a run).
struct alignas(16) ExecNode {
  int32_t variant;   // which tile function (see persistent.hip)
  int32_t n_tiles;   // tasks of this kernel (>= 1; an empty kernel has one no-op task)
  int32_t n_succ;    // successors: succ[succ_off .. succ_off + n_succ)
  int32_t succ_off;
  int32_t n_pred;    // number of distinct predecessor kernels
  int32_t pad[3];
  unsigned char args[96];  // GemmArgs / SoftmaxArgs / TransArgs / AddArgs
};

struct ExecArgs {
  const ExecNode *nodes;
  const int32_t *succ;
  const uint64_t *roots;   // initial queue content: the tasks of every kernel with no predecessor
  uint32_t *ctl;           // [0] head, [1] tail, [2] error, [3] unused
  uint32_t *pending;       // per kernel: predecessors not yet complete
  uint32_t *done;          // per kernel: tiles completed
  uint64_t *slots;         // work queue, one slot per task: ((kernel + 1) << 32) | tile, 0 = empty
  uint64_t *t_first;       // per kernel: device clock when its first tile started
  uint64_t *t_last;        // per kernel: device clock when its last tile finished
  uint64_t *t_start;       // device clock at queue reset
  int32_t n_nodes;
  int32_t n_roots;
  uint32_t total_tasks;
  uint32_t max_spin;       // bound on every wait: beyond it the run stops with ctl[2] = 1
};

// Builds the executor's description of a kernel from the launch it would use standalone.
// kind: psc_kind; dtypes: 0 = f32, 1 = bf16.
ExecNode make_exec_node(int kind, const unsigned char *args, int in_dtype, int out_dtype, int tile);

// Launch helpers (enqueue on `stream`).
hipError_t launch_exec_reset(const ExecArgs &a, hipStream_t stream);
hipError_t launch_exec(const ExecArgs &a, int workers, hipStream_t stream);
int exec_max_workers(int device);

}  // namespace psc
