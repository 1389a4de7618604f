// Device-side DAG executor (policy PSC_DEVICE): one persistent kernel runs every kernel of the DAG
// as tiles.  The host list-schedules the tiles onto the executor's workgroups (one ordered task
// list per workgroup); a workgroup waits for a task's predecessor kernels through per-kernel
// completion counters.  Host-side interface used by the runtime.
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
  int32_t n_pred;    // predecessor kernels: pred[pred_off .. pred_off + n_pred)
  int32_t pred_off;
  int32_t tile_m;    // output rows / columns covered by one task (cost estimates)
  int32_t tile_n;
  int32_t pad[2];
  unsigned char args[96];  // GemmArgs / SoftmaxArgs / TransArgs / AddArgs
};

// An isolated upload or read-back run by the executor's own workgroups (variant 420): rows of
// `width` bytes from src (row pitch spitch) to dst (dpitch), task t covering rows
// [t rows_per_task, (t + 1) rows_per_task).  One side is page-locked host memory the device
// reads or writes directly; the host fills the record before every run.
struct CopyArgs {
  const unsigned char *src;
  unsigned char *dst;
  int64_t spitch, dpitch, width;
  int32_t rows, rows_per_task;
};
constexpr int kCopyVariant = 420;
static_assert(sizeof(CopyArgs) <= sizeof(ExecNode::args), "copy record fits a node's arguments");

// One entry of a workgroup's task list.  signal > 0: after this task, publish `signal`
// completed tiles of `node` (the task and the ones of the same node right before it).
struct alignas(16) ExecTask {
  int32_t node;
  int32_t tile;
  int32_t signal;
  int32_t pad;
};

struct ExecArgs {
  const ExecNode *nodes;
  const int32_t *pred;
  const ExecTask *tasks;   // every workgroup's list, back to back
  const int32_t *work_off; // workgroup w runs tasks[work_off[w] .. work_off[w + 1])
  uint32_t *done;          // per kernel: tiles completed
  uint32_t *ctl;           // [0] error flags: 1 = a wait exceeded its bound
  uint32_t *host_err;      // page-locked host word: set to 1 by any workgroup that stops early
  uint64_t *t_first;       // per kernel: device clock when its first tile started
  uint64_t *t_last;        // per kernel: device clock when its last tile finished
  uint64_t *t_start;       // device clock at reset
  int32_t n_nodes;
  int32_t n_workers;
  uint64_t max_wait;       // device-clock ticks one wait may last before the run stops with an error
};

// Builds the executor's description of a kernel from the launch it would use standalone.
// kind: psc_kind; dtypes: 0 = f32, 1 = bf16; want: workgroups the kernel can expect to use
// (GEMM tiles are chosen to give at least that many tasks where possible).
ExecNode make_exec_node(int kind, const unsigned char *args, int in_dtype, int out_dtype, int tile, int want);

// Tile-function groups: the group bit of a node variant (0 for the empty variant 0).  Groups
// 0-5: FP32 GEMM tiles (64x64 and 32x32 staged through LDS, split-K, direct-load with 1, 2 and 4
// column blocks); 6-12: the BF16 ones (and a separate group for the unaligned direct-load
// tile); 13: softmax, transpose, add and the host copies; 14: the BF16 64x64 K-split tile (its
// registers alone exceed what two workgroups per CU leave, so only the one-per-CU instances hold
// it).
constexpr uint32_t kGElem = 1u << 13;
__host__ __device__ constexpr uint32_t exec_variant_group(int v) {
  return v == 110 || v == 111 ? 1u << 0
       : v == 114 || v == 115 ? 1u << 1
       : v >= 138 && v <= 151 ? 1u << 2
       : v >= 152 && v <= 155 ? 1u << 3
       : v == 158 || v == 159 ? 1u << 4
       : v == 162 || v == 163 ? 1u << 5
       : v == 210 || v == 211 ? 1u << 6
       : v == 214 || v == 215 ? 1u << 7
       : v >= 238 && v <= 251 ? 1u << 8
       : v == 252 || v == 253 ? 1u << 9
       : v == 254 || v == 255 ? 1u << 10
       : v == 258 || v == 259 ? 1u << 11
       : v == 262 || v == 263 ? 1u << 12
       : (v >= 300 && v <= 413) || v == 420 ? kGElem
       : v == 266 || v == 267 ? 1u << 14
                              : 0u;
}

// Compiled executor instances (0 .. exec_num_instances() - 1), each holding the tile-function
// groups exec_instance_groups(i); the last holds every group.  exec_max_workers: workgroups of
// instance i the device holds resident at once (CUs x workgroups per CU by its registers and LDS).
int exec_num_instances();
uint32_t exec_instance_groups(int instance);
int exec_max_workers(int device, int instance);

// Launch helpers (enqueue on `stream`).  The executor runs a.n_workers workgroups, at most as
// many as the GPU holds resident at once (a task may wait for any other workgroup's earlier task).
hipError_t launch_exec_reset(const ExecArgs &a, hipStream_t stream);
hipError_t launch_exec(const ExecArgs &a, int instance, hipStream_t stream);

}  // namespace psc
