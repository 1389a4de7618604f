// Device-side DAG executor (policy PSC_DEVICE).
//
// The fine-grained schedules of Sec. IV-B enforce a kernel's precedences with events between host
// queues; here the same precedences are enforced on the GPU, at tile granularity, by one
// persistent kernel.  Every DAG kernel is split into tasks (GEMM output tiles, groups of 16
// softmax rows, 64 x 64 transpose tiles, groups of 8 added rows).  A work queue in device memory
// holds one slot per task; the reset kernel fills it with the tasks of the kernels that have no
// predecessor.  Each workgroup of the executor repeatedly claims the next slot (an atomic head),
// waits until that slot has been published, runs the task's tile function, and counts the task
// as done; the workgroup that completes a kernel's last task decrements the pending-predecessor
// count of each successor, and publishes all tasks of every successor that reaches zero (an
// atomic tail reserves their slots).  Task results are published with agent-scope release
// (fence before the completion count) and read after an agent-scope acquire (the slot load and a
// fence), so tiles written on one XCD are visible to consumers on another.
//
// Progress: a claimed slot is published eventually because, while any task is unfinished, some
// published task has all its predecessors done (the DAG is acyclic) and only executing
// workgroups publish.  Every wait is bounded by max_spin polls: past it (or once another
// workgroup has flagged an error) the workgroup records ctl[2] = 1 and exits, so every wave of
// the grid reaches its exit even if a description were wrong; a workgroup whose loop runs more
// iterations than there are tasks also stops and flags an error.  Claims past the last task exit.
#include "persistent.hpp"

#include "tiles.hpp"

namespace psc {

namespace {

constexpr uint64_t kExit = ~uint64_t(0);

template <int NV, bool VEC, bool IN_BF16, bool OUT_BF16>
__device__ __forceinline__ void softmax_task(const SoftmaxArgs &p, int tile) {
  const int wave = threadIdx.x >> 6;
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    const int row = tile * 16 + j * 4 + wave;
    if (row < p.R) softmax_row<NV, VEC, IN_BF16, OUT_BF16>(p, row);
  }
}

template <bool IN_BF16, bool OUT_BF16>
__device__ __forceinline__ void add_task(const AddArgs &p, int tile) {
#pragma unroll 1
  for (int rr = 0; rr < 8; ++rr) {
    const int r = tile * 8 + rr;
    if (r >= p.R) break;
    for (int c = threadIdx.x; c < p.C; c += 256) {
      const float a = load_elem<IN_BF16>(p.A, int64_t(r) * p.lda + c);
      const float b = load_elem<IN_BF16>(p.B, int64_t(r) * p.ldb + c);
      store_elem<OUT_BF16>(p.Cp, int64_t(r) * p.ldc + c, a + b);
    }
  }
}

// Loads a kernel-argument record as wavefront-uniform (scalar) values.
template <typename T>
__device__ __forceinline__ T uniform_load(const unsigned char *p) {
  static_assert(sizeof(T) % 4 == 0, "argument records are whole dwords");
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i)
    w[i] = __builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t *>(p)[i]);
  T out;
  memcpy(&out, w, sizeof(T));
  return out;
}

__device__ __forceinline__ void run_task(const ExecNode *ndp, int tile, unsigned char *smem) {
  const ExecNode &nd = *ndp;
  switch (__builtin_amdgcn_readfirstlane(nd.variant)) {
    case 110: gemm_f32_tile<64, 64, 16, 32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 111: gemm_f32_tile<64, 64, 16, 32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 114: gemm_f32_tile<32, 32, 32, 16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 115: gemm_f32_tile<32, 32, 32, 16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 138: gemm_f32_splitk_tile<32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 139: gemm_f32_splitk_tile<32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 142: gemm_f32_splitk_tile<16, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 143: gemm_f32_splitk_tile<16, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 148: gemm_f32_splitk_tile<16, 16, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 149: gemm_f32_splitk_tile<16, 16, false, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 150: gemm_f32_splitk_tile<16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 151: gemm_f32_splitk_tile<16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 160: gemm_bf16_tile<64, 64, 64, 32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 161: gemm_bf16_tile<64, 64, 64, 32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 164: gemm_bf16_tile<32, 32, 64, 16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 165: gemm_bf16_tile<32, 32, 64, 16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 188: gemm_bf16_splitk_tile<32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 189: gemm_bf16_splitk_tile<32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 192: gemm_bf16_splitk_tile<16, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 193: gemm_bf16_splitk_tile<16, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 198: gemm_bf16_splitk_tile<16, 16, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 199: gemm_bf16_splitk_tile<16, 16, false, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 200: gemm_bf16_splitk_tile<16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 201: gemm_bf16_splitk_tile<16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem); break;
    case 300: softmax_task<0, false, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 301: softmax_task<0, false, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 302: softmax_task<0, false, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 303: softmax_task<0, false, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 312: softmax_task<1, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 313: softmax_task<1, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 314: softmax_task<1, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 315: softmax_task<1, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 320: softmax_task<2, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 321: softmax_task<2, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 322: softmax_task<2, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 323: softmax_task<2, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 328: softmax_task<4, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 329: softmax_task<4, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 330: softmax_task<4, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 331: softmax_task<4, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 336: softmax_task<8, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 337: softmax_task<8, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 338: softmax_task<8, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 339: softmax_task<8, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile); break;
    case 400: transpose_tile<float>(uniform_load<TransArgs>(nd.args), tile, smem); break;
    case 401: transpose_tile<uint16_t>(uniform_load<TransArgs>(nd.args), tile, smem); break;
    case 410: add_task<false, false>(uniform_load<AddArgs>(nd.args), tile); break;
    case 411: add_task<false, true>(uniform_load<AddArgs>(nd.args), tile); break;
    case 412: add_task<true, false>(uniform_load<AddArgs>(nd.args), tile); break;
    case 413: add_task<true, true>(uniform_load<AddArgs>(nd.args), tile); break;
    default: break;  // 0: empty kernel, nothing to compute
  }
}

constexpr int kExecSmem = 49152;  // the largest tile function's LDS (FP32 K-split tiles)

__global__ __launch_bounds__(256) void exec_reset_kernel(ExecArgs a) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < a.total_tasks) a.slots[i] = i < uint32_t(a.n_roots) ? a.roots[i] : 0;
  if (i < uint32_t(a.n_nodes)) {
    a.pending[i] = uint32_t(a.nodes[i].n_pred);
    a.done[i] = 0;
    a.t_first[i] = kExit;
    a.t_last[i] = 0;
  }
  if (i == 0) {
    a.ctl[0] = 0;
    a.ctl[1] = uint32_t(a.n_roots);
    a.ctl[2] = 0;
    a.ctl[3] = 0;
    *a.t_start = wall_clock64();
  }
}

// Completion of one task by thread 0: count it; the task that completes its kernel releases
// the successors whose last predecessor this was and publishes all their tasks.
__device__ __forceinline__ void complete_task(const ExecArgs &a, int32_t node) {
  const ExecNode &nd = a.nodes[node];
  const uint32_t d = __hip_atomic_fetch_add(&a.done[node], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  if (d + 1 != uint32_t(nd.n_tiles)) return;
  __hip_atomic_store(&a.t_last[node], uint64_t(wall_clock64()), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int32_t j = 0; j < nd.n_succ; ++j) {
    const int32_t s = a.succ[nd.succ_off + j];
    const uint32_t left = __hip_atomic_fetch_sub(&a.pending[s], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (left != 1) continue;
    const uint32_t nt = uint32_t(a.nodes[s].n_tiles);
    const uint32_t base = __hip_atomic_fetch_add(&a.ctl[1], nt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t t = 0; t < nt && base + t < a.total_tasks; ++t)
      __hip_atomic_store(&a.slots[base + t], (uint64_t(s + 1) << 32) | t, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Claim by thread 0: the next queue slot's task once published, or kExit (queue exhausted, an
// error flagged elsewhere, or this wait exceeded its bound -- then flag the error).
__device__ __forceinline__ uint64_t claim_task(const ExecArgs &a) {
  const uint32_t i = __hip_atomic_fetch_add(&a.ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (i >= a.total_tasks) return kExit;
  for (uint32_t spin = 0;; ++spin) {
    const uint64_t x = __hip_atomic_load(&a.slots[i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (x) return x;
    if (__hip_atomic_load(&a.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return kExit;
    if (spin >= a.max_spin) {
      __hip_atomic_fetch_or(&a.ctl[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return kExit;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Every branch that encloses a barrier depends only on wavefront-uniform values: the task word is
// broadcast through LDS and read with readfirstlane, so the exit test, the kernel index and the
// tile arguments live in scalar registers and all 256 threads take the same path each iteration.
__global__ __launch_bounds__(256) void exec_kernel(ExecArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kExecSmem];
  __shared__ uint64_t s_task;
  int32_t prev = -1;  // kernel of the task finished in the previous iteration (uniform)
  for (uint32_t iter = 0;; ++iter) {
    if (threadIdx.x == 0) {
      if (prev >= 0) complete_task(a, prev);
      // no workgroup can run more tasks than exist: a longer loop means the run is broken
      if (iter > a.total_tasks) {
        __hip_atomic_fetch_or(&a.ctl[2], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_task = kExit;
      } else {
        s_task = claim_task(a);
      }
    }
    __syncthreads();
    const uint64_t raw = s_task;
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(raw));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(raw >> 32));
    __syncthreads();
    if ((lo == 0xffffffffu && hi == 0xffffffffu) || iter > a.total_tasks) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int32_t node = int32_t(hi) - 1;
    const int32_t tile = int32_t(lo);
    if (threadIdx.x == 0)
      __hip_atomic_fetch_min(&a.t_first[node], uint64_t(wall_clock64()), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    run_task(a.nodes + node, tile, smem);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    prev = node;
  }
}

struct PCfg {
  int cfg, bm, bn;
};
constexpr PCfg kPersistentGemm[] = {{2, 64, 64}, {3, 32, 32}, {9, 32, 32}, {10, 16, 32}, {12, 16, 16}};

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

ExecNode make_exec_node(int kind, const unsigned char *args, int in_dtype, int out_dtype, int tile) {
  ExecNode n{};
  switch (kind) {
    case 0: {  // GEMM
      GemmArgs g;
      memcpy(&g, args, sizeof(g));
      if (g.M == 0 || g.N == 0) break;
      const bool vec = in_dtype == 0 ? (aligned16(g.A) && aligned16(g.B) && g.lda % 4 == 0 && g.ldb % 4 == 0)
                                     : (aligned16(g.A) && aligned16(g.B) && g.lda % 8 == 0 && g.ldb % 8 == 0);
      // nearest executor tile configuration to the standalone choice
      int cfg;
      switch (tile) {
        case 1: case 2: case 4: case 5: cfg = 2; break;
        case 3: cfg = 3; break;
        case 6: case 7: case 8: case 9: cfg = 9; break;
        case 10: case 11: cfg = 10; break;
        default: cfg = 12; break;
      }
      if (!vec) cfg = 12;
      int bm = 16, bn = 16;
      for (const PCfg &c : kPersistentGemm)
        if (c.cfg == cfg) { bm = c.bm; bn = c.bn; }
      g.tiles_n = (g.N + bn - 1) / bn;
      n.variant = 100 + in_dtype * 50 + cfg * 4 + (vec ? 2 : 0) + (out_dtype == 1 ? 1 : 0);
      n.n_tiles = ((g.M + bm - 1) / bm) * g.tiles_n;
      memcpy(n.args, &g, sizeof(g));
      return n;
    }
    case 2: {  // softmax
      SoftmaxArgs sa;
      memcpy(&sa, args, sizeof(sa));
      if (sa.R == 0 || sa.C == 0) break;
      const int ia = in_dtype ? 8 : 16, oa = out_dtype ? 8 : 16;
      const bool vec = (reinterpret_cast<uintptr_t>(sa.X) % ia == 0) && (reinterpret_cast<uintptr_t>(sa.Y) % oa == 0) &&
                       sa.ldx % 4 == 0 && sa.ldy % 4 == 0;
      int code = 0;
      if (vec) code = sa.C <= 256 ? 1 : sa.C <= 512 ? 2 : sa.C <= 1024 ? 3 : sa.C <= 2048 ? 4 : 0;
      n.variant = 300 + code * 8 + (code ? 4 : 0) + in_dtype * 2 + out_dtype;
      n.n_tiles = (sa.R + 15) / 16;
      memcpy(n.args, &sa, sizeof(sa));
      return n;
    }
    case 1: {  // transpose
      TransArgs ta;
      memcpy(&ta, args, sizeof(ta));
      if (ta.R == 0 || ta.C == 0) break;
      n.variant = 400 + in_dtype;
      n.n_tiles = ((ta.R + 63) / 64) * ((ta.C + 63) / 64);
      memcpy(n.args, &ta, sizeof(ta));
      return n;
    }
    case 3: {  // add
      AddArgs aa;
      memcpy(&aa, args, sizeof(aa));
      if (aa.R == 0 || aa.C == 0) break;
      n.variant = 410 + in_dtype * 2 + out_dtype;
      n.n_tiles = (aa.R + 7) / 8;
      memcpy(n.args, &aa, sizeof(aa));
      return n;
    }
  }
  n.variant = 0;  // nothing to compute: one no-op task keeps the successors' release path
  n.n_tiles = 1;
  return n;
}

hipError_t launch_exec_reset(const ExecArgs &a, hipStream_t stream) {
  const uint32_t n = a.total_tasks > uint32_t(a.n_nodes) ? a.total_tasks : uint32_t(a.n_nodes);
  void *args[] = {const_cast<ExecArgs *>(&a)};
  return hipLaunchKernel((const void *)&exec_reset_kernel, dim3((n + 255) / 256 > 0 ? (n + 255) / 256 : 1),
                         dim3(256), args, 0, stream);
}

hipError_t launch_exec(const ExecArgs &a, int workers, hipStream_t stream) {
  void *args[] = {const_cast<ExecArgs *>(&a)};
  return hipLaunchKernel((const void *)&exec_kernel, dim3(workers > 0 ? workers : 1), dim3(256), args, 0, stream);
}

int exec_max_workers(int device) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)&exec_kernel, 256, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return cus * per_cu;
}

}  // namespace psc
