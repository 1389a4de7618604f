// Device-side DAG executor (policy PSC_DEVICE).
//
// The fine-grained schedules of Sec. IV-B enforce a kernel's precedences with events between host
// queues; here the same precedences are enforced on the GPU, at tile granularity, by one
// persistent kernel.  Every DAG kernel is split into tasks (GEMM output tiles, groups of 16
// softmax rows, 64 x 64 transpose tiles, groups of 8 added rows).  As setup_cq maps kernels to
// command queues ahead of dispatch (Algorithm 1), the host maps tasks to the executor's
// workgroups ahead of the run: a list schedule in a topological order of the kernels, each task
// on the workgroup predicted to be free first.  A workgroup walks its list; before the first
// task of a kernel it waits until every predecessor kernel's completion counter reaches that
// kernel's tile count, and after its last consecutive task of a kernel it adds their number to
// the kernel's counter.  Tiles are published with an agent-scope release (fence, then the
// counter add) and read after an agent-scope acquire (counter loads, then a fence), so data
// written on one XCD is visible to consumers on another.
//
// Progress: every list is a subsequence of one global topological order of the tasks, and the
// grid is no larger than the number of workgroups the GPU holds at once, so once all workgroups
// are resident the earliest unfinished task always has its predecessors done and its workgroup
// at it (a workgroup not yet resident only has to wait for a CU that other work frees).  Every
// wait is also bounded in device-clock time: past the bound (or once another workgroup has
// flagged an error) the workgroup records the error in ctl[0] and leaves its loop, so every wave
// reaches its exit even if a description were wrong.
#include "persistent.hpp"

#include "tiles.hpp"

#include <utility>

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

// Copies rows [tile rpt, (tile + 1) rpt) of a host copy, the region taken as units of 16 bytes
// when every address, pitch and the width allow it (else 2 bytes: rows hold whole FP32 or BF16
// elements), eight units in flight per thread: over the host link one access takes microseconds.
__device__ __forceinline__ void copy_task(const CopyArgs &c, int tile) {
  const int64_t r0 = int64_t(tile) * c.rows_per_task;
  const int64_t nr = min(int64_t(c.rows), r0 + c.rows_per_task) - r0;
  if (nr <= 0) return;
  const bool v16 = ((reinterpret_cast<uintptr_t>(c.src) | reinterpret_cast<uintptr_t>(c.dst) |
                     uint64_t(c.spitch) | uint64_t(c.dpitch) | uint64_t(c.width)) & 15u) == 0;
  const unsigned char *src = c.src + r0 * c.spitch;
  unsigned char *dst = c.dst + r0 * c.dpitch;
  if (v16) {
    const int64_t upr = c.width / 16, n = nr * upr;
    for (int64_t base = threadIdx.x; base < n; base += 256 * 8) {
      uint4 v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t u = base + 256 * j;
        if (u < n) v[j] = *reinterpret_cast<const uint4 *>(src + (u / upr) * c.spitch + (u % upr) * 16);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t u = base + 256 * j;
        if (u < n) *reinterpret_cast<uint4 *>(dst + (u / upr) * c.dpitch + (u % upr) * 16) = v[j];
      }
    }
  } else {
    const int64_t upr = c.width / 2, n = nr * upr;
    for (int64_t base = threadIdx.x; base < n; base += 256 * 8) {
      uint16_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t u = base + 256 * j;
        if (u < n) v[j] = *reinterpret_cast<const uint16_t *>(src + (u / upr) * c.spitch + (u % upr) * 2);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t u = base + 256 * j;
        if (u < n) *reinterpret_cast<uint16_t *>(dst + (u / upr) * c.dpitch + (u % upr) * 2) = v[j];
      }
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

#define PSC_TASK(V, ...)                                \
  case V:                                               \
    if constexpr ((G & exec_variant_group(V)) != 0u) {  \
      __VA_ARGS__;                                      \
      return true;                                      \
    }                                                   \
    return false

constexpr uint32_t kGAll = kGElem | (1u << 14) | 0x1FFFu, kGF32All = kGElem | 0x3Fu,
                   kGBf16All = kGElem | (1u << 14) | 0x1FC0u;
// Wavefronts per SIMD each instance is compiled for, the most its tile functions fit without
// spilling registers to memory: the element-wise instance three (three workgroups' LDS fill a
// CU), the aligned direct-load and attention instances two, the instances with every FP32, every
// BF16 or every tile function one.
constexpr int exec_waves(uint32_t g) {
  return g == kGElem ? 3 : (g == kGAll || g == kGF32All || g == kGBf16All) ? 1 : 2;
}

// Runs one task; false if its variant's tile function is not compiled into this instance (the
// host picks an instance that covers every variant of the DAG, so this is a safeguard).
template <uint32_t G>
__device__ __forceinline__ bool run_task(const ExecNode *ndp, int tile, unsigned char *smem) {
  const ExecNode &nd = *ndp;
  const int v = __builtin_amdgcn_readfirstlane(nd.variant);
  switch (v) {
    PSC_TASK(110, gemm_f32_tile<64, 64, 16, 32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(111, gemm_f32_tile<64, 64, 16, 32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(114, gemm_f32_tile<32, 32, 32, 16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(115, gemm_f32_tile<32, 32, 32, 16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(138, gemm_f32_splitk_tile<32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(139, gemm_f32_splitk_tile<32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(142, gemm_f32_splitk_tile<16, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(143, gemm_f32_splitk_tile<16, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(148, gemm_f32_splitk_tile<16, 16, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(149, gemm_f32_splitk_tile<16, 16, false, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(150, gemm_f32_splitk_tile<16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(151, gemm_f32_splitk_tile<16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(152, gemm_direct_tile<1, false, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(153, gemm_direct_tile<1, false, false, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(154, gemm_direct_tile<1, false, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(155, gemm_direct_tile<1, false, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(158, gemm_direct_tile<2, false, true, false, 8>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(159, gemm_direct_tile<2, false, true, true, 8>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(162, gemm_direct_tile<4, false, true, false, 8>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(163, gemm_direct_tile<4, false, true, true, 8>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(210, gemm_bf16_tile<64, 64, 64, 32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(211, gemm_bf16_tile<64, 64, 64, 32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(266, gemm_bf16_splitk_tile<64, 64, true, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(267, gemm_bf16_splitk_tile<64, 64, true, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(214, gemm_bf16_tile<32, 32, 64, 16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(215, gemm_bf16_tile<32, 32, 64, 16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(238, gemm_bf16_splitk_tile<32, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(239, gemm_bf16_splitk_tile<32, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(242, gemm_bf16_splitk_tile<16, 32, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(243, gemm_bf16_splitk_tile<16, 32, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(248, gemm_bf16_splitk_tile<16, 16, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(249, gemm_bf16_splitk_tile<16, 16, false, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(250, gemm_bf16_splitk_tile<16, 16, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(252, gemm_direct_tile<1, true, false, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(253, gemm_direct_tile<1, true, false, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(254, gemm_direct_tile<1, true, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(255, gemm_direct_tile<1, true, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(258, gemm_direct_tile<2, true, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(259, gemm_direct_tile<2, true, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(262, gemm_direct_tile<4, true, true, false>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(263, gemm_direct_tile<4, true, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(251, gemm_bf16_splitk_tile<16, 16, true, true>(uniform_load<GemmArgs>(nd.args), tile, smem));
    PSC_TASK(300, softmax_task<0, false, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(301, softmax_task<0, false, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(302, softmax_task<0, false, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(303, softmax_task<0, false, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(312, softmax_task<1, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(313, softmax_task<1, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(314, softmax_task<1, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(315, softmax_task<1, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(320, softmax_task<2, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(321, softmax_task<2, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(322, softmax_task<2, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(323, softmax_task<2, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(328, softmax_task<4, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(329, softmax_task<4, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(330, softmax_task<4, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(331, softmax_task<4, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(336, softmax_task<8, true, false, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(337, softmax_task<8, true, false, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(338, softmax_task<8, true, true, false>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(339, softmax_task<8, true, true, true>(uniform_load<SoftmaxArgs>(nd.args), tile));
    PSC_TASK(400, transpose_tile<float>(uniform_load<TransArgs>(nd.args), tile, smem));
    PSC_TASK(401, transpose_tile<uint16_t>(uniform_load<TransArgs>(nd.args), tile, smem));
    PSC_TASK(420, copy_task(uniform_load<CopyArgs>(nd.args), tile));
    PSC_TASK(410, add_task<false, false>(uniform_load<AddArgs>(nd.args), tile));
    PSC_TASK(411, add_task<false, true>(uniform_load<AddArgs>(nd.args), tile));
    PSC_TASK(412, add_task<true, false>(uniform_load<AddArgs>(nd.args), tile));
    PSC_TASK(413, add_task<true, true>(uniform_load<AddArgs>(nd.args), tile));
    default: break;
  }
  return v == 0;  // 0: empty kernel, nothing to compute
}

#undef PSC_TASK

// LDS per workgroup: the largest tile function's -- 48 KiB (FP32 K-split tiles), or the 64 x 64
// BF16 K-split tile's 72 KiB in the instances holding group 14.
constexpr int exec_smem(uint32_t g) {
  return (g & (1u << 14)) ? (gemm_bf16_splitk_smem<64, 64>() > 49152 ? gemm_bf16_splitk_smem<64, 64>() : 49152) : 49152;
}

__global__ __launch_bounds__(256) void exec_reset_kernel(ExecArgs a) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < uint32_t(a.n_nodes)) {
    a.done[i] = 0;
    a.t_first[i] = kExit;
    a.t_last[i] = 0;
  }
  if (i == 0) {
    a.ctl[0] = 0;
    *a.t_start = wall_clock64();
  }
}

// Thread 0: wait until every predecessor of `node` has all its tiles done.  Returns false (and
// flags the error) if a wait exceeds a.max_wait ticks, or if another workgroup flagged one.
__device__ __forceinline__ bool wait_preds(const ExecArgs &a, const ExecNode &nd) {
  for (int32_t j = 0; j < nd.n_pred; ++j) {
    const int32_t p = a.pred[nd.pred_off + j];
    const uint32_t need = uint32_t(a.nodes[p].n_tiles);
    if (__hip_atomic_load(&a.done[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) continue;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(&a.done[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (__hip_atomic_load(&a.ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (wall_clock64() - t0 > a.max_wait) {
        __hip_atomic_fetch_or(&a.ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.host_err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return true;
}

// Every branch that encloses a barrier depends only on wavefront-uniform values: list bounds and
// task entries are read with readfirstlane, and the wait's verdict is broadcast through LDS and
// read the same way, so all 256 threads take the same path each iteration.
template <uint32_t G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(exec_waves(G)))) void exec_kernel(ExecArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[exec_smem(G)];
  __shared__ uint32_t s_ok;
  const int32_t w = __builtin_amdgcn_readfirstlane(int32_t(blockIdx.x));
  const int32_t lo = __builtin_amdgcn_readfirstlane(a.work_off[w]);
  const int32_t hi = __builtin_amdgcn_readfirstlane(a.work_off[w + 1]);
  int32_t checked = -1;  // node whose predecessors this workgroup has seen complete (uniform)
  for (int32_t i = lo; i < hi; ++i) {
    const ExecTask t = uniform_load<ExecTask>(reinterpret_cast<const unsigned char *>(a.tasks + i));
    const ExecNode *nd = a.nodes + t.node;
    if (t.node != checked) {
      if (__builtin_amdgcn_readfirstlane(nd->n_pred) > 0) {
        // One acquire for the workgroup: thread 0 observes the counters, then invalidates this
        // CU's L1 and the XCD's L2 (cache-wide operations) before the barrier releases the
        // other wavefronts to read the predecessors' outputs.
        if (threadIdx.x == 0) {
          const bool ok = wait_preds(a, *nd);
          if (ok) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(0);
          }
          s_ok = ok ? 1u : 0u;
        }
        __syncthreads();
        const uint32_t ok = __builtin_amdgcn_readfirstlane(s_ok);
        if (!ok) break;
      }
      checked = t.node;
    }
    if (threadIdx.x == 0)
      __hip_atomic_fetch_min(&a.t_first[t.node], uint64_t(wall_clock64()), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!run_task<G>(nd, t.tile, smem)) {  // uniform: the variant is read with readfirstlane
      if (threadIdx.x == 0) {
        __hip_atomic_fetch_or(&a.ctl[0], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.host_err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      break;
    }
    if (t.signal > 0) {
      // One release for the workgroup: every wavefront waits until its stores have reached the
      // L2, the barrier orders that before thread 0's release fence (a write-back of the whole
      // L2) and its counter update.
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // the end time is read before the add: a consumer may see the count complete (and stamp
        // its own start) while this returning add is still on its way back
        const uint64_t now = wall_clock64();
        const uint32_t before =
            __hip_atomic_fetch_add(&a.done[t.node], uint32_t(t.signal), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before + uint32_t(t.signal) == uint32_t(nd->n_tiles))
          __hip_atomic_store(&a.t_last[t.node], now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      __syncthreads();  // the next task reuses the LDS
    }
  }
}

// The compiled instances, each the tile-function groups it holds.  A single kernel holding every
// tile function needs the union of their registers (over 400 per lane with the matrix-core
// accumulators, one workgroup per CU); an instance holding only what a DAG uses fits several
// workgroups per CU.  The all-groups instance comes last and covers any DAG.
constexpr uint32_t kInstances[] = {
    kGElem,                                                    // element-wise kernels only
    kGElem | (1u << 3) | (1u << 4) | (1u << 5),                 // FP32: aligned direct-load tiles
    kGElem | (1u << 10) | (1u << 11) | (1u << 12),              // BF16: aligned direct-load tiles
    kGElem | (1u << 0) | (1u << 3) | (1u << 4) | (1u << 5),     // FP32 attention: + 64 x 64 tile
    kGElem | (1u << 6) | (1u << 10) | (1u << 11) | (1u << 12),  // BF16 attention: + 64 x 64 tile
    kGF32All,                                                  // every FP32 tile function
    kGBf16All,                                                 // every BF16 tile function
    kGAll};                                                    // everything
constexpr int kNumInstances = sizeof(kInstances) / sizeof(kInstances[0]);

template <int... I>
constexpr const void *instance_fn(int i, std::integer_sequence<int, I...>) {
  const void *fns[] = {(const void *)&exec_kernel<kInstances[I]>...};
  return fns[i];
}
const void *exec_fn(int i) { return instance_fn(i, std::make_integer_sequence<int, kNumInstances>{}); }

struct PCfg {
  int cfg, bm, bn;
};
constexpr PCfg kPersistentGemm[] = {{2, 64, 64},  {3, 32, 32},  {9, 32, 32}, {10, 16, 32}, {16, 64, 64},
                                    {12, 16, 16}, {13, 16, 16}, {14, 16, 32}, {15, 16, 64}};

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

ExecNode make_exec_node(int kind, const unsigned char *args, int in_dtype, int out_dtype, int tile, int want) {
  ExecNode n{};
  switch (kind) {
    case 0: {  // GEMM
      GemmArgs g;
      memcpy(&g, args, sizeof(g));
      if (g.M == 0 || g.N == 0) break;
      const bool vec = in_dtype == 0 ? (aligned16(g.A) && aligned16(g.B) && g.lda % 4 == 0 && g.ldb % 4 == 0)
                                     : (aligned16(g.A) && aligned16(g.B) && g.lda % 8 == 0 && g.ldb % 8 == 0);
      // The executor's own tile choice: its parallelism comes from kernels running side by side,
      // so a task should carry more work than the standalone kernels' small tiles (made to fill
      // the GPU with one kernel).  `want` is the number of workgroups this kernel can expect:
      // take the largest tile that still gives at least `want` tasks, else the smallest.
      // Candidates, largest first: 64 x 64 (LDS staged), then 16 x 64 / 16 x 32 / 16 x 16
      // direct-load tiles -- one memory round trip per wavefront for its share of K, where an
      // LDS-staged 32 x 32 tile pays one per K step (measured: the 512 x 512 x 512 output
      // projection of the attention DAG in 256 tasks, 3.6% shorter makespan).  A 16-row task
      // re-reads the whole K x N operand for 16 output rows; the 64 x 64 tile reads it a quarter
      // as often, which took the 12-layer DAG's 1024 x 64 x 1024 projections (16 tasks each)
      // from 3.78 to 3.16 ms.  A BF16 64 x 64 task with K >= 256 runs K-split instead (cfg 16:
      // each wavefront multiplies the whole 64 x 64 block over its own quarter of K, one 64-deep
      // chunk at a time, and the four partial blocks are summed through LDS): the staged tile
      // steps through K one 64-deep slice per block barrier, a memory round trip each, sixteen
      // for K = 1024 against four.  (`tile`, the standalone choice, is unused.)
      (void)tile;
      int cfg = -1;
      if (!vec) {
        cfg = in_dtype == 0 ? 13 : 12;
      } else {
        static constexpr int c0[] = {2, 15, 14, 13};
        constexpr int nc = sizeof(c0) / sizeof(c0[0]);
        for (int i = 0; i < nc && cfg < 0; ++i) {
          int bm = 16, bn = 16;
          for (const PCfg &c : kPersistentGemm)
            if (c.cfg == c0[i]) { bm = c.bm; bn = c.bn; }
          const int64_t tiles = int64_t((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
          if (tiles >= want || i == nc - 1) cfg = c0[i];
        }
        if (cfg == 2 && in_dtype == 1 && g.K >= 256) cfg = 16;
      }
      int bm = 16, bn = 16;
      for (const PCfg &c : kPersistentGemm)
        if (c.cfg == cfg) { bm = c.bm; bn = c.bn; }
      g.tiles_n = (g.N + bn - 1) / bn;
      n.variant = 100 + in_dtype * 100 + cfg * 4 + (vec ? 2 : 0) + (out_dtype == 1 ? 1 : 0);
      n.n_tiles = ((g.M + bm - 1) / bm) * g.tiles_n;
      n.tile_m = bm;
      n.tile_n = bn;
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
      n.tile_m = 16;
      n.tile_n = sa.C;
      memcpy(n.args, &sa, sizeof(sa));
      return n;
    }
    case 1: {  // transpose
      TransArgs ta;
      memcpy(&ta, args, sizeof(ta));
      if (ta.R == 0 || ta.C == 0) break;
      n.variant = 400 + in_dtype;
      n.n_tiles = ((ta.R + 63) / 64) * ((ta.C + 63) / 64);
      n.tile_m = 64;
      n.tile_n = 64;
      memcpy(n.args, &ta, sizeof(ta));
      return n;
    }
    case 3: {  // add
      AddArgs aa;
      memcpy(&aa, args, sizeof(aa));
      if (aa.R == 0 || aa.C == 0) break;
      n.variant = 410 + in_dtype * 2 + out_dtype;
      n.n_tiles = (aa.R + 7) / 8;
      n.tile_m = 8;
      n.tile_n = aa.C;
      memcpy(n.args, &aa, sizeof(aa));
      return n;
    }
  }
  n.variant = 0;  // nothing to compute: one no-op task keeps the successors' release path
  n.n_tiles = 1;
  return n;
}

hipError_t launch_exec_reset(const ExecArgs &a, hipStream_t stream) {
  const uint32_t n = uint32_t(a.n_nodes > 1 ? a.n_nodes : 1);
  void *args[] = {const_cast<ExecArgs *>(&a)};
  return hipLaunchKernel((const void *)&exec_reset_kernel, dim3((n + 255) / 256), dim3(256), args, 0, stream);
}

hipError_t launch_exec(const ExecArgs &a, int instance, hipStream_t stream) {
  if (instance < 0 || instance >= kNumInstances) return hipErrorInvalidValue;
  void *args[] = {const_cast<ExecArgs *>(&a)};
  return hipLaunchKernel(exec_fn(instance), dim3(a.n_workers > 0 ? a.n_workers : 1), dim3(256), args, 0, stream);
}

int exec_num_instances() { return kNumInstances; }

uint32_t exec_instance_groups(int instance) {
  return instance >= 0 && instance < kNumInstances ? kInstances[instance] : 0u;
}

int exec_max_workers(int device, int instance) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    (void)hipGetLastError();
    cus = 256;
  }
  if (instance < 0 || instance >= kNumInstances ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, exec_fn(instance), 256, 0) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  return cus * per_cu;
}

}  // namespace psc
