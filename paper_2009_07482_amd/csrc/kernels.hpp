// Argument records and launch factories of the gfx950 kernel library (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <vector>

namespace psc {

struct GemmArgs {           // C (M x N) = alpha * A (M x K) * B (K x N), row-major, leading dims
  const void *A;
  const void *B;
  void *C;
  int64_t lda, ldb, ldc;    // in elements
  int32_t M, N, K;
  float alpha;
  int32_t tiles_n;          // filled by make_gemm
  int32_t pad;
};

struct SoftmaxArgs {        // Y (R x C) = row-softmax(X)
  const void *X;
  void *Y;
  int64_t ldx, ldy;
  int32_t R, C;
};

struct TransArgs {          // B (C x R) = A (R x C)^T
  const void *A;
  void *B;
  int64_t lda, ldb;
  int32_t R, C;
};

struct AddArgs {            // Cp (R x C) = A + B
  const void *A;
  const void *B;
  void *Cp;
  int64_t lda, ldb, ldc;
  int32_t R, C;
};

// A prepared kernel launch: hipLaunchKernel(func, grid, block, {args}, shmem, stream).
struct Launch {
  const void *func = nullptr;
  dim3 grid, block;
  unsigned shmem = 0;
  bool empty = false;       // nothing to compute (an empty operand): skip the launch
  int tile = 0;             // GEMM tile configuration used
  alignas(16) unsigned char args[96];
};

// dtype codes: 0 = f32, 1 = bf16
bool make_gemm(Launch &L, GemmArgs a, int ab_dtype, int c_dtype, int tile);
bool make_softmax(Launch &L, SoftmaxArgs a, int in_dtype, int out_dtype);
bool make_transpose(Launch &L, TransArgs a, int dtype, int tile = 0);
bool make_add(Launch &L, AddArgs a, int in_dtype, int out_dtype);
int gemm_num_tiles();
// One-thread kernel that stores the device wall clock (wall_clock64) to *slot.
void make_mark(Launch &L, uint64_t *slot);
// Fills bytes / 4 32-bit words at p with values uniform in [-1, 1) from a hash of (index, seed):
// one FP32 value per word, or (bf16) two bfloat16 values.  Timing operands for the autotuner
// (the matrix cores' power, and with it the clock, depends on the data).
void make_fill(Launch &L, void *p, int64_t bytes, int bf16, uint32_t seed);
void tile_cache_set(int M, int N, int K, int ab, int c, int tile);
int tile_cache_get(int M, int N, int K, int ab, int c);
void tile_cache_clear();
size_t tile_cache_size();
std::vector<std::array<int, 6>> tile_cache_entries();   // (M, N, K, operand dtype, output dtype, tile)
int gemm_auto_tile(int M, int N, int K, int dtype);

}  // namespace psc
