// Standalone gfx950 kernels of the DAG (one tile function call per block; the tile functions live
// in tiles.hpp) and the launch factories that pick a kernel instance for a problem and fill a
// Launch record that the runtime passes to hipLaunchKernel.
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tiles.hpp"

namespace psc {

// Tile choices measured by the autotuner, keyed by (M, N, K, operand dtype, output dtype); the
// automatic choice of make_gemm consults it first.
namespace {
std::mutex g_tile_mu;
std::map<std::tuple<int, int, int, int, int>, int> g_tile_cache;
}  // namespace

void tile_cache_set(int M, int N, int K, int ab, int c, int tile) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  if (tile <= 0) g_tile_cache.erase({M, N, K, ab, c});
  else g_tile_cache[{M, N, K, ab, c}] = tile;
}

int tile_cache_get(int M, int N, int K, int ab, int c) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tile_cache.find({M, N, K, ab, c});
  return it == g_tile_cache.end() ? 0 : it->second;
}

void tile_cache_clear() {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_cache.clear();
}

size_t tile_cache_size() {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  return g_tile_cache.size();
}

std::vector<std::array<int, 6>> tile_cache_entries() {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  std::vector<std::array<int, 6>> out;
  for (const auto &kv : g_tile_cache) {
    const auto &k = kv.first;
    out.push_back({std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), kv.second});
  }
  return out;
}

// ---------------------------------------------------------------------------------------------
// Standalone kernels: one tile function call per 256-thread block.
// ---------------------------------------------------------------------------------------------
template <int BM, int BN, int BK, int WM, int WN, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_f32_smem<BM, BN, BK>()];
  gemm_f32_tile<BM, BN, BK, WM, WN, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <int BM, int BN, int BK, int WM, int WN, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_bf16_smem<BM, BN, BK>()];
  gemm_bf16_tile<BM, BN, BK, WM, WN, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <int TM, int TN, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_f32_splitk_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_f32_splitk_smem<TM, TN>()];
  gemm_f32_splitk_tile<TM, TN, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <int TM, int TN, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_bf16_splitk_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_bf16_splitk_smem<TM, TN>()];
  gemm_bf16_splitk_tile<TM, TN, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <int TM, int TN, int D, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_bf16_deep_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_bf16_deep_smem<TM, TN, D>()];
  gemm_bf16_deep_tile<TM, TN, D, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <bool OUT_BF16>
__global__ __launch_bounds__(512) void gemm_bf16_big_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_bf16_big_smem()];
  // 4-row groups of tiles per XCD (measured 1-3% faster than plain rows at 4096^3 and 8192^3)
  gemm_bf16_big_tile<OUT_BF16>(p, group_tile(xcd_tile(blockIdx.x, gridDim.x), gridDim.x / p.tiles_n, p.tiles_n, 4), smem);
}

template <int WN, bool OUT_BF16>
__global__ __launch_bounds__(128 * WN) void gemm_bf16_w4_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_bf16_w4_smem()];
  gemm_bf16_w4_tile<WN, OUT_BF16>(p, group_tile(xcd_tile(blockIdx.x, gridDim.x), gridDim.x / p.tiles_n, p.tiles_n, 4), smem);
}

template <int FN, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_f32_direct_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_direct_smem<FN, false>()];
  gemm_direct_tile<FN, false, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <int FN, bool VEC, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_bf16_direct_kernel(GemmArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_direct_smem<FN, true>()];
  gemm_direct_tile<FN, true, VEC, OUT_BF16>(p, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <int NV, bool VEC, bool IN_BF16, bool OUT_BF16, bool NT = false, int CW = 4>
__global__ __launch_bounds__(256) void softmax_kernel(SoftmaxArgs p) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row < p.R) softmax_row<NV, VEC, IN_BF16, OUT_BF16, NT, CW>(p, row);
}

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(TransArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[64 * 65 * sizeof(T)];
  transpose_tile<T>(p, blockIdx.x, smem);
}

template <typename T, bool NT>
__global__ __launch_bounds__(256) void transpose_vec_kernel(TransArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[64 * 65 * sizeof(T)];
  transpose_tile_vec<T, NT>(p, blockIdx.x, smem);
}

template <typename T, int TR, int TC, bool NT>
__global__ __launch_bounds__(256) void transpose_rc_kernel(TransArgs p) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[transpose_rc_smem<TR, TC, T>()];
  transpose_rc_tile<T, TR, TC, NT>(p, blockIdx.x, smem);
}

template <bool IN_BF16, bool OUT_BF16>
__global__ __launch_bounds__(256) void add_kernel(AddArgs p) {
  add_block<IN_BF16, OUT_BF16>(p, blockIdx.x);
}

template <bool IN_BF16, bool OUT_BF16, bool NT = false>
__global__ __launch_bounds__(256) void add_vec_kernel(AddArgs p) {
  add_block_vec<IN_BF16, OUT_BF16, NT>(p, blockIdx.x);
}

// ---------------------------------------------------------------------------------------------
// Launch factories
// ---------------------------------------------------------------------------------------------
namespace {

// Softmax and transpose launches whose output is at least this large (bytes, the size of the
// last-level cache) read and write with streaming hints: neither operand would stay cached for a
// consumer.
constexpr int64_t kStreamBytes = int64_t(256) << 20;

template <typename Args>
void set_args(Launch &L, const Args &a) {
  static_assert(sizeof(Args) <= sizeof(L.args), "argument struct too large");
  memcpy(L.args, &a, sizeof(Args));
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

struct TileCfg {
  int bm, bn;
  bool splitk;  // K split across the block's four wavefronts
};
// 1..5: large tiles; 6..12: K split over the wavefronts, operands through LDS; 13..15: K split
// over the wavefronts, operands read directly into matrix-core registers (16-row tiles);
// 16: 256 x 256 BF16 tile, eight wavefronts, 512 threads (for FP32 operands it means tile 1);
// 17..19: BF16 K split over the wavefronts with each wavefront's K share loaded at once (16 x 16
// and 16 x 32 with four 64-deep chunks in flight, 32 x 32 with two); for FP32 operands they mean
// the staged split-K tiles of the same shape (12, 10, 9).

// GEMM tile configurations (index = psc_kernel_params.tile; 0 = automatic)
constexpr TileCfg kTiles[] = {{0, 0, false},     {128, 128, false}, {64, 64, false},  {32, 32, false},
                              {128, 64, false},  {64, 128, false},  {64, 64, true},   {32, 64, true},
                              {64, 32, true},    {32, 32, true},    {16, 32, true},   {32, 16, true},
                              {16, 16, true},    {16, 16, true},    {16, 32, true},   {16, 64, true},
                              {256, 256, false}, {16, 16, true},    {16, 32, true},   {32, 32, true},
                              {256, 256, false}, {256, 256, false}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

#define PSC_VO(KERNEL, ...)                                                                     \
  (vec ? (obf ? (const void *)&KERNEL<__VA_ARGS__, true, true> : (const void *)&KERNEL<__VA_ARGS__, true, false>) \
       : (obf ? (const void *)&KERNEL<__VA_ARGS__, false, true> : (const void *)&KERNEL<__VA_ARGS__, false, false>))

const void *gemm_fn(int ab_dtype, int tile, bool vec, bool obf) {
  if (ab_dtype == 0) {
    switch (tile) {
      case 1: return PSC_VO(gemm_f32_kernel, 128, 128, 16, 64, 64);
      case 2: return PSC_VO(gemm_f32_kernel, 64, 64, 16, 32, 32);
      case 3: return PSC_VO(gemm_f32_kernel, 32, 32, 32, 16, 16);
      case 4: return PSC_VO(gemm_f32_kernel, 128, 64, 16, 64, 32);
      case 5: return PSC_VO(gemm_f32_kernel, 64, 128, 16, 32, 64);
      case 6: return PSC_VO(gemm_f32_splitk_kernel, 64, 64);
      case 7: return PSC_VO(gemm_f32_splitk_kernel, 32, 64);
      case 8: return PSC_VO(gemm_f32_splitk_kernel, 64, 32);
      case 9: return PSC_VO(gemm_f32_splitk_kernel, 32, 32);
      case 10: return PSC_VO(gemm_f32_splitk_kernel, 16, 32);
      case 11: return PSC_VO(gemm_f32_splitk_kernel, 32, 16);
      case 12: return PSC_VO(gemm_f32_splitk_kernel, 16, 16);
      case 13: return PSC_VO(gemm_f32_direct_kernel, 1);
      case 14: return PSC_VO(gemm_f32_direct_kernel, 2);
      case 15: return PSC_VO(gemm_f32_direct_kernel, 4);
    }
  } else {
    switch (tile) {
      case 1: return PSC_VO(gemm_bf16_kernel, 128, 128, 64, 64, 64);
      case 2: return PSC_VO(gemm_bf16_kernel, 64, 64, 64, 32, 32);
      case 3: return PSC_VO(gemm_bf16_kernel, 32, 32, 64, 16, 16);
      case 4: return PSC_VO(gemm_bf16_kernel, 128, 64, 64, 64, 32);
      case 5: return PSC_VO(gemm_bf16_kernel, 64, 128, 64, 32, 64);
      case 6: return PSC_VO(gemm_bf16_splitk_kernel, 64, 64);
      case 7: return PSC_VO(gemm_bf16_splitk_kernel, 32, 64);
      case 8: return PSC_VO(gemm_bf16_splitk_kernel, 64, 32);
      case 9: return PSC_VO(gemm_bf16_splitk_kernel, 32, 32);
      case 10: return PSC_VO(gemm_bf16_splitk_kernel, 16, 32);
      case 11: return PSC_VO(gemm_bf16_splitk_kernel, 32, 16);
      case 12: return PSC_VO(gemm_bf16_splitk_kernel, 16, 16);
      case 13: return PSC_VO(gemm_bf16_direct_kernel, 1);
      case 14: return PSC_VO(gemm_bf16_direct_kernel, 2);
      case 15: return PSC_VO(gemm_bf16_direct_kernel, 4);
      case 16: return obf ? (const void *)&gemm_bf16_big_kernel<true> : (const void *)&gemm_bf16_big_kernel<false>;
      case 17: return PSC_VO(gemm_bf16_deep_kernel, 16, 16, 4);
      case 18: return PSC_VO(gemm_bf16_deep_kernel, 16, 32, 4);
      case 19: return PSC_VO(gemm_bf16_deep_kernel, 32, 32, 2);
      case 20: return obf ? (const void *)&gemm_bf16_w4_kernel<2, true> : (const void *)&gemm_bf16_w4_kernel<2, false>;
      case 21: return obf ? (const void *)&gemm_bf16_w4_kernel<4, true> : (const void *)&gemm_bf16_w4_kernel<4, false>;
    }
  }
  return nullptr;
}
#undef PSC_VO

int64_t tiles_of(int t, int M, int N) {
  return int64_t((M + kTiles[t].bm - 1) / kTiles[t].bm) * ((N + kTiles[t].bn - 1) / kTiles[t].bn);
}

}  // namespace

int gemm_num_tiles() { return kNumTiles; }

// (external linkage: the AQL dispatcher finds kernels by the name of their host handle)
__global__ __launch_bounds__(64) void mark_kernel(uint64_t *slot) {
  if (threadIdx.x == 0) *slot = wall_clock64();
}

void make_mark(Launch &L, uint64_t *slot) {
  L = Launch{};
  L.func = reinterpret_cast<const void *>(&mark_kernel);
  L.grid = dim3(1, 1, 1);
  L.block = dim3(64, 1, 1);
  std::memcpy(L.args, &slot, sizeof(slot));
}

namespace {
struct FillArgs {
  uint32_t *p;
  int64_t words;
  int32_t bf16;
  uint32_t seed;
};
// 32-bit integer mix (xor-shift-multiply rounds); only its spread matters here
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352du;
  x ^= x >> 15; x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__global__ __launch_bounds__(256) void fill_kernel(FillArgs a) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < a.words; i += int64_t(gridDim.x) * 256) {
    const uint32_t h = mix32(uint32_t(i) ^ mix32(uint32_t(i >> 32) + a.seed));
    const float lo = float(h & 0xffffu) * (1.0f / 32768.0f) - 1.0f, hi = float(h >> 16) * (1.0f / 32768.0f) - 1.0f;
    a.p[i] = a.bf16 ? uint32_t(f32_to_bf16(lo)) | (uint32_t(f32_to_bf16(hi)) << 16) : __float_as_uint(lo);
  }
}
}  // namespace

void make_fill(Launch &L, void *p, int64_t bytes, int bf16, uint32_t seed) {
  L = Launch{};
  const FillArgs a{static_cast<uint32_t *>(p), bytes / 4, bf16, seed};
  L.func = reinterpret_cast<const void *>(&fill_kernel);
  L.grid = dim3(unsigned(std::min<int64_t>(4096, std::max<int64_t>(1, (a.words + 255) / 256))), 1, 1);
  L.block = dim3(256, 1, 1);
  L.empty = a.words == 0;
  std::memcpy(L.args, &a, sizeof(a));
}

int gemm_auto_tile(int M, int N, int K, int dtype) {
  // BF16 shapes of whole 256 x 256 tiles that fill the chip: the four-wavefront tile with direct
  // global-to-LDS copies (the launch factory still checks alignment).  Otherwise, enough output tiles to fill the chip: the
  // large-tile kernels; else the split-K kernels, which run four wavefronts per tile along K: the
  // largest tile that still yields >= 256 blocks (>= 128 when K is long), else the smallest tile.
  if (dtype == 1 && M % 256 == 0 && N % 256 == 0 && K % 64 == 0 && K > 0 && tiles_of(20, M, N) >= 256) return 20;
  for (int t : {1, 4, 5, 2})
    if (tiles_of(t, M, N) >= 256) return t;
  const int64_t want = K >= 256 ? 128 : 256;
  for (int t : {6, 7, 8, 9, 10, 11, 12})
    if (tiles_of(t, M, N) >= want) return t;
  return 12;
}

bool make_gemm(Launch &L, GemmArgs a, int ab_dtype, int c_dtype, int tile) {
  if (tile <= 0 || tile >= kNumTiles) tile = tile_cache_get(a.M, a.N, a.K, ab_dtype, c_dtype);
  if (tile <= 0 || tile >= kNumTiles) tile = gemm_auto_tile(a.M, a.N, a.K, ab_dtype);
  if ((tile == 16 || tile >= 20) && ab_dtype == 0) tile = 1;  // the 256 x 256 tiles exist for BF16 only
  if (ab_dtype == 0 && tile >= 17 && tile <= 19) tile = tile == 17 ? 12 : tile == 18 ? 10 : 9;  // BF16 only
  if (tile == 16 || tile >= 20) {  // whole tiles, aligned operands only
    const bool fits = a.M % 256 == 0 && a.N % 256 == 0 && a.K % 64 == 0 && a.K > 0 && aligned16(a.A) &&
                      aligned16(a.B) && a.lda % 8 == 0 && a.ldb % 8 == 0;
    if (!fits) tile = 4;
  }
  const int bm = kTiles[tile].bm, bn = kTiles[tile].bn;
  a.tiles_n = (a.N + bn - 1) / bn;
  const int tiles_m = (a.M + bm - 1) / bm;
  const bool obf = c_dtype == 1;
  const bool vec = ab_dtype == 0
                       ? (aligned16(a.A) && aligned16(a.B) && a.lda % 4 == 0 && a.ldb % 4 == 0)
                       : (aligned16(a.A) && aligned16(a.B) && a.lda % 8 == 0 && a.ldb % 8 == 0);
  const void *fn = gemm_fn(ab_dtype, tile, vec, obf);
  if (!fn) return false;
  L.func = fn;
  L.grid = dim3(unsigned(int64_t(tiles_m) * a.tiles_n), 1, 1);
  L.block = dim3(tile == 16 || tile == 21 ? 512 : 256, 1, 1);  // four wavefronts, eight for tiles 16 and 21
  L.shmem = 0;
  L.empty = a.M == 0 || a.N == 0;
  L.tile = tile;
  set_args(L, a);
  return true;
}

bool make_softmax(Launch &L, SoftmaxArgs a, int in_dtype, int out_dtype) {
  const bool ib = in_dtype == 1, ob = out_dtype == 1;
  const int in_align = ib ? 8 : 16, out_align = ob ? 8 : 16;
  const bool vec = (reinterpret_cast<uintptr_t>(a.X) % in_align == 0) &&
                   (reinterpret_cast<uintptr_t>(a.Y) % out_align == 0) && a.ldx % 4 == 0 && a.ldy % 4 == 0;
  int nv = 0;
  if (a.C <= 256) nv = 1;
  else if (a.C <= 512) nv = 2;
  else if (a.C <= 1024) nv = 4;
  else if (a.C <= 2048) nv = 8;
  const bool nt = vec && nv > 0 && int64_t(a.R) * a.C * (ob ? 2 : 4) >= kStreamBytes;
  // bf16 input in 16-byte chunks of eight where both operands allow it
  const bool w16 = vec && ib && nv >= 2 && aligned16(a.X) && aligned16(a.Y) && a.ldx % 8 == 0 && a.ldy % 8 == 0;
#define PSC_SMB(NV, NT, W)                                                                          \
  (w16 ? (ob ? (const void *)&softmax_kernel<NV, true, true, true, NT, W> : (const void *)&softmax_kernel<NV, true, true, false, NT, W>) \
       : (ob ? (const void *)&softmax_kernel<NV, true, true, true, NT> : (const void *)&softmax_kernel<NV, true, true, false, NT>))
#define PSC_SM4(NV, NT, W)                                                                          \
  (ib ? PSC_SMB(NV, NT, W)                                                                          \
      : (ob ? (const void *)&softmax_kernel<NV, true, false, true, NT> : (const void *)&softmax_kernel<NV, true, false, false, NT>))
#define PSC_SMS(NV)                                                                                 \
  (ib ? (ob ? (const void *)&softmax_kernel<NV, false, true, true> : (const void *)&softmax_kernel<NV, false, true, false>) \
      : (ob ? (const void *)&softmax_kernel<NV, false, false, true> : (const void *)&softmax_kernel<NV, false, false, false>))
#define PSC_SM(NV, W) (vec ? (nt ? PSC_SM4(NV, true, W) : PSC_SM4(NV, false, W)) : PSC_SMS(NV))
  switch (nv) {
    case 1: L.func = PSC_SM(1, 4); break;   // (no eight-wide chunks for rows of at most 256)
    case 2: L.func = PSC_SM(2, 8); break;
    case 4: L.func = PSC_SM(4, 8); break;
    case 8: L.func = PSC_SM(8, 8); break;
    default: L.func = PSC_SMS(0); break;
  }
#undef PSC_SM
#undef PSC_SMS
#undef PSC_SM4
#undef PSC_SMB
  L.grid = dim3(unsigned((a.R + 3) / 4), 1, 1);
  L.block = dim3(256, 1, 1);
  L.shmem = 0;
  L.empty = a.R == 0 || a.C == 0;
  set_args(L, a);
  return true;
}

#define PSC_TRC(T, TR, TC) (nt ? (const void *)&transpose_rc_kernel<T, TR, TC, true> : (const void *)&transpose_rc_kernel<T, TR, TC, false>)

// tile: 1 64 x 64, 2 64 x 128, 3 128 x 64, 4 64 x 256 (rows x columns of the input); the
// rectangular tiles need aligned operands (else 64 x 64).  Automatic (0): 64 x 256 for streaming
// sizes, 64 x 64 otherwise.  Measured on a 16384^2 transpose with streaming hints (HBM fraction,
// FP32 / BF16): 64 x 256 70.2-70.5% / 71.2-72.1%; 128 x 256 (BF16) 71.2%; 64 x 128 66.9% / 67.9%;
// 64 x 64 65.4% / 67.1%; 128 x 128 66.3% / 68.2%; 32 x 256 68.7-68.9% / 52.5%; 64 x 512 (BF16)
// 68.3%; without the hints every shape 1.5-4 points lower.
bool make_transpose(Launch &L, TransArgs a, int dtype, int tile) {
  const int64_t v = dtype == 1 ? 8 : 4;  // elements per 16-byte vector
  const bool vec = aligned16(a.A) && aligned16(a.B) && a.lda % v == 0 && a.ldb % v == 0;
  const bool nt = int64_t(a.R) * a.C * (dtype == 1 ? 2 : 4) >= kStreamBytes;
  if (tile < 1 || tile > 4) tile = nt ? 4 : 1;
  if (!vec) tile = 1;
  int tr = 64, tcl = 64;
  if (tile == 1 && vec)
    L.func = dtype == 1 ? (nt ? (const void *)&transpose_vec_kernel<uint16_t, true> : (const void *)&transpose_vec_kernel<uint16_t, false>)
                        : (nt ? (const void *)&transpose_vec_kernel<float, true> : (const void *)&transpose_vec_kernel<float, false>);
  else if (tile == 1)
    L.func = dtype == 1 ? (const void *)&transpose_kernel<uint16_t> : (const void *)&transpose_kernel<float>;
  else if (tile == 2)
    L.func = dtype == 1 ? PSC_TRC(uint16_t, 64, 128) : PSC_TRC(float, 64, 128), tcl = 128;
  else if (tile == 4)
    L.func = dtype == 1 ? PSC_TRC(uint16_t, 64, 256) : PSC_TRC(float, 64, 256), tcl = 256;
  else
    L.func = dtype == 1 ? PSC_TRC(uint16_t, 128, 64) : PSC_TRC(float, 128, 64), tr = 128;
  L.tile = tile;
  L.grid = dim3(unsigned(int64_t((a.R + tr - 1) / tr) * ((a.C + tcl - 1) / tcl)), 1, 1);
  L.block = dim3(256, 1, 1);
  L.shmem = 0;
  L.empty = a.R == 0 || a.C == 0;
  set_args(L, a);
  return true;
}

bool make_add(Launch &L, AddArgs a, int in_dtype, int out_dtype) {
  const bool ib = in_dtype == 1, ob = out_dtype == 1;
  const bool vec = aligned16(a.A) && aligned16(a.B) && aligned16(a.Cp) && a.lda % 8 == 0 && a.ldb % 8 == 0 &&
                   a.ldc % 8 == 0;
  if (vec) {
    // plain loads and stores: streaming hints measured slower for the two-input add
    L.func = ib ? (ob ? (const void *)&add_vec_kernel<true, true> : (const void *)&add_vec_kernel<true, false>)
                : (ob ? (const void *)&add_vec_kernel<false, true> : (const void *)&add_vec_kernel<false, false>);
    L.grid = dim3(unsigned(int64_t((a.C + 2047) / 2048) * a.R), 1, 1);
  } else {
    L.func = ib ? (ob ? (const void *)&add_kernel<true, true> : (const void *)&add_kernel<true, false>)
                : (ob ? (const void *)&add_kernel<false, true> : (const void *)&add_kernel<false, false>);
    L.grid = dim3(unsigned(int64_t((a.C + 255) / 256) * a.R), 1, 1);
  }
  L.block = dim3(256, 1, 1);
  L.shmem = 0;
  L.empty = a.R == 0 || a.C == 0;
  set_args(L, a);
  return true;
}

}  // namespace psc
