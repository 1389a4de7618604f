// Device tile functions of the gfx950 kernel library: GEMM on the matrix cores (FP32 and BF16
// operands, FP32 accumulation), row softmax with wavefront reductions, LDS-tiled transpose and
// element-wise add.  Each function computes one block-sized piece of its kernel (a GEMM output
// tile, one softmax row per wavefront, a 64 x 64 transpose tile, a 256-column row segment) with
// 256 threads and caller-provided LDS, so the same code serves the standalone kernels
// (kernels.hip, one piece per block) and the persistent DAG executor (persistent.hip, pieces
// pulled from a device work queue).  Every function handles ragged shapes with bounds checks;
// vector loads are used only where the host has checked alignment.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>

#include "kernels.hpp"

namespace psc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// 16- and 8-byte global loads and stores.  NT: with the non-temporal (streaming) hint, for
// operands far larger than the last-level cache, which are read or written once and would only
// evict data still to be used.
template <bool NT>
__device__ __forceinline__ u32x4 load16(const void *src) {
  if constexpr (NT) return __builtin_nontemporal_load(static_cast<const u32x4 *>(src));
  else return *static_cast<const u32x4 *>(src);
}
template <bool NT>
__device__ __forceinline__ u32x2 load8(const void *src) {
  if constexpr (NT) return __builtin_nontemporal_load(static_cast<const u32x2 *>(src));
  else return *static_cast<const u32x2 *>(src);
}
template <bool NT>
__device__ __forceinline__ void store16(void *dst, u32x4 w) {
  if constexpr (NT) __builtin_nontemporal_store(w, static_cast<u32x4 *>(dst));
  else *static_cast<u32x4 *>(dst) = w;
}
template <bool NT>
__device__ __forceinline__ void store8(void *dst, u32x2 w) {
  if constexpr (NT) __builtin_nontemporal_store(w, static_cast<u32x2 *>(dst));
  else *static_cast<u32x2 *>(dst) = w;
}

// ---------------------------------------------------------------------------------------------
// bfloat16 <-> float.  A bfloat16 is the upper 16 bits of an IEEE binary32; conversion from
// float rounds to nearest, ties to even, on those 16 bits; NaN stays a (quiet) NaN.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

template <bool BF16>
__device__ __forceinline__ float load_elem(const void *p, int64_t i) {
  if constexpr (BF16) return bf16_to_f32(static_cast<const uint16_t *>(p)[i]);
  else return static_cast<const float *>(p)[i];
}
template <bool BF16>
__device__ __forceinline__ void store_elem(void *p, int64_t i, float v) {
  if constexpr (BF16) static_cast<uint16_t *>(p)[i] = f32_to_bf16(v);
  else static_cast<float *>(p)[i] = v;
}

// ---------------------------------------------------------------------------------------------
// XCD-aware tile order.  The GPU deals workgroups round robin over its 8 XCDs (workgroup b runs on
// XCD b % 8), and each XCD has its own L2.  Giving every XCD a contiguous range of the row-major
// tile order keeps the tiles that share an A row panel (consecutive tile indices) on one XCD, so
// the panel is fetched from HBM once instead of once per XCD.  A bijection of [0, n): correct for
// any XCD count; only the locality assumes 8.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int X = 8;
  const int per = n / X, rem = n % X;
  const int x = b % X, i = b / X;
  return x * per + (x < rem ? x : rem) + i;
}

// Grouped tile order: consecutive tile indices walk G tile rows column by column, so the tiles an
// XCD runs at one time form a G-row block (4 x 8 for 32 compute units) that shares G row panels
// of A and a few column panels of B in that XCD's L2, instead of one or two full tile rows that
// each need every column panel of B.
__device__ __forceinline__ int group_tile(int t, int tiles_m, int tiles_n, int G) {
  const int per = G * tiles_n, g = t / per, w = t % per;
  const int rows = min(G, tiles_m - g * G);
  return (g * G + w % rows) * tiles_n + w / rows;
}

// ---------------------------------------------------------------------------------------------
// GEMM, C = alpha * A * B.  Block tile BM x BN, K step BK, each wavefront a WM x WN sub-tile made
// of 16 x 16 matrix-core blocks.  Operand tiles are staged through LDS with padded pitches so that
// the per-lane fragment reads hit distinct banks.
//
// Matrix-core operand layouts (16 x 16 output block, lane l of 64):
//   v_mfma_f32_16x16x4_f32:   A: row l%16, k l/16          B: col l%16, k l/16
//   v_mfma_f32_16x16x32_bf16: A: row l%16, k 8*(l/16)+e    B: col l%16, k 8*(l/16)+e  (e < 8)
//   accumulator (both): element r of lane l is row 4*(l/16)+r, col l%16.
// ---------------------------------------------------------------------------------------------
template <int BM, int BN, int BK>
constexpr int gemm_f32_smem() {
  return 4 * BK * ((((BM + 63) / 64) * 64 + 16) + (((BN + 63) / 64) * 64 + 16));
}

template <int BM, int BN, int BK, int WM, int WN, bool VEC, bool OUT_BF16>
__device__ __forceinline__ void gemm_f32_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  static_assert(64 * (BM / WM) * (BN / WN) == 256, "four wavefronts per block");
  constexpr int NWN = BN / WN, NT = 64 * (BM / WM) * NWN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int SA = ((BM + 63) / 64) * 64 + 16;  // pitch = 16 (mod 64) dwords
  constexpr int SB = ((BN + 63) / 64) * 64 + 16;
  // A is written transposed (k-major), four k rows per float4: with the pitch above those rows
  // start in the same banks, so A's column index is XOR-swizzled by the k row's group of four
  // (bits 4-5): the four writes of a float4 land 16 banks apart, and a fragment read, whose
  // lanes share k / 4, still covers 64 distinct banks.
  auto swz = [](int k) { return ((k >> 2) & 3) << 4; };
  constexpr int UA = BM * (BK / 4), UB = BK * (BN / 4);  // float4 units per tile
  constexpr int NA = (UA + NT - 1) / NT, NB = (UB + NT - 1) / NT;
  float *As = reinterpret_cast<float *>(smem);  // k-major: As[k][m]
  float *Bs = As + BK * SA;                     // k-major: Bs[k][n]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const float *A = static_cast<const float *>(p.A);
  const float *B = static_cast<const float *>(p.B);

  float4 ra[NA], rb[NB];
  auto load = [&](int k0) {  // next tile into registers (zero outside the matrices)
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int u = tid + NT * j, r = u / (BK / 4), c = (u % (BK / 4)) * 4;
      const int gr = m0 + r, gc = k0 + c;
      if (u < UA && VEC && gr < p.M && gc + 3 < p.K) {
        ra[j] = *reinterpret_cast<const float4 *>(A + int64_t(gr) * p.lda + gc);
      } else {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[e] = (u < UA && gr < p.M && gc + e < p.K) ? A[int64_t(gr) * p.lda + gc + e] : 0.f;
        ra[j] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int u = tid + NT * j, r = u / (BN / 4), c = (u % (BN / 4)) * 4;
      const int gr = k0 + r, gc = n0 + c;
      if (u < UB && VEC && gr < p.K && gc + 3 < p.N) {
        rb[j] = *reinterpret_cast<const float4 *>(B + int64_t(gr) * p.ldb + gc);
      } else {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          v[e] = (u < UB && gr < p.K && gc + e < p.N) ? B[int64_t(gr) * p.ldb + gc + e] : 0.f;
        rb[j] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  };

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  load(0);
  for (int k0 = 0; k0 < p.K; k0 += BK) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int u = tid + NT * j, r = u / (BK / 4), c = (u % (BK / 4)) * 4;
      if (u < UA) {
        As[(c + 0) * SA + (r ^ swz(c + 0))] = ra[j].x;
        As[(c + 1) * SA + (r ^ swz(c + 1))] = ra[j].y;
        As[(c + 2) * SA + (r ^ swz(c + 2))] = ra[j].z;
        As[(c + 3) * SA + (r ^ swz(c + 3))] = ra[j].w;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int u = tid + NT * j, r = u / (BN / 4), c = (u % (BN / 4)) * 4;
      if (u < UB) *reinterpret_cast<float4 *>(&Bs[r * SB + c]) = rb[j];
    }
    __syncthreads();
    if (k0 + BK < p.K) load(k0 + BK);  // in flight while this tile is multiplied
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + (lane >> 4);
      float a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[k * SA + ((wm * WM + i * 16 + (lane & 15)) ^ swz(k))];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[k * SB + wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + r;
        if (row < p.M && col < p.N) store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * acc[i][j][r]);
      }
    }
}

template <int BM, int BN, int BK>
constexpr int gemm_bf16_smem() {
  return 2 * (BM + BN) * (BK + 8);
}

template <int BM, int BN, int BK, int WM, int WN, bool VEC, bool OUT_BF16>
__device__ __forceinline__ void gemm_bf16_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  static_assert(BK % 32 == 0, "BK must be a multiple of the 32-deep matrix-core step");
  static_assert(64 * (BM / WM) * (BN / WN) == 256, "four wavefronts per block");
  constexpr int NWN = BN / WN, NT = 64 * (BM / WM) * NWN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int KP = BK + 8;  // row pitch in bf16 elements: (KP/2) = 4 * odd dwords
  constexpr int UA = BM * (BK / 8), UB = (BK / 2) * (BN / 8);
  constexpr int NA = (UA + NT - 1) / NT, NB = (UB + NT - 1) / NT;
  uint16_t *As = reinterpret_cast<uint16_t *>(smem);  // As[m][k]
  uint16_t *Bt = As + BM * KP;                         // Bt[n][k] (B transposed)

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const uint16_t *A = static_cast<const uint16_t *>(p.A);
  const uint16_t *B = static_cast<const uint16_t *>(p.B);

  uint4 ra[NA], rb0[NB], rb1[NB];
  auto load = [&](int k0) {
    // A: units of 8 consecutive k in one row
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int u = tid + NT * j, r = u / (BK / 8), c = (u % (BK / 8)) * 8;
      const int gr = m0 + r, gc = k0 + c;
      if (u < UA && VEC && gr < p.M && gc + 7 < p.K) {
        ra[j] = *reinterpret_cast<const uint4 *>(A + int64_t(gr) * p.lda + gc);
      } else {
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (u < UA && gr < p.M && gc + e < p.K) ? A[int64_t(gr) * p.lda + gc + e] : 0;
        memcpy(&ra[j], v, 16);
      }
    }
    // B: units of two consecutive k rows x 8 consecutive n, stored transposed as (k, k+1) pairs
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int u = tid + NT * j, kp = u / (BN / 8), c = (u % (BN / 8)) * 8;
      const int gk = k0 + 2 * kp, gc = n0 + c;
      if (u < UB && VEC && gk + 1 < p.K && gc + 7 < p.N) {
        rb0[j] = *reinterpret_cast<const uint4 *>(B + int64_t(gk) * p.ldb + gc);
        rb1[j] = *reinterpret_cast<const uint4 *>(B + int64_t(gk + 1) * p.ldb + gc);
      } else {
        uint16_t lo[8], hi[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          lo[e] = (u < UB && gk < p.K && gc + e < p.N) ? B[int64_t(gk) * p.ldb + gc + e] : 0;
          hi[e] = (u < UB && gk + 1 < p.K && gc + e < p.N) ? B[int64_t(gk + 1) * p.ldb + gc + e] : 0;
        }
        memcpy(&rb0[j], lo, 16);
        memcpy(&rb1[j], hi, 16);
      }
    }
  };

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  load(0);
  for (int k0 = 0; k0 < p.K; k0 += BK) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int u = tid + NT * j, r = u / (BK / 8), c = (u % (BK / 8)) * 8;
      if (u < UA) *reinterpret_cast<uint4 *>(&As[r * KP + c]) = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int u = tid + NT * j, kp = u / (BN / 8), c = (u % (BN / 8)) * 8;
      if (u < UB) {
        uint16_t lo[8], hi[8];
        memcpy(lo, &rb0[j], 16);
        memcpy(hi, &rb1[j], 16);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          *reinterpret_cast<uint32_t *>(&Bt[(c + e) * KP + 2 * kp]) = uint32_t(lo[e]) | (uint32_t(hi[e]) << 16);
      }
    }
    __syncthreads();
    if (k0 + BK < p.K) load(k0 + BK);  // in flight while this tile is multiplied
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      bf16x8 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm * WM + i * 16 + (lane & 15)) * KP + kq]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(&Bt[(wn * WN + j * 16 + (lane & 15)) * KP + kq]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + r;
        if (row < p.M && col < p.N) store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * acc[i][j][r]);
      }
    }
}

// ---------------------------------------------------------------------------------------------
// Small-output GEMM with the K dimension split across the block's four wavefronts.  The block
// owns a TM x TN output tile; wavefront w multiplies K chunks w, w+4, w+8, ... into its own
// accumulators (each wavefront stages its chunk in a private LDS region), prefetching the next
// chunk into registers while it multiplies the current one.  The four partial tiles are then
// summed through LDS in the fixed order w = 0, 1, 2, 3, so results do not depend on timing.
// Trip counts are uniform across wavefronts (chunks past the end are zero-filled), so every
// __syncthreads is reached by all of them.
// ---------------------------------------------------------------------------------------------
template <int TM>
struct SkPitch {  // k-major FP32 pitch = 16 (mod 32) dwords: conflict-free fragment reads
  static constexpr int value = (TM % 32 == 0) ? TM + 16 : TM + 32;
};

template <int TM, int TN>
constexpr int gemm_f32_splitk_smem() {
  return 4 * (4 * 32 * (SkPitch<TM>::value + SkPitch<TN>::value) > 4 * TM * TN
                  ? 4 * 32 * (SkPitch<TM>::value + SkPitch<TN>::value)
                  : 4 * TM * TN);
}

template <int TM, int TN, bool VEC, bool OUT_BF16>
__device__ __forceinline__ void gemm_f32_splitk_tile(const GemmArgs &p, int bid, unsigned char *smem_raw) {
  constexpr int BK = 32, FM = TM / 16, FN = TN / 16;
  constexpr int SA = SkPitch<TM>::value, SB = SkPitch<TN>::value;
  constexpr int UA = TM * BK / 4 / 64, UB = BK * TN / 4 / 64;  // float4 loads per lane
  float *smem = reinterpret_cast<float *>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  float *As = smem + w * BK * SA;
  float *Bs = smem + 4 * BK * SA + w * BK * SB;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * TM, n0 = tn * TN;
  const float *A = static_cast<const float *>(p.A);
  const float *B = static_cast<const float *>(p.B);
  const int nchunks = (p.K + BK - 1) / BK;
  const int iters = (nchunks + 3) / 4;

  float4 ra[UA], rb[UB];
  auto load = [&](int chunk) {
    const int k0 = chunk * BK;
#pragma unroll
    for (int j = 0; j < UA; ++j) {
      const int u = lane + 64 * j, r = u / (BK / 4), c = (u % (BK / 4)) * 4;
      const int gr = m0 + r, gc = k0 + c;
      if (VEC && gr < p.M && gc + 3 < p.K) {
        ra[j] = *reinterpret_cast<const float4 *>(A + int64_t(gr) * p.lda + gc);
      } else {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (gr < p.M && gc + e < p.K) ? A[int64_t(gr) * p.lda + gc + e] : 0.f;
        ra[j] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
#pragma unroll
    for (int j = 0; j < UB; ++j) {
      const int u = lane + 64 * j, r = u / (TN / 4), c = (u % (TN / 4)) * 4;
      const int gr = k0 + r, gc = n0 + c;
      if (VEC && gr < p.K && gc + 3 < p.N) {
        rb[j] = *reinterpret_cast<const float4 *>(B + int64_t(gr) * p.ldb + gc);
      } else {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (gr < p.K && gc + e < p.N) ? B[int64_t(gr) * p.ldb + gc + e] : 0.f;
        rb[j] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  };

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  load(w);  // chunk w; chunks >= nchunks load zeros
  for (int it = 0; it < iters; ++it) {
    // no block barrier in this loop: each wavefront stages and reads only its own LDS region,
    // and one wavefront's LDS operations take effect in program order
#pragma unroll
    for (int j = 0; j < UA; ++j) {
      const int u = lane + 64 * j, r = u / (BK / 4), c = (u % (BK / 4)) * 4;
      As[(c + 0) * SA + r] = ra[j].x;
      As[(c + 1) * SA + r] = ra[j].y;
      As[(c + 2) * SA + r] = ra[j].z;
      As[(c + 3) * SA + r] = ra[j].w;
    }
#pragma unroll
    for (int j = 0; j < UB; ++j) {
      const int u = lane + 64 * j, r = u / (TN / 4), c = (u % (TN / 4)) * 4;
      *reinterpret_cast<float4 *>(&Bs[r * SB + c]) = rb[j];
    }
    if (it + 1 < iters) load((it + 1) * 4 + w);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + (lane >> 4);
      float a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[k * SA + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[k * SB + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();
  float *red = smem;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[w * TM * TN + (i * 16 + (lane >> 4) * 4 + r) * TN + j * 16 + (lane & 15)] = acc[i][j][r];
  __syncthreads();
  for (int e = tid; e < TM * TN; e += 256) {
    const int row = m0 + e / TN, col = n0 + e % TN;
    const float v = ((red[e] + red[TM * TN + e]) + red[2 * TM * TN + e]) + red[3 * TM * TN + e];
    if (row < p.M && col < p.N) store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * v);
  }
}

template <int TM, int TN>
constexpr int gemm_bf16_splitk_smem() {
  return 4 * (TM + TN) * 72 * 2 > 4 * TM * TN * 4 ? 4 * (TM + TN) * 72 * 2 : 4 * TM * TN * 4;
}

// PREFETCH = false loads each chunk just before staging it instead of during the previous
// chunk's products: no staging registers live beside the fragments and accumulators (for the
// 64 x 64 tile, whose 64 accumulator registers per lane would otherwise push a two-wavefront-per-
// SIMD kernel into spills), at the price of the overlap, which matters little when a wavefront
// has only a few chunks.
template <int TM, int TN, bool VEC, bool OUT_BF16, bool PREFETCH = true>
__device__ __forceinline__ void gemm_bf16_splitk_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  constexpr int BK = 64, KP = BK + 8, FM = TM / 16, FN = TN / 16;
  constexpr int UA = TM * (BK / 8) / 64;        // uint4 (8 x bf16) loads per lane
  constexpr int UB = (BK / 2) * (TN / 8) / 64;  // (k, k+1) x 8-column units per lane
  static_assert(UA >= 1 && UB >= 1, "tile too small for one load per lane");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint16_t *As = reinterpret_cast<uint16_t *>(smem) + w * TM * KP;
  uint16_t *Bt = reinterpret_cast<uint16_t *>(smem) + 4 * TM * KP + w * TN * KP;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * TM, n0 = tn * TN;
  const uint16_t *A = static_cast<const uint16_t *>(p.A);
  const uint16_t *B = static_cast<const uint16_t *>(p.B);
  const int nchunks = (p.K + BK - 1) / BK;
  const int iters = (nchunks + 3) / 4;

  uint4 ra[UA], rb0[UB], rb1[UB];
  auto load = [&](int chunk) {
    const int k0 = chunk * BK;
#pragma unroll
    for (int j = 0; j < UA; ++j) {
      const int u = lane + 64 * j, r = u / (BK / 8), c = (u % (BK / 8)) * 8;
      const int gr = m0 + r, gc = k0 + c;
      if (VEC && gr < p.M && gc + 7 < p.K) {
        ra[j] = *reinterpret_cast<const uint4 *>(A + int64_t(gr) * p.lda + gc);
      } else {
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (gr < p.M && gc + e < p.K) ? A[int64_t(gr) * p.lda + gc + e] : 0;
        memcpy(&ra[j], v, 16);
      }
    }
#pragma unroll
    for (int j = 0; j < UB; ++j) {
      const int u = lane + 64 * j, kp = u / (TN / 8), c = (u % (TN / 8)) * 8;
      const int gk = k0 + 2 * kp, gc = n0 + c;
      if (VEC && gk + 1 < p.K && gc + 7 < p.N) {
        rb0[j] = *reinterpret_cast<const uint4 *>(B + int64_t(gk) * p.ldb + gc);
        rb1[j] = *reinterpret_cast<const uint4 *>(B + int64_t(gk + 1) * p.ldb + gc);
      } else {
        uint16_t lo[8], hi[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          lo[e] = (gk < p.K && gc + e < p.N) ? B[int64_t(gk) * p.ldb + gc + e] : 0;
          hi[e] = (gk + 1 < p.K && gc + e < p.N) ? B[int64_t(gk + 1) * p.ldb + gc + e] : 0;
        }
        memcpy(&rb0[j], lo, 16);
        memcpy(&rb1[j], hi, 16);
      }
    }
  };

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  if (PREFETCH) load(w);
  for (int it = 0; it < iters; ++it) {
    // no block barrier in this loop: each wavefront stages and reads only its own LDS region,
    // and one wavefront's LDS operations take effect in program order
    if (!PREFETCH) load(it * 4 + w);
#pragma unroll
    for (int j = 0; j < UA; ++j) {
      const int u = lane + 64 * j, r = u / (BK / 8), c = (u % (BK / 8)) * 8;
      *reinterpret_cast<uint4 *>(&As[r * KP + c]) = ra[j];
    }
#pragma unroll
    for (int j = 0; j < UB; ++j) {
      const int u = lane + 64 * j, kp = u / (TN / 8), c = (u % (TN / 8)) * 8;
      uint16_t lo[8], hi[8];
      memcpy(lo, &rb0[j], 16);
      memcpy(hi, &rb1[j], 16);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        *reinterpret_cast<uint32_t *>(&Bt[(c + e) * KP + 2 * kp]) = uint32_t(lo[e]) | (uint32_t(hi[e]) << 16);
    }
    if (PREFETCH && it + 1 < iters) load((it + 1) * 4 + w);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      bf16x8 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[(i * 16 + (lane & 15)) * KP + kq]);
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bt[(j * 16 + (lane & 15)) * KP + kq]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();
  float *red = reinterpret_cast<float *>(smem);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[w * TM * TN + (i * 16 + (lane >> 4) * 4 + r) * TN + j * 16 + (lane & 15)] = acc[i][j][r];
  __syncthreads();
  for (int e = tid; e < TM * TN; e += 256) {
    const int row = m0 + e / TN, col = n0 + e % TN;
    const float v = ((red[e] + red[TM * TN + e]) + red[2 * TM * TN + e]) + red[3 * TM * TN + e];
    if (row < p.M && col < p.N) store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * v);
  }
}

// ---------------------------------------------------------------------------------------------
// Latency-bound BF16 GEMM with K split over the block's four wavefronts, each wavefront's whole
// share of K in flight at once.  Wavefront w owns the contiguous K chunks (64 deep) [w q, (w+1) q),
// q = ceil(chunks / 4); it loads D of them into registers in one go -- for K up to 256 D one
// memory round trip in all -- stages them in its own LDS region (A as rows, B as (k, k + 1) pairs
// per column, as in the tile above), then multiplies them in order.  The four partial tiles are
// summed through LDS in the order w = 0, 1, 2, 3.  Trip counts are uniform across wavefronts
// (chunks past the end are zero-filled), so every __syncthreads is reached by all of them.
// For the attention projections (1024 x 64 x 1024: few output tiles, a long K) the staged tile
// above pays four memory round trips and eight barriers per block instead of one and two.
// ---------------------------------------------------------------------------------------------
template <int TM, int TN, int D>
constexpr int gemm_bf16_deep_smem() {
  return 4 * D * (TM + TN) * 72 * 2 > 4 * TM * TN * 4 ? 4 * D * (TM + TN) * 72 * 2 : 4 * TM * TN * 4;
}

template <int TM, int TN, int D, bool VEC, bool OUT_BF16>
__device__ __forceinline__ void gemm_bf16_deep_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  constexpr int BK = 64, KP = BK + 8, FM = TM / 16, FN = TN / 16;
  constexpr int UA = TM * (BK / 8) / 64;        // uint4 (8 x bf16) A loads per lane per chunk
  constexpr int UB = (BK / 2) * (TN / 8) / 64;  // (k, k+1) x 8-column B units per lane per chunk
  static_assert(UA >= 1 && UB >= 1, "tile too small for one load per lane");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint16_t *const region = reinterpret_cast<uint16_t *>(smem) + w * D * (TM + TN) * KP;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * TM, n0 = tn * TN;
  const uint16_t *A = static_cast<const uint16_t *>(p.A);
  const uint16_t *B = static_cast<const uint16_t *>(p.B);
  const int nchunks = (p.K + BK - 1) / BK;
  const int q = (nchunks + 3) / 4;                // chunks per wavefront
  const int c_begin = w * q, c_end = min(nchunks, c_begin + q);
  const int rounds = (q + D - 1) / D;

  uint4 ra[D][UA], rb0[D][UB], rb1[D][UB];
  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int rd = 0; rd < rounds; ++rd) {
    // every load of the round first
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int chunk = c_begin + rd * D + d;
      const bool live = chunk < c_end;
      const int k0 = chunk * BK;
#pragma unroll
      for (int j = 0; j < UA; ++j) {
        const int u = lane + 64 * j, r = u / (BK / 8), c = (u % (BK / 8)) * 8;
        const int gr = m0 + r, gc = k0 + c;
        if (VEC && live && gr < p.M && gc + 7 < p.K) {
          ra[d][j] = *reinterpret_cast<const uint4 *>(A + int64_t(gr) * p.lda + gc);
        } else {
          uint16_t v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (live && gr < p.M && gc + e < p.K) ? A[int64_t(gr) * p.lda + gc + e] : 0;
          memcpy(&ra[d][j], v, 16);
        }
      }
#pragma unroll
      for (int j = 0; j < UB; ++j) {
        const int u = lane + 64 * j, kp = u / (TN / 8), c = (u % (TN / 8)) * 8;
        const int gk = k0 + 2 * kp, gc = n0 + c;
        if (VEC && live && gk + 1 < p.K && gc + 7 < p.N) {
          rb0[d][j] = *reinterpret_cast<const uint4 *>(B + int64_t(gk) * p.ldb + gc);
          rb1[d][j] = *reinterpret_cast<const uint4 *>(B + int64_t(gk + 1) * p.ldb + gc);
        } else {
          uint16_t lo[8], hi[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            lo[e] = (live && gk < p.K && gc + e < p.N) ? B[int64_t(gk) * p.ldb + gc + e] : 0;
            hi[e] = (live && gk + 1 < p.K && gc + e < p.N) ? B[int64_t(gk + 1) * p.ldb + gc + e] : 0;
          }
          memcpy(&rb0[d][j], lo, 16);
          memcpy(&rb1[d][j], hi, 16);
        }
      }
    }
    __syncthreads();   // the previous round's products are done with the LDS regions
#pragma unroll
    for (int d = 0; d < D; ++d) {
      uint16_t *As = region + d * (TM + TN) * KP;
      uint16_t *Bt = As + TM * KP;
#pragma unroll
      for (int j = 0; j < UA; ++j) {
        const int u = lane + 64 * j, r = u / (BK / 8), c = (u % (BK / 8)) * 8;
        *reinterpret_cast<uint4 *>(&As[r * KP + c]) = ra[d][j];
      }
#pragma unroll
      for (int j = 0; j < UB; ++j) {
        const int u = lane + 64 * j, kp = u / (TN / 8), c = (u % (TN / 8)) * 8;
        uint16_t lo[8], hi[8];
        memcpy(lo, &rb0[d][j], 16);
        memcpy(hi, &rb1[d][j], 16);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          *reinterpret_cast<uint32_t *>(&Bt[(c + e) * KP + 2 * kp]) = uint32_t(lo[e]) | (uint32_t(hi[e]) << 16);
      }
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const uint16_t *As = region + d * (TM + TN) * KP;
      const uint16_t *Bt = As + TM * KP;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 32) {
        const int kq = kk + 8 * (lane >> 4);
        bf16x8 a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[(i * 16 + (lane & 15)) * KP + kq]);
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bt[(j * 16 + (lane & 15)) * KP + kq]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  __syncthreads();
  float *red = reinterpret_cast<float *>(smem);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[w * TM * TN + (i * 16 + (lane >> 4) * 4 + r) * TN + j * 16 + (lane & 15)] = acc[i][j][r];
  __syncthreads();
  for (int e = tid; e < TM * TN; e += 256) {
    const int row = m0 + e / TN, col = n0 + e % TN;
    const float v = ((red[e] + red[TM * TN + e]) + red[2 * TM * TN + e]) + red[3 * TM * TN + e];
    if (row < p.M && col < p.N) store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * v);
  }
}

// Eight consecutive bf16 at p[0..8), element e only if ok_e(e), packed into one uint4.
template <typename F>
__device__ __forceinline__ uint4 pack8_guarded(const uint16_t *p, F ok_e) {
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = ok_e(2 * q) ? uint32_t(p[2 * q]) : 0u;
    const uint32_t hi = ok_e(2 * q + 1) ? uint32_t(p[2 * q + 1]) : 0u;
    w[q] = lo | (hi << 16);
  }
  return uint4{w[0], w[1], w[2], w[3]};
}

// ---------------------------------------------------------------------------------------------
// Large BF16 GEMM tile: 256 x 256 outputs per 512-thread block, K step 64, eight wavefronts
// (2 along M x 4 along N) each owning a 128 x 64 sub-tile (8 x 4 blocks of
// v_mfma_f32_16x16x32_bf16, 128 accumulators per lane); two wavefronts per SIMD.  The next K
// step's operands are loaded into registers while the current step is multiplied out of LDS; two
// LDS buffers alternate, so each step needs one barrier.  Shapes are whole tiles (no edge guards,
// no per-load branches), every load an offset from one per-thread base pointer.
// Both operands are staged as they lie in memory, with 16-byte copies: A as As[m][k], B as
// Bs[k][n].  Row pitches 80 and 280 elements: measured with the LDS bank-conflict counter, a
// pitch of 72 for A stalled 37% of the LDS-active cycles on conflicts, 80 stalls 17% (and the
// tile runs ~4% faster); B's pitch changes neither.  The
// matrix core needs, per lane, eight consecutive k of one B column; gfx950's transposing LDS read
// (ds_read_b64_tr_b16) provides them: within each aligned group of 16 lanes, the 16 lanes' 4-wide
// reads form a 16 x 4 matrix M and lane j receives M[j/4 + 4e][j%4], e < 4.  So when lane r of the
// group reads the four columns 4 (r%4) .. 4 (r%4) + 3 of B row k0 + r/4, lane j gets
// B[k0 + e][j] -- four consecutive k of column j; two such reads (k0 and k0 + 4) give the eight.
// ---------------------------------------------------------------------------------------------
constexpr int kBigKP = 80, kBigBP = 280;
constexpr int gemm_bf16_big_smem() { return 2 * (256 * kBigKP + 64 * kBigBP) * 2; }

typedef short shortx4 __attribute__((ext_vector_type(4)));

// Requires M % 256 == 0, N % 256 == 0, K % 64 == 0, 16-byte aligned operands and leading
// dimensions that are multiples of 8 (the launch factory checks; other shapes use tile 4).
template <bool OUT_BF16>
__device__ __forceinline__ void gemm_bf16_big_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  constexpr int BM = 256, BK = 64, KP = kBigKP, BP = kBigBP, FM = 8, FN = 4;
  constexpr int BUF = BM * KP + BK * BP;  // elements per LDS buffer
  uint16_t *const buf0 = reinterpret_cast<uint16_t *>(smem);
  uint16_t *const buf1 = buf0 + BUF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;  // 8 wavefronts
  const int wm = wave >> 2, wn = wave & 3;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * BM, n0 = tn * 256;
  // A units: row ar + 64 j (j < 4), 8 k at ac.  B units: k row br + 16 j (j < 4), 8 n at bc.
  const int ar = tid >> 3, ac = (tid & 7) * 8;
  const int br = tid >> 5, bc = (tid & 31) * 8;
  const uint16_t *pa = static_cast<const uint16_t *>(p.A) + int64_t(m0 + ar) * p.lda + ac;
  const uint16_t *pb = static_cast<const uint16_t *>(p.B) + int64_t(br) * p.ldb + n0 + bc;
  const int64_t a_step = int64_t(64) * p.lda, b_step = int64_t(16) * p.ldb;

  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;  // one K step in flight
#define PSC_BIG_LOAD(k0)                                                                         \
  do {                                                                                           \
    const uint16_t *qa_ = pa + (k0);                                                             \
    ra0 = *reinterpret_cast<const uint4 *>(qa_);                                                 \
    ra1 = *reinterpret_cast<const uint4 *>(qa_ + a_step);                                        \
    ra2 = *reinterpret_cast<const uint4 *>(qa_ + 2 * a_step);                                    \
    ra3 = *reinterpret_cast<const uint4 *>(qa_ + 3 * a_step);                                    \
    const uint16_t *qb_ = pb + int64_t(k0) * p.ldb;                                              \
    rb0 = *reinterpret_cast<const uint4 *>(qb_);                                                 \
    rb1 = *reinterpret_cast<const uint4 *>(qb_ + b_step);                                        \
    rb2 = *reinterpret_cast<const uint4 *>(qb_ + 2 * b_step);                                    \
    rb3 = *reinterpret_cast<const uint4 *>(qb_ + 3 * b_step);                                    \
  } while (0)
  auto store = [&](uint16_t *buf) {
    uint16_t *As = buf + ar * KP + ac;
    *reinterpret_cast<uint4 *>(As) = ra0;
    *reinterpret_cast<uint4 *>(As + 64 * KP) = ra1;
    *reinterpret_cast<uint4 *>(As + 128 * KP) = ra2;
    *reinterpret_cast<uint4 *>(As + 192 * KP) = ra3;
    uint16_t *Bs = buf + BM * KP + br * BP + bc;
    *reinterpret_cast<uint4 *>(Bs) = rb0;
    *reinterpret_cast<uint4 *>(Bs + 16 * BP) = rb1;
    *reinterpret_cast<uint4 *>(Bs + 32 * BP) = rb2;
    *reinterpret_cast<uint4 *>(Bs + 48 * BP) = rb3;
  };

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // this lane's part of the transposing B reads: row 8 (lane / 16) + r / 4 of the slice, columns
  // 4 (r % 4) .. + 3 of the 16-column block (r = lane % 16)
  const int b_lane = (8 * (lane >> 4) + ((lane & 15) >> 2)) * BP + wn * 64 + 4 * (lane & 3);
  auto compute = [&](const uint16_t *buf) {
    const uint16_t *As = buf + (wm * 128 + (lane & 15)) * KP + 8 * (lane >> 4);
    const uint16_t *Bs = buf + BM * KP + b_lane;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      // all fragments of this 32-deep slice first, so the LDS latency is paid once per slice
      bf16x8 b[FN], a[FM];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const uint16_t *q = Bs + kk * BP + j * 16;
        const shortx4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (__attribute__((address_space(3))) shortx4 *)(q));
        const shortx4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (__attribute__((address_space(3))) shortx4 *)(q + 4 * BP));
        const short v[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        memcpy(&b[j], v, 16);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(As + i * 16 * KP + kk);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // ask the scheduler to interleave the LDS reads with the matrix products (measured ~5% faster)
    __builtin_amdgcn_iglp_opt(0);
  };

  const int steps = p.K / BK;
  PSC_BIG_LOAD(0);
  store(buf0);
  __syncthreads();
  for (int s = 0; s < steps; ++s) {
    uint16_t *cur = (s & 1) ? buf1 : buf0, *nxt = (s & 1) ? buf0 : buf1;
    if (s + 1 < steps) PSC_BIG_LOAD((s + 1) * BK);
    compute(cur);
    if (s + 1 < steps) store(nxt);
    __syncthreads();
  }
#undef PSC_BIG_LOAD
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 128 + i * 16 + (lane >> 4) * 4 + r;
        store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * acc[i][j][r]);
      }
    }
}

// ---------------------------------------------------------------------------------------------
// Large BF16 GEMM tile with one wavefront per SIMD and direct global-to-LDS copies: 256 x 256
// outputs per 256-thread block, K step 64, four wavefronts (2 x 2) each owning a 128 x 128
// sub-tile of 4 x 4 blocks of v_mfma_f32_32x32x16_bf16 (256 accumulators per lane, held in the
// accumulator registers).  Against the eight-wavefront tile above, a 128 x 128 sub-tile reads
// (128 + 128) x 64 fragment elements per K step instead of (128 + 64) x 64 for half the outputs:
// 128 KB of LDS fragment reads per K step per CU instead of 192 KB for the same products.
// Operands go from global memory straight into LDS (global_load_lds_dwordx4: each lane names its
// own 16-byte source, the 64 lanes of one instruction fill 1 KB of LDS in lane order), so a stage
// in flight holds no registers and costs no LDS write instructions.  Two 64 KB stages; the copy
// of step s + 1 is issued right after the barrier that opens step s, one barrier per step.
// LDS layout of a stage, unpadded and XOR-swizzled in 16-byte units so that the fragment reads
// of 16 lanes touch distinct banks:
//   A (256 rows x 64 k, 128 B a row):  k unit c of row r is stored at unit c ^ ((r / 2) % 8)
//   B (64 k rows x 256 n, 512 B a row): n unit c of row k is stored at unit c ^ (2 (k % 4))
// Matrix-core layouts (32 x 32 output block, lane l of 64):
//   A: row l % 32, k 8 (l / 32) + e;   B: column l % 32, k 8 (l / 32) + e   (e < 8)
//   accumulator element r of lane l: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
// B's eight k per lane come from two transposing LDS reads per 16-lane group: group g covers
// columns 16 (g % 2) .. + 15 and k 8 (g / 2) .. + 7; lane rl of the group reads k row
// 8 (g / 2) + rl / 4 (and 4 rows below), columns 4 (rl % 4) .. + 3.
// Requires M % 256 == 0, N % 256 == 0, K % 64 == 0, 16-byte aligned operands and leading
// dimensions that are multiples of 8 (the launch factory checks).
// ---------------------------------------------------------------------------------------------
constexpr int gemm_bf16_w4_smem() { return 2 * 65536; }

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;

// WN wavefront columns: WN = 2, four wavefronts of 128 x 128 (one per SIMD); WN = 4, eight
// wavefronts of 128 x 64 (two per SIMD, 128 accumulators each).
template <int WN, bool OUT_BF16>
__device__ __forceinline__ void gemm_bf16_w4_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  constexpr int BK = 64, FM = 4, FN = 8 / WN, STAGE = 65536, BOFF = 32768;
  constexpr int NW = 2 * WN, CPW = 32 / NW;  // wavefronts; A (and B) chunks each copies per stage
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * 256, n0 = tn * 256;

  // Copies.  A chunk q (rows 8q .. 8q + 7): lane l fills unit l % 8 of row 8q + l / 8 with k unit
  // (l % 8) ^ ((4q + l / 16) % 8) = (l % 8) ^ (l / 16) ^ 4 (q % 2).  B chunk q (k rows 2q, 2q + 1):
  // lane l fills unit l % 32 of row 2q + l / 32 with n unit (l % 32) ^ (2 (l / 32)) ^ 4 (q % 2).
  // Wavefront w copies the A chunks and the B chunks CPW w .. CPW w + CPW - 1 of every stage
  // (CPW even, so a chunk's parity is its index's within the wavefront's share).
  const int a_unit = (lane & 7) ^ (lane >> 4), b_unit = (lane & 31) ^ (2 * (lane >> 5));
  const int a_odd = 8 * ((a_unit ^ 4) - a_unit), b_odd = 8 * ((b_unit ^ 4) - b_unit);
  const uint16_t *const a_src =
      static_cast<const uint16_t *>(p.A) + int64_t(m0 + 8 * CPW * wave + (lane >> 3)) * p.lda + 8 * a_unit;
  const uint16_t *const b_src =
      static_cast<const uint16_t *>(p.B) + int64_t(2 * CPW * wave + (lane >> 5)) * p.ldb + n0 + 8 * b_unit;
  const int64_t a_chunk = int64_t(8) * p.lda, b_chunk = int64_t(2) * p.ldb;
  auto copy = [&](int k0, unsigned char *stage) {
    const uint16_t *qa = a_src + k0;
    const uint16_t *qb = b_src + int64_t(k0) * p.ldb;
    unsigned char *da = stage + wave * CPW * 1024, *db = stage + BOFF + wave * CPW * 1024;
#pragma unroll
    for (int i = 0; i < CPW; ++i)
      __builtin_amdgcn_global_load_lds(qa + i * a_chunk + ((i & 1) ? a_odd : 0), (lds_void *)(da + i * 1024), 16, 0, 0);
#pragma unroll
    for (int i = 0; i < CPW; ++i)
      __builtin_amdgcn_global_load_lds(qb + i * b_chunk + ((i & 1) ? b_odd : 0), (lds_void *)(db + i * 1024), 16, 0, 0);
  };

  // Fragment reads.  A: row wm 128 + 32 i + l % 32, k unit 2m + l / 32 for the slice kk = 16 m,
  // stored at unit (2m) ^ v with v = (l / 32) ^ ((l % 32) / 2 % 8).  B: n unit
  // wn 16 + 4 j + u with u = 2 (g % 2) + (rl % 4) / 2 in k row kk + 8 (g / 2) + rl / 4, stored at
  // unit wn 16 + 4 (j ^ (x / 4)) + x % 4 with x = u ^ (2 ((rl / 4) % 4)).
  const int v = (lane >> 5) ^ (((lane & 31) >> 1) & 7);
  const int a_row = (wm * 128 + (lane & 31)) * 128;
  const int g = lane >> 4, rl = lane & 15;
  const int x = (2 * (g & 1) + ((rl & 3) >> 1)) ^ (2 * ((rl >> 2) & 3));
  const int b_base = BOFF + (8 * (g >> 1) + (rl >> 2)) * 512 + 16 * (wn * 4 * FN + (x & 3)) + 8 * (rl & 1);
  const int b_even = b_base + 64 * (x >> 2), b_oddj = b_base + 64 * (1 - (x >> 2));  // j = 0 / j = 1

  floatx16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  // One step: the fragment reads of slices 0 and 1, the products of slice 0 interleaved with the
  // reads of slices 2 and 3, the copy of the next K step into the other stage, then the products
  // of slices 1 to 3 while that copy is in flight.  The compiler cannot tell the two stages apart
  // and waits for outstanding copies before any later LDS read; with no read after the copy inside
  // a step, that wait falls on the barrier of the next step, where it is needed anyway.  The last
  // step copies K step 0 again into the idle stage (no branch in the step, so the instruction
  // groups below apply), and the loop's end waits for it.
  auto step = [&](const unsigned char *stage, int k_next, unsigned char *next) {
    bf16x8 a[BK / 16][FM], b[BK / 16][FN];
#pragma unroll
    for (int m = 0; m < BK / 16; ++m) {
      const unsigned char *pa = stage + a_row + 16 * ((2 * m) ^ v);
#pragma unroll
      for (int i = 0; i < FM; ++i) a[m][i] = *reinterpret_cast<const bf16x8 *>(pa + i * 4096);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const unsigned char *q = stage + ((j & 1) ? b_oddj : b_even) + (j >> 1) * 128 + m * 16 * 512;
        const shortx4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (__attribute__((address_space(3))) shortx4 *)(q));
        const shortx4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (__attribute__((address_space(3))) shortx4 *)(q + 4 * 512));
        const short e[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        memcpy(&b[m][j], e, 16);
      }
    }
    copy(k_next, next);
#pragma unroll
    for (int m = 0; m < BK / 16; ++m)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[m][i], b[m][j], acc[i][j], 0, 0, 0);
    // instruction groups (masks: 0x100 LDS read, 0x008 matrix product, 0x020 global read): the
    // reads of slices 0 and 1, slice 0's products each followed by two of the reads of slices 2
    // and 3, the copy, the other products
    constexpr int RD = FM + 2 * FN, PR = FM * FN;  // LDS reads and products per slice
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * RD, 0);
#pragma unroll
    for (int t = 0; t < RD; ++t) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    }
    if constexpr (PR > RD) __builtin_amdgcn_sched_group_barrier(0x008, PR - RD, 0);
    __builtin_amdgcn_sched_group_barrier(0x020, 2 * CPW, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 3 * PR, 0);
  };

  const int steps = p.K / BK;
  copy(0, smem);
  for (int s = 0; s < steps; ++s) {
    // vmcnt(0): this wavefront's copies into the stage of step s have reached LDS; the barrier
    // then covers every wavefront's, and the end of every wavefront's reads of step s - 1
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    step(smem + (s & 1) * STAGE, s + 1 < steps ? (s + 1) * BK : 0, smem + ((s + 1) & 1) * STAGE);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // the last step's copy
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * 32 * FN + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 128 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        store_elem<OUT_BF16>(p.C, int64_t(row) * p.ldc + col, p.alpha * acc[i][j][r]);
      }
    }
}

// ---------------------------------------------------------------------------------------------
// Skinny GEMM tile for few output tiles and a long K: a 16 x TN output tile (TN = 16 * FN), K cut
// into four contiguous ranges, one per wavefront; no barrier inside the K loop.  Per k step each
// lane reads one vector of its A row (E consecutive k: 4 FP32 or 8 BF16) straight into its
// matrix-core register.  B (row-major, k-major rows) must reach each lane as E consecutive k of
// one column:
//   FP32: each lane reads the 4 k of its column directly (coalesced across the 16 lanes that
//         share those k); the sum over k is order-free, so the 16 k of a step are assigned
//         k = 4 * (l / 16) + e over the four products e, identically for A and B.
//   BF16: lanes read 16-byte runs of two consecutive B rows (k, k + 1) and write them, paired,
//         into a k-contiguous copy in the wavefront's own LDS region, from which each lane reads
//         its 8 k with one 16-byte LDS read.
// G steps of loads are issued together before their products (one memory latency per group
// instead of one per step).  The four partial tiles are added through LDS in a fixed order.
// ---------------------------------------------------------------------------------------------
template <int FN>
constexpr int gemm_direct_bkp() {  // BF16: LDS pitch (bf16 elements) of one k-contiguous column
  return 32 + 8;
}
template <int FN, bool BF16>
constexpr int gemm_direct_smem() {
  constexpr int red = 4 * 16 * 16 * FN * 4;
  constexpr int stage = BF16 ? 4 * (8 / FN) * 16 * FN * gemm_direct_bkp<FN>() * 2 : 0;  // 4 waves x G x TN x pitch
  return red > stage ? red : stage;
}


// G: K steps per load group (default 8 / FN: bounded registers for the standalone kernels; the
// device executor, which runs one workgroup per CU anyway, uses 8 for FP32).
// FP32 B, two ways to reach each lane's E rows of its columns (measured, FN = 2 and 4):
//   BCOL = false: the FN consecutive columns FN c .. FN c + FN - 1 of one B row in one vector
//     load (block j then holds the tile columns = j mod FN): 4x fewer load instructions, 256
//     contiguous bytes per 16 lanes -- faster with short load groups (9.8 -> 7.6 us for a
//     512 x 64 x 512 GEMM in 16 x 64 tiles);
//   BCOL = true: one 4-byte load per (block, row), block j holding columns 16 j .. 16 j + 15 --
//     faster with the executor's groups of 8 steps (its projection tasks ran ~10% longer with
//     the vector loads, 128 of them in flight per lane).
template <int FN, bool BF16, bool VEC, bool OUT_BF16, int G = 8 / FN, bool BCOL = (G > 8 / FN)>
__device__ __forceinline__ void gemm_direct_tile(const GemmArgs &p, int bid, unsigned char *smem) {
  static_assert(!BF16 || G == 8 / FN, "the BF16 staging area is sized for G = 8 / FN");
  constexpr int TN = 16 * FN;
  constexpr int E = BF16 ? 8 : 4;     // consecutive k per lane per step
  constexpr int STEP = 4 * E;         // k per step
  constexpr int KP = gemm_direct_bkp<FN>();
  constexpr int UB = (16 * (TN / 8) + 63) / 64;  // BF16: (k-pair, 8-column) units per lane per step
  using T = typename std::conditional<BF16, uint16_t, float>::type;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tm = bid / p.tiles_n, tn = bid % p.tiles_n;
  const int m0 = tm * 16, n0 = tn * TN;
  const int row = m0 + (lane & 15);
  const int kl = E * (lane >> 4);
  const int kq = ((p.K + 3) / 4 + STEP - 1) / STEP * STEP;
  const int kb = min(p.K, w * kq), ke = min(p.K, kb + kq);
  const int steps = (ke - kb + STEP - 1) / STEP;
  const T *A = static_cast<const T *>(p.A);
  const T *B = static_cast<const T *>(p.B);
  const bool row_ok = row < p.M;
  const T *arow = A + int64_t(row_ok ? row : 0) * p.lda;
  uint16_t *Bt = reinterpret_cast<uint16_t *>(smem) + w * G * TN * KP;  // BF16: this wave's staging

  floatx4 acc[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};

  uint4 ra[G];                                           // A: E consecutive k (16 bytes)
  float rbf[BF16 ? 1 : G][BF16 ? 1 : FN][E];             // FP32 B: the lane's column, E k
  uint4 rb0[BF16 ? G : 1][UB], rb1[BF16 ? G : 1][UB];    // BF16 B: rows k and k + 1, 8 columns
  for (int s0 = 0; s0 < steps; s0 += G) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k = kb + (s0 + g) * STEP + kl;
      if (VEC && row_ok && k + E <= ke) {
        ra[g] = *reinterpret_cast<const uint4 *>(arow + k);
      } else if constexpr (BF16) {
        ra[g] = pack8_guarded(reinterpret_cast<const uint16_t *>(arow) + k, [&](int e) { return row_ok && k + e < ke; });
      } else {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (row_ok && k + e < ke) ? reinterpret_cast<const float *>(arow)[k + e] : 0.f;
        memcpy(&ra[g], v, 16);
      }
      if constexpr (BF16) {
        const int ks = kb + (s0 + g) * STEP;
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int unit = lane + 64 * u, kp = unit / (TN / 8), c = n0 + (unit % (TN / 8)) * 8;
          const int k0 = ks + 2 * kp;
          const bool uok = unit < 16 * (TN / 8);
          const uint16_t *b0 = reinterpret_cast<const uint16_t *>(B) + int64_t(k0) * p.ldb + c;
          if (uok && VEC && k0 + 1 < ke && c + 7 < p.N) {
            rb0[g][u] = *reinterpret_cast<const uint4 *>(b0);
            rb1[g][u] = *reinterpret_cast<const uint4 *>(b0 + p.ldb);
          } else {
            rb0[g][u] = pack8_guarded(b0, [&](int e) { return uok && k0 < ke && c + e < p.N; });
            rb1[g][u] = pack8_guarded(b0 + p.ldb, [&](int e) { return uok && k0 + 1 < ke && c + e < p.N; });
          }
        }
      } else if constexpr (BCOL) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = n0 + 16 * j + (lane & 15);
          const bool col_ok = col < p.N;
#pragma unroll
          for (int e = 0; e < E; ++e)
            rbf[g][j][e] = (col_ok && k + e < ke) ? reinterpret_cast<const float *>(B)[int64_t(k + e) * p.ldb + col] : 0.f;
        }
      } else {
        // FP32 B: the lane's FN consecutive columns of one B row in one load (block j holds the
        // columns = j mod FN of the tile), for each of its E rows k + e
        const int colb = n0 + FN * (lane & 15);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float *brow = reinterpret_cast<const float *>(B) + int64_t(k + e) * p.ldb + colb;
          if (VEC && FN > 1 && colb + FN <= p.N && k + e < ke) {
            if constexpr (FN == 4) {
              const float4 v = *reinterpret_cast<const float4 *>(brow);
              rbf[g][0][e] = v.x; rbf[g][FN > 1 ? 1 : 0][e] = v.y; rbf[g][FN > 2 ? 2 : 0][e] = v.z; rbf[g][FN > 3 ? 3 : 0][e] = v.w;
            } else if constexpr (FN == 2) {
              const float2 v = *reinterpret_cast<const float2 *>(brow);
              rbf[g][0][e] = v.x; rbf[g][FN > 1 ? 1 : 0][e] = v.y;
            }
          } else {
#pragma unroll
            for (int j = 0; j < FN; ++j)
              rbf[g][j][e] = (colb + j < p.N && k + e < ke) ? brow[j] : 0.f;
          }
        }
      }
    }
    if constexpr (BF16) {
      // stage the group's B into this wave's LDS as k-contiguous columns, (k, k+1) per 32-bit write
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int unit = lane + 64 * u, kp = unit / (TN / 8), c = (unit % (TN / 8)) * 8;
          if (unit < 16 * (TN / 8)) {
            const uint32_t lo[4] = {rb0[g][u].x, rb0[g][u].y, rb0[g][u].z, rb0[g][u].w};
            const uint32_t hi[4] = {rb1[g][u].x, rb1[g][u].y, rb1[g][u].z, rb1[g][u].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {  // columns c + 2q (low halves) and c + 2q + 1 (high halves)
              *reinterpret_cast<uint32_t *>(&Bt[(g * TN + c + 2 * q) * KP + 2 * kp]) =
                  (lo[q] & 0xffffu) | (hi[q] << 16);
              *reinterpret_cast<uint32_t *>(&Bt[(g * TN + c + 2 * q + 1) * KP + 2 * kp]) =
                  (lo[q] >> 16) | (hi[q] & 0xffff0000u);
            }
          }
        }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int g = 0; g < G; ++g) {
        bf16x8 av, bv;
        memcpy(&av, &ra[g], 16);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          bv = *reinterpret_cast<const bf16x8 *>(&Bt[(g * TN + j * 16 + (lane & 15)) * KP + kl]);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[j], 0, 0, 0);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float((&ra[g].x)[e]), rbf[g][j][e], acc[j], 0, 0, 0);
    }
  }
  __syncthreads();  // all waves done with their staging before the LDS holds partial sums
  float *red = reinterpret_cast<float *>(smem);
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    // block j, lane column slot c: tile column 16 j + c (BF16, FP32 with BCOL) or FN c + j
    const int tc = (BF16 || BCOL) ? j * 16 + (lane & 15) : FN * (lane & 15) + j;
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w * 16 * TN + ((lane >> 4) * 4 + r) * TN + tc] = acc[j][r];
  }
  __syncthreads();
  for (int e = tid; e < 16 * TN; e += 256) {
    const int orow = m0 + e / TN, col = n0 + e % TN;
    const float v = ((red[e] + red[16 * TN + e]) + red[2 * 16 * TN + e]) + red[3 * 16 * TN + e];
    if (orow < p.M && col < p.N) store_elem<OUT_BF16>(p.C, int64_t(orow) * p.ldc + col, p.alpha * v);
  }
  __syncthreads();  // the LDS may be reused by the caller's next tile
}

// ---------------------------------------------------------------------------------------------
// Row softmax: one wavefront per row, four rows per 256-thread block.  NV > 0: the row is held in
// registers, 4 NV values per lane (rows up to 256*NV); NV == 0: three passes over memory.
// The max and the sum are reduced across the wavefront with butterfly shuffles, in FP32.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NV, bool VEC, bool IN_BF16, bool OUT_BF16, bool NT = false, int CW = 4>
__device__ __forceinline__ void softmax_row(const SoftmaxArgs &p, int row) {
  const int lane = threadIdx.x & 63;
  const int64_t xo = int64_t(row) * p.ldx, yo = int64_t(row) * p.ldy;
  const float ninf = -__builtin_huge_valf();
  if constexpr (NV > 0) {
    // NC chunks of CW consecutive elements per lane; chunk t of lane l starts at column
    // (64 t + l) CW.  CW = 8 (bf16 input only): 16-byte loads of eight bf16 values.
    constexpr int NC = NV * 4 / CW;
    static_assert(CW == 4 || (CW == 8 && IN_BF16 && NV % 2 == 0), "chunk width");
    float v[NC][CW];
    float m = ninf;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int c = (t * 64 + lane) * CW;
      if (VEC && c + CW - 1 < p.C) {
        if constexpr (IN_BF16 && CW == 8) {
          const u32x4 w = load16<NT>(static_cast<const uint16_t *>(p.X) + xo + c);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            v[t][2 * q] = __uint_as_float(w[q] << 16);
            v[t][2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
          }
        } else if constexpr (IN_BF16) {
          const u32x2 w = load8<NT>(static_cast<const uint16_t *>(p.X) + xo + c);
          v[t][0] = __uint_as_float(w.x << 16); v[t][1] = __uint_as_float(w.x & 0xffff0000u);
          v[t][2] = __uint_as_float(w.y << 16); v[t][3] = __uint_as_float(w.y & 0xffff0000u);
        } else {
          const u32x4 w = load16<NT>(static_cast<const float *>(p.X) + xo + c);
          v[t][0] = __uint_as_float(w.x); v[t][1] = __uint_as_float(w.y);
          v[t][2] = __uint_as_float(w.z); v[t][3] = __uint_as_float(w.w);
        }
      } else {
#pragma unroll
        for (int e = 0; e < CW; ++e) v[t][e] = (c + e < p.C) ? load_elem<IN_BF16>(p.X, xo + c + e) : ninf;
      }
#pragma unroll
      for (int e = 0; e < CW; ++e) m = fmaxf(m, v[t][e]);
    }
    m = wave_max(m);
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < NC; ++t)
#pragma unroll
      for (int e = 0; e < CW; ++e) {
        const float ex = (v[t][e] == ninf) ? 0.f : __expf(v[t][e] - m);
        v[t][e] = ex;
        s += ex;
      }
    s = wave_sum(s);
    const float inv = 1.0f / s;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int c = (t * 64 + lane) * CW;
      if (VEC && c + CW - 1 < p.C) {
#pragma unroll
        for (int h = 0; h < CW / 4; ++h) {
          const float *q = &v[t][4 * h];
          if constexpr (OUT_BF16 && CW == 8) {
            if (h == 0) {
              const float *q8 = v[t];
              u32x4 w;
#pragma unroll
              for (int k = 0; k < 4; ++k)
                w[k] = uint32_t(f32_to_bf16(q8[2 * k] * inv)) | (uint32_t(f32_to_bf16(q8[2 * k + 1] * inv)) << 16);
              store16<NT>(static_cast<uint16_t *>(p.Y) + yo + c, w);
            }
          } else if constexpr (OUT_BF16) {
            const u32x2 w = {uint32_t(f32_to_bf16(q[0] * inv)) | (uint32_t(f32_to_bf16(q[1] * inv)) << 16),
                             uint32_t(f32_to_bf16(q[2] * inv)) | (uint32_t(f32_to_bf16(q[3] * inv)) << 16)};
            store8<NT>(static_cast<uint16_t *>(p.Y) + yo + c + 4 * h, w);
          } else {
            const u32x4 w = {__float_as_uint(q[0] * inv), __float_as_uint(q[1] * inv),
                             __float_as_uint(q[2] * inv), __float_as_uint(q[3] * inv)};
            store16<NT>(static_cast<float *>(p.Y) + yo + c + 4 * h, w);
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < CW; ++e)
          if (c + e < p.C) store_elem<OUT_BF16>(p.Y, yo + c + e, v[t][e] * inv);
      }
    }
  } else {
    float m = ninf;
    for (int c = lane; c < p.C; c += 64) m = fmaxf(m, load_elem<IN_BF16>(p.X, xo + c));
    m = wave_max(m);
    float s = 0.f;
    for (int c = lane; c < p.C; c += 64) s += __expf(load_elem<IN_BF16>(p.X, xo + c) - m);
    s = wave_sum(s);
    const float inv = 1.0f / s;
    for (int c = lane; c < p.C; c += 64)
      store_elem<OUT_BF16>(p.Y, yo + c, __expf(load_elem<IN_BF16>(p.X, xo + c) - m) * inv);
  }
}

// ---------------------------------------------------------------------------------------------
// Transpose through a padded 64 x 64 LDS tile: coalesced reads along A's rows, coalesced writes
// along B's rows.  Element size ES bytes (4: f32, 2: bf16); bit-exact.
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void transpose_tile(const TransArgs &p, int bid, unsigned char *smem) {
  T(*tile)[65] = reinterpret_cast<T(*)[65]>(smem);
  const int tiles_c = (p.C + 63) / 64;
  const int tr = bid / tiles_c, tc = bid % tiles_c;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const T *A = static_cast<const T *>(p.A);
  T *B = static_cast<T *>(p.B);
  T v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {  // all sixteen loads in flight before the first LDS write
    const int r = tr * 64 + ty + 4 * i, c = tc * 64 + tx;
    v[i] = (r < p.R && c < p.C) ? A[int64_t(r) * p.lda + c] : T(0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) tile[ty + 4 * i][tx] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = tile[tx][ty + 4 * i];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int orow = tc * 64 + ty + 4 * i, ocol = tr * 64 + tx;
    if (orow < p.C && ocol < p.R) B[int64_t(orow) * p.ldb + ocol] = v[i];
  }
}

// Vector variant for aligned operands (base addresses 16-byte aligned, leading dimensions
// multiples of V = 16 / sizeof(T)): 16-byte global reads along A's rows and 16-byte global writes
// along B's rows; elements move through the padded LDS tile one by one.  Tiles inside the matrix
// take an unchecked path with all sixteen-byte loads in flight at once; edge tiles check every
// vector and fall back to element accesses where one crosses the edge.  NT: streaming loads and
// stores.
template <typename T, bool CHECK, bool NT>
__device__ __forceinline__ void transpose_vec_load(const TransArgs &p, int tr, int tc, T (*tile)[65]) {
  constexpr int V = 16 / int(sizeof(T)), VPR = 64 / V, RPP = 256 / VPR, PASSES = 64 / RPP;
  const int vx = threadIdx.x % VPR, vy = threadIdx.x / VPR;
  const T *A = static_cast<const T *>(p.A);
  u32x4 v[PASSES];
#pragma unroll
  for (int i = 0; i < PASSES; ++i) {
    const int r = tr * 64 + vy + RPP * i, c = tc * 64 + vx * V;
    if (!CHECK || (r < p.R && c + V <= p.C)) {
      v[i] = load16<NT>(A + int64_t(r) * p.lda + c);
    } else {
      T e[V];
#pragma unroll
      for (int j = 0; j < V; ++j) e[j] = (r < p.R && c + j < p.C) ? A[int64_t(r) * p.lda + c + j] : T(0);
      memcpy(&v[i], e, 16);
    }
  }
#pragma unroll
  for (int i = 0; i < PASSES; ++i) {
    T e[V];
    memcpy(e, &v[i], 16);
#pragma unroll
    for (int j = 0; j < V; ++j) tile[vy + RPP * i][vx * V + j] = e[j];
  }
}

template <typename T, bool CHECK, bool NT>
__device__ __forceinline__ void transpose_vec_store(const TransArgs &p, int tr, int tc, T (*tile)[65]) {
  constexpr int V = 16 / int(sizeof(T)), VPR = 64 / V, RPP = 256 / VPR, PASSES = 64 / RPP;
  const int vx = threadIdx.x % VPR, vy = threadIdx.x / VPR;
  T *B = static_cast<T *>(p.B);
#pragma unroll
  for (int i = 0; i < PASSES; ++i) {
    // output row orow = input column; V consecutive output columns = V consecutive input rows
    const int oc = vy + RPP * i, orow = tc * 64 + oc, ocol = tr * 64 + vx * V;
    T e[V];
#pragma unroll
    for (int j = 0; j < V; ++j) e[j] = tile[vx * V + j][oc];
    if (!CHECK || (orow < p.C && ocol + V <= p.R)) {
      u32x4 w;
      memcpy(&w, e, 16);
      store16<NT>(B + int64_t(orow) * p.ldb + ocol, w);
    } else if (orow < p.C) {
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (ocol + j < p.R) B[int64_t(orow) * p.ldb + ocol + j] = e[j];
    }
  }
}

template <typename T, bool NT = false>
__device__ __forceinline__ void transpose_tile_vec(const TransArgs &p, int bid, unsigned char *smem) {
  T(*tile)[65] = reinterpret_cast<T(*)[65]>(smem);
  const int tiles_c = (p.C + 63) / 64, tiles_r = (p.R + 63) / 64;
  // diagonal order: consecutive workgroups take different tile rows as well as different tile
  // columns, so the ones in flight together write different column ranges of B (with a
  // power-of-two leading dimension, equal column ranges of many rows share HBM channels)
  const int tc = bid % tiles_c, tr = (bid / tiles_c + tc) % tiles_r;
  if ((tr + 1) * 64 <= p.R && (tc + 1) * 64 <= p.C) {
    transpose_vec_load<T, false, NT>(p, tr, tc, tile);
    __syncthreads();
    transpose_vec_store<T, false, NT>(p, tr, tc, tile);
  } else {
    transpose_vec_load<T, true, NT>(p, tr, tc, tile);
    __syncthreads();
    transpose_vec_store<T, true, NT>(p, tr, tc, tile);
  }
}

// Rectangular tiles for aligned operands: TR rows x TC columns of A per 256-thread block, so a
// block reads TR runs of TC elements and writes TC runs of TR elements (64 x 128 doubles the
// contiguous read runs of the 64 x 64 tile, 128 x 64 the write runs).  Tiles inside the matrix go
// through 16-byte vectors, edge tiles element by element with checks.  Diagonal tile order as
// above.
template <int TR, int TC, typename T>
constexpr int transpose_rc_smem() { return TR * (TC + 1) * int(sizeof(T)); }

template <typename T, int TR, int TC, bool NT>
__device__ __forceinline__ void transpose_rc_tile(const TransArgs &p, int bid, unsigned char *smem) {
  constexpr int V = 16 / int(sizeof(T));
  constexpr int VPR = TC / V, NV = TR * VPR / 256;    // read vectors per A row, per thread
  constexpr int VPB = TR / V, NVB = TC * VPB / 256;   // write vectors per B row, per thread
  static_assert(NV >= 1 && NVB >= 1 && TR * VPR % 256 == 0 && TC * VPB % 256 == 0, "tile shape");
  T(*tile)[TC + 1] = reinterpret_cast<T(*)[TC + 1]>(smem);
  const int tiles_c = (p.C + TC - 1) / TC, tiles_r = (p.R + TR - 1) / TR;
  const int tc = bid % tiles_c, tr = (bid / tiles_c + tc) % tiles_r;
  const int r0 = tr * TR, c0 = tc * TC;
  const T *A = static_cast<const T *>(p.A);
  T *B = static_cast<T *>(p.B);
  if (r0 + TR <= p.R && c0 + TC <= p.C) {
    u32x4 v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {   // every read of the tile in flight at once
      const int idx = threadIdx.x + 256 * i, r = idx / VPR, cv = idx % VPR;
      v[i] = load16<NT>(A + int64_t(r0 + r) * p.lda + c0 + cv * V);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int idx = threadIdx.x + 256 * i, r = idx / VPR, cv = idx % VPR;
      T e[V];
      memcpy(e, &v[i], 16);
#pragma unroll
      for (int j = 0; j < V; ++j) tile[r][cv * V + j] = e[j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NVB; ++i) {
      const int idx = threadIdx.x + 256 * i, orow = idx / VPB, ov = idx % VPB;
      T e[V];
#pragma unroll
      for (int j = 0; j < V; ++j) e[j] = tile[ov * V + j][orow];
      u32x4 w;
      memcpy(&w, e, 16);
      store16<NT>(B + int64_t(c0 + orow) * p.ldb + r0 + ov * V, w);
    }
  } else {
    for (int idx = threadIdx.x; idx < TR * TC; idx += 256) {
      const int r = idx / TC, c = idx % TC;
      tile[r][c] = (r0 + r < p.R && c0 + c < p.C) ? A[int64_t(r0 + r) * p.lda + c0 + c] : T(0);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < TC * TR; idx += 256) {
      const int orow = idx / TR, ocol = idx % TR;
      if (c0 + orow < p.C && r0 + ocol < p.R) B[int64_t(c0 + orow) * p.ldb + r0 + ocol] = tile[ocol][orow];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Element-wise add in FP32: grid (ceil(C/256), R), one element per thread.
// ---------------------------------------------------------------------------------------------
template <bool IN_BF16, bool OUT_BF16>
__device__ __forceinline__ void add_block(const AddArgs &p, int bid) {
  const int nbx = (p.C + 255) / 256;
  const int c = (bid % nbx) * 256 + threadIdx.x;
  const int r = bid / nbx;
  if (c >= p.C || r >= p.R) return;
  const float a = load_elem<IN_BF16>(p.A, int64_t(r) * p.lda + c);
  const float b = load_elem<IN_BF16>(p.B, int64_t(r) * p.ldb + c);
  store_elem<OUT_BF16>(p.Cp, int64_t(r) * p.ldc + c, a + b);
}

// Vector variant (operands 16-byte aligned, leading dimensions multiples of 8): each thread adds
// 8 consecutive elements per row of a 2048-column chunk; a workgroup covers one chunk of one row.
// The FP32 sum of two values is rounded once to the output type, as in add_block.
template <bool IN_BF16, bool OUT_BF16, bool NT = false>
__device__ __forceinline__ void add_block_vec(const AddArgs &p, int bid) {
  const int nbx = (p.C + 2047) / 2048;
  const int c = (bid % nbx) * 2048 + threadIdx.x * 8;
  const int r = bid / nbx;
  if (c >= p.C || r >= p.R) return;
  const int64_t ia = int64_t(r) * p.lda + c, ib = int64_t(r) * p.ldb + c, ic = int64_t(r) * p.ldc + c;
  float a[8], b[8];
  if (c + 8 <= p.C) {
    if constexpr (IN_BF16) {
      const u32x4 x = load16<NT>(static_cast<const uint16_t *>(p.A) + ia);
      const u32x4 y = load16<NT>(static_cast<const uint16_t *>(p.B) + ib);
      const uint32_t xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[2 * q] = __uint_as_float(xs[q] << 16);
        a[2 * q + 1] = __uint_as_float(xs[q] & 0xffff0000u);
        b[2 * q] = __uint_as_float(ys[q] << 16);
        b[2 * q + 1] = __uint_as_float(ys[q] & 0xffff0000u);
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const u32x4 x = load16<NT>(static_cast<const float *>(p.A) + ia + 4 * h);
        const u32x4 y = load16<NT>(static_cast<const float *>(p.B) + ib + 4 * h);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a[4 * h + e] = __uint_as_float(x[e]);
          b[4 * h + e] = __uint_as_float(y[e]);
        }
      }
    }
    if constexpr (OUT_BF16) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        w[q] = uint32_t(f32_to_bf16(a[2 * q] + b[2 * q])) | (uint32_t(f32_to_bf16(a[2 * q + 1] + b[2 * q + 1])) << 16);
      store16<NT>(static_cast<uint16_t *>(p.Cp) + ic, u32x4{w[0], w[1], w[2], w[3]});
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h)
        store16<NT>(static_cast<float *>(p.Cp) + ic + 4 * h,
                    u32x4{__float_as_uint(a[4 * h] + b[4 * h]), __float_as_uint(a[4 * h + 1] + b[4 * h + 1]),
                          __float_as_uint(a[4 * h + 2] + b[4 * h + 2]), __float_as_uint(a[4 * h + 3] + b[4 * h + 3])});
    }
  } else {
    for (int e = 0; c + e < p.C; ++e)
      store_elem<OUT_BF16>(p.Cp, ic + e, load_elem<IN_BF16>(p.A, ia + e) + load_elem<IN_BF16>(p.B, ib + e));
  }
}

}  // namespace psc
