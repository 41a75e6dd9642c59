// gemm_bf16.h -- generic BF16 x BF16 -> FP32 MFMA GEMM for gfx950 (library-internal).
//
// C[M,N] = sum_k A[m,k] B[k,n] with operands fetched through loader functors
// (so a GEMM can read a transposed matrix or a concatenation without
// materialising it) and results handed to an epilogue functor (bias, ReLU,
// masks, BF16 stores, split-K partial sums).
//
// Tiling: a workgroup of 256 threads (4 waves) owns a BM x BN tile of C; the
// waves are arranged WM x WN and each accumulates a (BM/WM) x (BN/WN) sub-tile
// in 16x16 MFMA fragments.  K advances BK per stage: the A and B tiles are
// staged in LDS as [row][k] (k contiguous, rows padded by 8 elements against
// bank conflicts), double buffered, with the next stage's global loads in
// registers while the current stage feeds the MFMAs.  A large BK keeps enough
// bytes in flight per CU to cover HBM latency with one workgroup per CU.
// The finished tile is staged through LDS as FP32 so that the epilogue sees
// eight consecutive columns of a row per call (16-byte loads and stores).
//
// MFMA v_mfma_f32_16x16x32_bf16 lane layout (wave64): lane l supplies
// A[l%16][8*(l/16) .. +7] and B[8*(l/16) .. +7][l%16]; it receives
// C[4*(l/16) + i][l%16] for i = 0..3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aslam {
namespace gemm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t lane16(const uint4& v, int j) {
  const uint32_t w = j < 2 ? v.x : j < 4 ? v.y : j < 6 ? v.z : v.w;
  return (uint16_t)(w >> ((j & 1) * 16));
}

// Loader contract (eight BF16 packed in a uint4, element j in bits 16j..16j+15):
//   static constexpr bool kMajor;
//   kMajor  : fetch(i, k) = X(i, k + j), j < 8 (k multiple of 8)
//   !kMajor : fetch(i, k) = X(i + j, k), j < 8 (i multiple of 8)
// where X(i, k) is A(m = i, k) for the A operand and B(k, n = i) for B.
// Out-of-range elements must read as 0.
//
// Epilogue contract: store8(m, n0, v, nvalid) for row m < M and the eight
// columns n0 .. n0 + 7 (n0 multiple of 8), of which the first nvalid are < N.

template <int BM, int BN, int BK, int WM, int WN>
struct Cfg {
  static_assert(WM * WN == 4, "four waves");
  static constexpr int TM = BM / WM, TN = BN / WN;   // wave sub-tile
  static constexpr int FM = TM / 16, FN = TN / 16;   // fragments per wave
  static_assert(FM * 16 == TM && FN * 16 == TN, "fragment tiling");
  static_assert(BK % 32 == 0, "BK is a multiple of the MFMA depth");
  static constexpr int PADK = BK + 8;                 // LDS row length in elements
  static constexpr int VA = BM * BK / 8, VB = BN * BK / 8;            // 8-element vectors per stage
  static constexpr int PA = (VA + 255) / 256, PB = (VB + 255) / 256;  // vectors per thread
  static constexpr int kStageBytes = 2 * (BM + BN) * PADK * 2;        // double-buffered A and B
  static constexpr int kEpiBytes = BM * (BN + 4) * 4;                 // FP32 tile (rows padded)
  static constexpr int kLds = kStageBytes > kEpiBytes ? kStageBytes : kEpiBytes;
};

template <class L, int ROWS, int BK, int P>
__device__ __forceinline__ void fetch_tile(const L& ld, int row0, int k0, uint4 (&regs)[P]) {
  constexpr int V = ROWS * BK / 8;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int v = threadIdx.x + p * 256;
    if (V % 256 == 0 || v < V) {
      if (L::kMajor) {
        const int i = v / (BK / 8), kq = v % (BK / 8);
        regs[p] = ld.fetch(row0 + i, k0 + kq * 8);
      } else {
        const int k = v / (ROWS / 8), iq = v % (ROWS / 8);
        regs[p] = ld.fetch(row0 + iq * 8, k0 + k);
      }
    }
  }
}

template <class L, int ROWS, int BK, int P>
__device__ __forceinline__ void store_tile(uint16_t* s, const uint4 (&regs)[P]) {
  constexpr int V = ROWS * BK / 8, PADK = BK + 8;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int v = threadIdx.x + p * 256;
    if (V % 256 == 0 || v < V) {
      if (L::kMajor) {
        const int i = v / (BK / 8), kq = v % (BK / 8);
        *reinterpret_cast<uint4*>(s + i * PADK + kq * 8) = regs[p];
      } else {
        const int k = v / (ROWS / 8), iq = v % (ROWS / 8);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[(iq * 8 + j) * PADK + k] = lane16(regs[p], j);
      }
    }
  }
}

template <int BM, int BN, int BK, int WM, int WN, class LA, class LB, class EPI>
__global__ __launch_bounds__(256) void k_gemm(LA la, LB lb, EPI epi, int M, int N, int K, int k_split) {
  using C = Cfg<BM, BN, BK, WM, WN>;
  constexpr int PADK = C::PADK;
  __shared__ __align__(16) unsigned char smem[C::kLds];
  uint16_t* sA = reinterpret_cast<uint16_t*>(smem);           // [2][BM * PADK]
  uint16_t* sB = sA + 2 * BM * PADK;                          // [2][BN * PADK]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave / WN, wn = wave % WN;
  const int m_blk = blockIdx.x * BM, n_blk = blockIdx.y * BN;   // M tiles on x (up to 2^31 - 1)
  const int kb = blockIdx.z * k_split;
  const int ke = min(K, kb + k_split);
  f32x4 acc[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  uint4 ra[C::PA], rb[C::PB];
  const int nsteps = (ke - kb + BK - 1) / BK;
  if (nsteps > 0) {
    fetch_tile<LA, BM, BK>(la, m_blk, kb, ra);
    fetch_tile<LB, BN, BK>(lb, n_blk, kb, rb);
    store_tile<LA, BM, BK>(sA, ra);
    store_tile<LB, BN, BK>(sB, rb);
  }
  __syncthreads();
  for (int t = 0; t < nsteps; ++t) {
    const int buf = t & 1;
    const bool more = t + 1 < nsteps;
    if (more) {
      fetch_tile<LA, BM, BK>(la, m_blk, kb + (t + 1) * BK, ra);
      fetch_tile<LB, BN, BK>(lb, n_blk, kb + (t + 1) * BK, rb);
    }
    const uint16_t* a_base = sA + buf * BM * PADK + (wm * C::TM + (lane & 15)) * PADK + 8 * (lane >> 4);
    const uint16_t* b_base = sB + buf * BN * PADK + (wn * C::TN + (lane & 15)) * PADK + 8 * (lane >> 4);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8 bf[C::FN];
#pragma unroll
      for (int j = 0; j < C::FN; ++j)
        bf[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(b_base + j * 16 * PADK + kk));
#pragma unroll
      for (int i = 0; i < C::FM; ++i) {
        const bf16x8 af = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(a_base + i * 16 * PADK + kk));
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      store_tile<LA, BM, BK>(sA + (buf ^ 1) * BM * PADK, ra);
      store_tile<LB, BN, BK>(sB + (buf ^ 1) * BN * PADK, rb);
    }
    __syncthreads();
  }
  // stage the FP32 tile through LDS, then hand rows of eight columns to the epilogue
  float* sc = reinterpret_cast<float*>(smem);
  constexpr int LDC = BN + 4;
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wm * C::TM + i * 16 + 4 * (lane >> 4) + e;
        const int c = wn * C::TN + j * 16 + (lane & 15);
        sc[r * LDC + c] = acc[i][j][e];
      }
  __syncthreads();
  constexpr int kVecPerRow = BN / 8;
  for (int v = threadIdx.x; v < BM * kVecPerRow; v += 256) {
    const int r = v / kVecPerRow, c0 = (v % kVecPerRow) * 8;
    const int m = m_blk + r, n0 = n_blk + c0;
    if (m >= M || n0 >= N) continue;
    const float4 lo = *reinterpret_cast<const float4*>(sc + r * LDC + c0);
    const float4 hi = *reinterpret_cast<const float4*>(sc + r * LDC + c0 + 4);
    const float vals[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    epi.store8(m, n0, vals, min(8, N - n0));
  }
}

template <int BM, int BN, int BK, int WM, int WN, class LA, class LB, class EPI>
hipError_t run(const LA& la, const LB& lb, const EPI& epi, int M, int N, int K, int splits, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  int k_split = (K + splits - 1) / splits;
  k_split = (k_split + BK - 1) / BK * BK;
  const int nz = K > 0 ? (K + k_split - 1) / k_split : 1;
  if ((N + BN - 1) / BN > 65535 || nz > 65535) return hipErrorInvalidValue;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, nz);
  k_gemm<BM, BN, BK, WM, WN, LA, LB, EPI><<<grid, 256, 0, st>>>(la, lb, epi, M, N, K, k_split);
  return hipGetLastError();
}

}  // namespace gemm
}  // namespace aslam
