// gemm_bf16.h -- generic BF16 x BF16 -> FP32 MFMA GEMM for gfx950 (library-internal).
//
// C[M,N] = sum_k A[m,k] B[k,n] with operands fetched through loader functors
// (so a GEMM can read a transposed matrix, an im2col view or a concatenation
// without materialising it) and results handed to an epilogue functor (bias,
// ReLU, masks, BF16 stores, split-K partial sums).
//
// Tiling: a workgroup of 256 threads (4 waves) owns a BM x BN tile of C.  The
// waves are arranged WM x WN x WK; each wave accumulates a (BM/WM) x (BN/WN)
// sub-tile in 16x16 MFMA fragments over the K steps congruent to its WK index,
// and WK > 1 waves are summed through LDS at the end.  K advances 32 at a
// time: A and B tiles are converted to BF16 and staged in LDS as [row][k]
// (k contiguous, rows padded by 8 elements), double buffered, with the next
// tile's global loads in flight while the current one feeds the MFMAs.
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

constexpr int BK = 32;
constexpr int PADK = BK + 8;   // LDS row length in elements (16-byte pad against bank conflicts)

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Loader contract:
//   static constexpr bool kMajor;
//   kMajor  : fetch(i, k, v) fills v[j] = X(i, k + j), j < 8 (k multiple of 8)
//   !kMajor : fetch(i, k, v) fills v[j] = X(i + j, k), j < 8 (i multiple of 8)
// where X(i, k) is A(m = i, k) for the A operand and B(k, n = i) for B.
// Out-of-range elements must read as 0.

template <int BM, int BN, int WM, int WN, int WK>
struct Cfg {
  static_assert(WM * WN * WK == 4, "four waves");
  static constexpr int TM = BM / WM, TN = BN / WN;   // wave sub-tile
  static constexpr int FM = TM / 16, FN = TN / 16;   // fragments per wave
  static_assert(FM * 16 == TM && FN * 16 == TN, "fragment tiling");
  static constexpr int VA = BM * BK / 8, VB = BN * BK / 8;  // 8-element vectors per tile
  static constexpr int PA = (VA + 255) / 256, PB = (VB + 255) / 256;  // vectors per thread
};

template <class L, int ROWS>
__device__ __forceinline__ void fetch_tile(const L& ld, int row0, int k0, uint16_t (*regs)[8], int per_thread) {
  constexpr int V = ROWS * BK / 8;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p >= per_thread) break;
    const int v = threadIdx.x + p * 256;
    if (v < V) {
      if (L::kMajor) {
        const int i = v / (BK / 8), kq = v % (BK / 8);
        ld.fetch(row0 + i, k0 + kq * 8, regs[p]);
      } else {
        const int k = v / (ROWS / 8), iq = v % (ROWS / 8);
        ld.fetch(row0 + iq * 8, k0 + k, regs[p]);
      }
    }
  }
}

template <class L, int ROWS>
__device__ __forceinline__ void store_tile(uint16_t* s, uint16_t (*regs)[8], int per_thread) {
  constexpr int V = ROWS * BK / 8;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p >= per_thread) break;
    const int v = threadIdx.x + p * 256;
    if (v < V) {
      if (L::kMajor) {
        const int i = v / (BK / 8), kq = v % (BK / 8);
        uint4 w;
        w.x = (uint32_t)regs[p][0] | ((uint32_t)regs[p][1] << 16);
        w.y = (uint32_t)regs[p][2] | ((uint32_t)regs[p][3] << 16);
        w.z = (uint32_t)regs[p][4] | ((uint32_t)regs[p][5] << 16);
        w.w = (uint32_t)regs[p][6] | ((uint32_t)regs[p][7] << 16);
        *reinterpret_cast<uint4*>(s + i * PADK + kq * 8) = w;
      } else {
        const int k = v / (ROWS / 8), iq = v % (ROWS / 8);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[(iq * 8 + j) * PADK + k] = regs[p][j];
      }
    }
  }
}

// Epilogue contract: store(m, n, value, valid) for every element of the tile;
// the kernel passes valid = (m < M && n < N).
template <int BM, int BN, int WM, int WN, int WK, class LA, class LB, class EPI>
__global__ __launch_bounds__(256) void k_gemm(LA la, LB lb, EPI epi, int M, int N, int K, int k_split) {
  using C = Cfg<BM, BN, WM, WN, WK>;
  __shared__ __align__(16) uint16_t sA[2][BM * PADK];
  __shared__ __align__(16) uint16_t sB[2][BN * PADK];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wk = wave % WK;
  const int wmn = wave / WK;
  const int wm = wmn / WN, wn = wmn % WN;
  const int m_blk = blockIdx.x * BM, n_blk = blockIdx.y * BN;   // M tiles on x (up to 2^31 - 1)
  const int kb = blockIdx.z * k_split;
  const int ke = min(K, kb + k_split);
  f32x4 acc[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  uint16_t ra[C::PA][8], rb[C::PB][8];
  const int nsteps = (ke - kb + BK - 1) / BK;
  if (nsteps > 0) {
    fetch_tile<LA, BM>(la, m_blk, kb, ra, C::PA);
    fetch_tile<LB, BN>(lb, n_blk, kb, rb, C::PB);
    store_tile<LA, BM>(sA[0], ra, C::PA);
    store_tile<LB, BN>(sB[0], rb, C::PB);
  }
  __syncthreads();
  for (int t = 0; t < nsteps; ++t) {
    const int buf = t & 1;
    const bool more = t + 1 < nsteps;
    if (more) {
      fetch_tile<LA, BM>(la, m_blk, kb + (t + 1) * BK, ra, C::PA);
      fetch_tile<LB, BN>(lb, n_blk, kb + (t + 1) * BK, rb, C::PB);
    }
    if ((t % WK) == wk) {
      const uint16_t* a_base = sA[buf] + (wm * C::TM + (lane & 15)) * PADK + 8 * (lane >> 4);
      const uint16_t* b_base = sB[buf] + (wn * C::TN + (lane & 15)) * PADK + 8 * (lane >> 4);
      bf16x8 bf[C::FN];
#pragma unroll
      for (int j = 0; j < C::FN; ++j)
        bf[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(b_base + j * 16 * PADK));
#pragma unroll
      for (int i = 0; i < C::FM; ++i) {
        const bf16x8 af = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(a_base + i * 16 * PADK));
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      store_tile<LA, BM>(sA[buf ^ 1], ra, C::PA);
      store_tile<LB, BN>(sB[buf ^ 1], rb, C::PB);
    }
    __syncthreads();
  }
  if (WK > 1) {
    // sum the K-split waves through LDS (reuses the staging buffers)
    float* red = reinterpret_cast<float*>(&sA[0][0]);
    constexpr int per_wave = C::FM * C::FN * 4 * 64;
    static_assert((WK - 1) * (4 / WK) * per_wave * 4 <= (int)sizeof(sA) + (int)sizeof(sB), "reduction space");
    if (wk > 0) {
      float* dst = red + ((wk - 1) * (4 / WK) + wmn) * per_wave;
#pragma unroll
      for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) dst[((i * C::FN + j) * 4 + e) * 64 + lane] = acc[i][j][e];
    }
    __syncthreads();
    if (wk == 0) {
      for (int q = 1; q < WK; ++q) {
        const float* src = red + ((q - 1) * (4 / WK) + wmn) * per_wave;
#pragma unroll
        for (int i = 0; i < C::FM; ++i)
#pragma unroll
          for (int j = 0; j < C::FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i][j][e] += src[((i * C::FN + j) * 4 + e) * 64 + lane];
      }
    }
    if (wk != 0) return;
  }
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m_blk + wm * C::TM + i * 16 + 4 * (lane >> 4) + e;
        const int n = n_blk + wn * C::TN + j * 16 + (lane & 15);
        epi.store(m, n, acc[i][j][e], m < M && n < N);
      }
}

template <int BM, int BN, int WM, int WN, int WK, class LA, class LB, class EPI>
hipError_t run(const LA& la, const LB& lb, const EPI& epi, int M, int N, int K, int splits, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  int k_split = (K + splits - 1) / splits;
  k_split = (k_split + BK - 1) / BK * BK;
  const int nz = K > 0 ? (K + k_split - 1) / k_split : 1;
  if ((N + BN - 1) / BN > 65535 || nz > 65535) return hipErrorInvalidValue;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, nz);
  k_gemm<BM, BN, WM, WN, WK, LA, LB, EPI><<<grid, 256, 0, st>>>(la, lb, epi, M, N, K, k_split);
  return hipGetLastError();
}

}  // namespace gemm
}  // namespace aslam
