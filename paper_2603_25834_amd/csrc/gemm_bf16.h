// gemm_bf16.h -- generic BF16 x BF16 -> FP32 MFMA GEMM for gfx950 (library-internal).
//
// C[M,N] = sum_k A[m,k] B[k,n] with operands fetched through loader functors
// (so a GEMM can read a transposed matrix or a concatenation without
// materialising it) and results handed to an epilogue functor (bias, ReLU,
// masks, BF16 stores, split-K partial sums).
//
// Tiling: a workgroup of 256 threads (4 waves) owns a BM x BN tile of C; the
// waves are arranged WM x WN and each accumulates a (BM/WM) x (BN/WN) sub-tile
// in 16x16 MFMA fragments.  K advances BK per stage, double buffered in LDS,
// with the global loads of the next two stages in registers while the current
// stage feeds the MFMAs (one stage ahead on edge tiles).  Both operands are staged as [row][k]
// (rows padded by 8 elements) and read as one 16-byte fragment per lane.  An
// operand whose source is contiguous along the row index is transposed on the
// way in: a thread loads the same eight rows at k and k + 1 and stores eight
// 32-bit (k, k + 1) pairs; the 16-byte chunks of a row are XOR-swizzled with
// (row / 8) so that those stores, eight rows apart across lanes, spread over
// the LDS banks.
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
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // staged loads (a plain vector type stays in registers)

// Round-to-nearest-even FP32 -> BF16 bits: the hardware conversion (v_cvt_pk_bf16_f32 on gfx950,
// two values per instruction when the compiler pairs them).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
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
// columns n0 .. n0 + 7 (n0 multiple of 8), of which the first nvalid are < N;
// an epilogue of split-K partial sums declares kSliced = true and provides
// store8z(z, m, n0, v, nvalid) instead, z being the K slice of the workgroup.
// An epilogue that reads global memory declares kPrefetch = true and provides
// fetch(m, n0, nvalid) -> uint4 and store8_pre(m, n0, v, nvalid, fetched): the
// engine issues those reads at kernel start, so their latency hides behind the
// main loop (others declare kPrefetch = false).

// Several products in one launch (the split-precision forward: hi x hi, hi x lo, lo x hi): an operand
// given as HiLo reads its `lo` matrix in product p when bit p of lo_mask is set, else its `hi` matrix
// (a plain loader is the same in every product).  Two ways to lay them out: over the z index, each
// product into its own group of K slices (more workgroups in flight: the wide FC1), or inside the
// workgroup, its K loop run once per product with the accumulator carried across (no extra partial
// sums, so a bias epilogue can finish the sum directly: the short-K FC2).
template <class L>
struct HiLo {
  L hi, lo;
  unsigned lo_mask;
};

template <class L>
__device__ __forceinline__ L bind_product(const L& l, int) { return l; }
template <class L>
__device__ __forceinline__ L bind_product(const HiLo<L>& l, int p) { return ((l.lo_mask >> p) & 1u) ? l.lo : l.hi; }

template <class L>
struct BoundT {
  using type = L;
};
template <class L>
struct BoundT<HiLo<L>> {
  using type = L;
};
template <class L>
using Bound = typename BoundT<L>::type;

// LDS elements of one stage of an operand with ROWS rows ([row][k], rows padded by 8).
template <bool KMAJOR, int ROWS, int BK>
struct Stage {
  static constexpr int kLd = BK + 8;
  static constexpr int kElems = ROWS * kLd;
  // element (r, k) of a transposed (!KMAJOR) stage: 16-byte chunk k / 8 swizzled with (r / 8)
  __device__ static __forceinline__ int at(int r, int k) {
    return KMAJOR ? r * kLd + k : r * kLd + ((((k >> 3) ^ (r >> 3)) & (BK / 8 - 1)) << 3) + (k & 7);
  }
};

template <int BM, int BN, int BK, int WM, int WN>
struct Cfg {
  static_assert(WM * WN == 4, "four waves");
  static constexpr int TM = BM / WM, TN = BN / WN;   // wave sub-tile
  static constexpr int FM = TM / 16, FN = TN / 16;   // fragments per wave
  static_assert(FM * 16 == TM && FN * 16 == TN, "fragment tiling");
  static_assert(BK % 32 == 0, "BK is a multiple of the MFMA depth");
  static constexpr int VA = BM * BK / 8, VB = BN * BK / 8;            // 8-element vectors per stage
  // vectors per thread, rounded up to even (a transposed operand is fetched in pairs)
  static constexpr int PA = ((VA + 255) / 256 + 1) & ~1, PB = ((VB + 255) / 256 + 1) & ~1;
  static constexpr int kEpiBytes = BM * (BN + 4) * 4;                 // FP32 tile (rows padded)
};

// kMajor: register p holds vector v = tid + 256 p = (row v / (BK/8), k-chunk v % (BK/8)).
// !kMajor: registers 2q, 2q + 1 hold pair w = tid + 256 q = (k = 2 (w / (ROWS/8)), row-chunk w % (ROWS/8))
// at k and k + 1 (consecutive lanes read consecutive row-chunks of the same source rows).
// Element offsets, from the tile origin, of the vectors fetch_tile loads into this thread's registers
// (the same assignment as fetch_tile), used by the unchecked path for tiles that lie wholly inside a
// plain strided matrix (loader fields p, ld, rows, cols): 256 threads cover whole rows (k-major) or
// whole k pairs, so the offset of register p (pair q) is base + p * step (base + q * step, + ld for k + 1).
struct TileOff {
  int64_t base, step;
};

template <class L, int ROWS, int BK>
__device__ __forceinline__ TileOff tile_offsets(const L& ld) {
  static_assert(256 % (BK / 8) == 0 && 256 % (ROWS / 8) == 0, "256 threads cover whole rows / k pairs");
  TileOff o;
  if (L::kMajor) {
    o.base = (int64_t)(threadIdx.x / (BK / 8)) * ld.ld + (threadIdx.x % (BK / 8)) * 8;
    o.step = (int64_t)(256 / (BK / 8)) * ld.ld;
  } else {
    o.base = (int64_t)(2 * (threadIdx.x / (ROWS / 8))) * ld.ld + (threadIdx.x % (ROWS / 8)) * 8;
    o.step = (int64_t)(2 * (256 / (ROWS / 8))) * ld.ld;
  }
  return o;
}

// The tile at (row0, k0) lies wholly inside the matrix and its rows start on 16-byte boundaries.
template <class L, int ROWS, int BK>
__device__ __forceinline__ bool tile_interior(const L& ld, int row0, int k0) {
  return row0 + ROWS <= ld.rows && k0 + BK <= ld.cols && (ld.ld & 7) == 0 &&
         (reinterpret_cast<uintptr_t>(ld.p) & 15) == 0;
}

// The loads of a tile known to lie wholly inside the matrix, with no branch, so that a
// software-pipelined loop issues a fixed number of loads per step.
template <class L, int ROWS, int BK, int P>
__device__ __forceinline__ void fetch_fast(const L& ld, int row0, int k0, u32x4 (&regs)[P], const TileOff& off) {
  constexpr int V = ROWS * BK / 8;
  const uint16_t* base = (L::kMajor ? ld.p + (int64_t)row0 * ld.ld + k0 : ld.p + (int64_t)k0 * ld.ld + row0) + off.base;
  if (L::kMajor) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int v = threadIdx.x + p * 256;
      if (V % 256 == 0 || v < V) regs[p] = *reinterpret_cast<const u32x4*>(base + p * off.step);
    }
  } else {
#pragma unroll
    for (int q = 0; q < P / 2; ++q) {
      const int w = threadIdx.x + q * 256;
      if (V / 2 % 256 == 0 || w < V / 2) {
        regs[2 * q] = *reinterpret_cast<const u32x4*>(base + q * off.step);
        regs[2 * q + 1] = *reinterpret_cast<const u32x4*>(base + q * off.step + ld.ld);
      }
    }
  }
}

template <class L, int ROWS, int BK, int P>
__device__ __forceinline__ void fetch_tile(const L& ld, int row0, int k0, u32x4 (&regs)[P], const TileOff& off) {
  constexpr int V = ROWS * BK / 8;
  if (tile_interior<L, ROWS, BK>(ld, row0, k0)) {
    fetch_fast<L, ROWS, BK>(ld, row0, k0, regs, off);
    return;
  }
  if (L::kMajor) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int v = threadIdx.x + p * 256;
      if (V % 256 == 0 || v < V) {
        const int i = v / (BK / 8), kq = v % (BK / 8);
        const uint4 u = ld.fetch(row0 + i, k0 + kq * 8);
        regs[p] = u32x4{u.x, u.y, u.z, u.w};
      }
    }
  } else {
    constexpr int VP = V / 2;
#pragma unroll
    for (int q = 0; q < P / 2; ++q) {
      const int w = threadIdx.x + q * 256;
      if (VP % 256 == 0 || w < VP) {
        const int k = 2 * (w / (ROWS / 8)), iq = w % (ROWS / 8);
        const uint4 u0 = ld.fetch(row0 + iq * 8, k0 + k), u1 = ld.fetch(row0 + iq * 8, k0 + k + 1);
        regs[2 * q] = u32x4{u0.x, u0.y, u0.z, u0.w};
        regs[2 * q + 1] = u32x4{u1.x, u1.y, u1.z, u1.w};
      }
    }
  }
}

// The rows row0 .. row0 + ROWS - 1 of the operand lie inside the matrix and its rows start on 16-byte
// boundaries (every K step of such a tile that ends by ld.cols is interior).
template <class L, int ROWS>
__device__ __forceinline__ bool rows_interior(const L& ld, int row0) {
  return row0 + ROWS <= ld.rows && (ld.ld & 7) == 0 && (reinterpret_cast<uintptr_t>(ld.p) & 15) == 0;
}

template <class L, int ROWS, int BK, int P>
__device__ __forceinline__ void store_tile(uint16_t* s, const u32x4 (&regs)[P]) {
  using S = Stage<L::kMajor, ROWS, BK>;
  constexpr int V = ROWS * BK / 8;
  if (L::kMajor) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int v = threadIdx.x + p * 256;
      if (V % 256 == 0 || v < V) {
        const int i = v / (BK / 8), kq = v % (BK / 8);
        *reinterpret_cast<u32x4*>(s + S::at(i, kq * 8)) = regs[p];
      }
    }
  } else {
    constexpr int VP = V / 2;
#pragma unroll
    for (int q = 0; q < P / 2; ++q) {
      const int w = threadIdx.x + q * 256;
      if (VP % 256 == 0 || w < VP) {
        const int k = 2 * (w / (ROWS / 8)), iq = w % (ROWS / 8);
        const u32x4 a = regs[2 * q], b = regs[2 * q + 1];
        const uint32_t wa[4] = {a[0], a[1], a[2], a[3]}, wb[4] = {b[0], b[1], b[2], b[3]};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t lo = (wa[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
          const uint32_t hi = (wb[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
          *reinterpret_cast<uint32_t*>(s + S::at(iq * 8 + j, k)) = lo | (hi << 16);
        }
      }
    }
  }
}

// MFMA fragment of row r (tile-local) and k values kk .. kk + 7 (kk multiple of 8).
template <bool KMAJOR, int ROWS, int BK>
__device__ __forceinline__ bf16x8 load_frag(const uint16_t* s, int r, int kk) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(s + Stage<KMAJOR, ROWS, BK>::at(r, kk)));
}

// The MFMAs of one staged K step: the wave's FM x FN fragments of C, BK / 32 products each.
template <int BM, int BN, int BK, int WM, int WN, bool AMAJ, bool BMAJ>
__device__ __forceinline__ void mma_stage(const uint16_t* a_st, const uint16_t* b_st, int ra0, int rb0, int kl,
                                          f32x4 (&acc)[Cfg<BM, BN, BK, WM, WN>::FM][Cfg<BM, BN, BK, WM, WN>::FN]) {
  using C = Cfg<BM, BN, BK, WM, WN>;
#pragma unroll
  for (int kk = 0; kk < BK; kk += 32) {
    bf16x8 bf[C::FN];
#pragma unroll
    for (int j = 0; j < C::FN; ++j) bf[j] = load_frag<BMAJ, BN, BK>(b_st, rb0 + j * 16, kk + kl);
#pragma unroll
    for (int i = 0; i < C::FM; ++i) {
      const bf16x8 af = load_frag<AMAJ, BM, BK>(a_st, ra0 + i * 16, kk + kl);
#pragma unroll
      for (int j = 0; j < C::FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j], acc[i][j], 0, 0, 0);
    }
  }
}

// Tile (tm, tn, tz) of the workgroup.  The dispatcher hands consecutive workgroups of a grid to the
// eight XCDs in turn, and each XCD has its own L2, so the tiles that share an operand are given to
// workgroups eight apart: workgroup L runs on XCD L % 8 as that XCD's (L / 8)-th, and the XCDs take
// consecutive runs of the tile order.  That order walks groups of kGroupM tile rows: within a group,
// the rows vary fastest and the columns next, so a B panel is read by kGroupM workgroups in a row
// and the group's A panels stay in the XCD's L2 across all columns; the K slice varies slowest.
constexpr int kGroupM = 8;

struct TileId {
  int tm, tn, tz;
};

__device__ __forceinline__ TileId xcd_tile() {
  const int nx = gridDim.x, ny = gridDim.y;
  const int64_t total = (int64_t)nx * ny * gridDim.z;
  const int64_t L = blockIdx.x + (int64_t)nx * (blockIdx.y + (int64_t)ny * blockIdx.z);
  const int64_t q = total >> 3, r = total & 7, xcd = L & 7, j = L >> 3;
  const int64_t V = xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
  TileId t;
  const int64_t plane = (int64_t)nx * ny;
  t.tz = (int)(V / plane);
  const int64_t w = V - (int64_t)t.tz * plane;
  const int64_t g = w / ((int64_t)kGroupM * ny), rg = w - g * kGroupM * ny;
  const int gm = min(kGroupM, nx - (int)g * kGroupM);
  t.tm = (int)g * kGroupM + (int)(rg % gm);
  t.tn = (int)(rg / gm);
  return t;
}

template <int BM, int BN, int BK, int WM, int WN, class LA0, class LB0, class EPI>
__global__ __launch_bounds__(256) void k_gemm(LA0 la0, LB0 lb0, EPI epi, int M, int N, int K, int k_split,
                                              int zper, int kprod) {
  using LA = Bound<LA0>;
  using LB = Bound<LB0>;
  using C = Cfg<BM, BN, BK, WM, WN>;
  using SA = Stage<LA::kMajor, BM, BK>;
  using SB = Stage<LB::kMajor, BN, BK>;
  constexpr int kStageBytes = 2 * (SA::kElems + SB::kElems) * 2;   // double-buffered A and B
  constexpr int kLds = kStageBytes > C::kEpiBytes ? kStageBytes : C::kEpiBytes;
  __shared__ __align__(16) unsigned char smem[kLds];
  uint16_t* sA = reinterpret_cast<uint16_t*>(smem);           // [2][SA::kElems]
  uint16_t* sB = sA + 2 * SA::kElems;                         // [2][SB::kElems]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave / WN, wn = wave % WN;
  const TileId tile = xcd_tile();
  const int m_blk = tile.tm * BM, n_blk = tile.tn * BN;   // M tiles on x (up to 2^31 - 1)
  const int zg = zper > 0 ? tile.tz / zper : 0;   // product group of the z index
  const int kb = (tile.tz - zg * zper) * k_split;
  const int ke = min(K, kb + k_split);
  f32x4 acc[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // epilogue vectors of this thread: v = threadIdx.x + 256 i, row v / (BN/8), columns 8 (v % (BN/8)) ..
  constexpr int kVecPerRow = BN / 8;
  constexpr int kEpiVec = (BM * kVecPerRow + 255) / 256;
  uint4 epre[EPI::kPrefetch ? kEpiVec : 1];
  if constexpr (EPI::kPrefetch) {
#pragma unroll
    for (int i = 0; i < kEpiVec; ++i) {
      const int v = threadIdx.x + 256 * i;
      const int m = m_blk + v / kVecPerRow, n0 = n_blk + (v % kVecPerRow) * 8;
      epre[i] = (v < BM * kVecPerRow && m < M && n0 < N) ? epi.fetch(m, n0, min(8, N - n0))
                                                           : make_uint4(0u, 0u, 0u, 0u);
    }
  }
  const int nsteps = (ke - kb + BK - 1) / BK;
  const int ra0 = wm * C::TM + (lane & 15), rb0 = wn * C::TN + (lane & 15), kl = 8 * (lane >> 4);
  uint16_t* const sA1 = sA + SA::kElems;
  uint16_t* const sB1 = sB + SB::kElems;
  for (int ip = 0; ip < kprod; ++ip) {   // every path below ends at a barrier: the stages are free again
  const LA la = bind_product(la0, zg * kprod + ip);
  const LB lb = bind_product(lb0, zg * kprod + ip);
  const TileOff oa = tile_offsets<LA, BM, BK>(la), ob = tile_offsets<LB, BN, BK>(lb);
  // Steps whose tiles are interior in both operands (rows inside, K step whole) run a loop with two
  // stages of loads in registers: step t's MFMAs overlap the loads of step t + 2, and the stores of
  // step t + 1 wait only for loads issued a whole step earlier.  Every step issues the same loads
  // (past the last step they re-read it), so the waits are exact counts.
  // (An epilogue that prefetches holds its own registers through the loop: one stage there.)
  int nfast = 0;
  if (!EPI::kPrefetch && rows_interior<LA, BM>(la, m_blk) && rows_interior<LB, BN>(lb, n_blk))
    nfast = max(0, (min(ke, min(la.cols, lb.cols)) - kb) / BK);
  int t = 0;
  u32x4 ra_e[C::PA], rb_e[C::PB], ra_o[C::PA], rb_o[C::PB];   // even / odd steps (the edge loop: ra_e, rb_e)
  if (nfast > 0) {
    fetch_fast<LA, BM, BK>(la, m_blk, kb, ra_e, oa);
    fetch_fast<LB, BN, BK>(lb, n_blk, kb, rb_e, ob);
    const int k1 = kb + BK * min(1, nfast - 1);
    fetch_fast<LA, BM, BK>(la, m_blk, k1, ra_o, oa);
    fetch_fast<LB, BN, BK>(lb, n_blk, k1, rb_o, ob);
    store_tile<LA, BM, BK>(sA, ra_e);
    store_tile<LB, BN, BK>(sB, rb_e);
    __syncthreads();
    for (; t + 2 <= nfast; t += 2) {
      const int k2 = kb + BK * min(t + 2, nfast - 1);
      fetch_fast<LA, BM, BK>(la, m_blk, k2, ra_e, oa);
      fetch_fast<LB, BN, BK>(lb, n_blk, k2, rb_e, ob);
      mma_stage<BM, BN, BK, WM, WN, LA::kMajor, LB::kMajor>(sA, sB, ra0, rb0, kl, acc);
      store_tile<LA, BM, BK>(sA1, ra_o);
      store_tile<LB, BN, BK>(sB1, rb_o);
      __syncthreads();
      const int k3 = kb + BK * min(t + 3, nfast - 1);
      fetch_fast<LA, BM, BK>(la, m_blk, k3, ra_o, oa);
      fetch_fast<LB, BN, BK>(lb, n_blk, k3, rb_o, ob);
      mma_stage<BM, BN, BK, WM, WN, LA::kMajor, LB::kMajor>(sA1, sB1, ra0, rb0, kl, acc);
      if (t + 2 < nfast) {
        store_tile<LA, BM, BK>(sA, ra_e);
        store_tile<LB, BN, BK>(sB, rb_e);
      }
      __syncthreads();
    }
    if (t < nfast) {   // an odd count: the last step is in buffer 0
      mma_stage<BM, BN, BK, WM, WN, LA::kMajor, LB::kMajor>(sA, sB, ra0, rb0, kl, acc);
      __syncthreads();
      ++t;
    }
  }
  // the remaining steps (edge tiles, a partial last K step): bounds-checked loads, one stage ahead
  if (t < nsteps) {
    fetch_tile<LA, BM, BK>(la, m_blk, kb + t * BK, ra_e, oa);
    fetch_tile<LB, BN, BK>(lb, n_blk, kb + t * BK, rb_e, ob);
    store_tile<LA, BM, BK>(sA, ra_e);
    store_tile<LB, BN, BK>(sB, rb_e);
    __syncthreads();
    for (int u = 0; t < nsteps; ++t, ++u) {
      const int buf = u & 1;
      const bool more = t + 1 < nsteps;
      if (more) {
        fetch_tile<LA, BM, BK>(la, m_blk, kb + (t + 1) * BK, ra_e, oa);
        fetch_tile<LB, BN, BK>(lb, n_blk, kb + (t + 1) * BK, rb_e, ob);
      }
      mma_stage<BM, BN, BK, WM, WN, LA::kMajor, LB::kMajor>(sA + buf * SA::kElems, sB + buf * SB::kElems, ra0, rb0, kl,
                                                             acc);
      if (more) {
        store_tile<LA, BM, BK>(sA + (buf ^ 1) * SA::kElems, ra_e);
        store_tile<LB, BN, BK>(sB + (buf ^ 1) * SB::kElems, rb_e);
      }
      __syncthreads();
    }
  }
  }   // products
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
#pragma unroll
  for (int i = 0; i < kEpiVec; ++i) {
    const int v = threadIdx.x + 256 * i;
    const int r = v / kVecPerRow, c0 = (v % kVecPerRow) * 8;
    const int m = m_blk + r, n0 = n_blk + c0;
    if (v >= BM * kVecPerRow || m >= M || n0 >= N) continue;
    const float4 lo = *reinterpret_cast<const float4*>(sc + r * LDC + c0);
    const float4 hi = *reinterpret_cast<const float4*>(sc + r * LDC + c0 + 4);
    const float vals[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    if constexpr (EPI::kPrefetch) epi.store8_pre(m, n0, vals, min(8, N - n0), epre[i]);
    else if constexpr (EPI::kSliced) epi.store8z(tile.tz, m, n0, vals, min(8, N - n0));
    else epi.store8(m, n0, vals, min(8, N - n0));
  }
}

// `products` products (HiLo operands), K split `splits` ways (nz = the slices K actually splits into):
// over z, product p's slice z at z index p * nz + z (in_kernel = false); or summed in each workgroup,
// slice z at z index z (in_kernel = true).
template <int BM, int BN, int BK, int WM, int WN, class LA, class LB, class EPI>
hipError_t run(const LA& la, const LB& lb, const EPI& epi, int M, int N, int K, int splits, hipStream_t st,
               int products = 1, bool in_kernel = false) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  if (products < 1) products = 1;
  int k_split = (K + splits - 1) / splits;
  k_split = (k_split + BK - 1) / BK * BK;
  const int nz = K > 0 ? (K + k_split - 1) / k_split : 1;
  const int zprod = in_kernel ? 1 : products;
  if ((N + BN - 1) / BN > 65535 || (int64_t)nz * zprod > 65535) return hipErrorInvalidValue;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, nz * zprod);
  k_gemm<BM, BN, BK, WM, WN, LA, LB, EPI><<<grid, 256, 0, st>>>(la, lb, epi, M, N, K, k_split,
                                                                 zprod > 1 ? nz : 0, in_kernel ? products : 1);
  return hipGetLastError();
}

}  // namespace gemm
}  // namespace aslam
