// conv_fused.h -- the actor-critic's convolutional encoder in one kernel (gfx950).
//
// conv1 (1 -> 16) and conv2 (16 -> 32), both 3x3 with stride 2 and padding 1
// and ReLU, for one sample at a time per workgroup, with the 32x32x16 conv1
// activation kept in LDS: HBM sees only the 64x64 int16 crop coming in and the
// 8192 BF16 features going out.  Both convolutions run on MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation) with the same rounding points
// as the layer-by-layer path: crop L/256, weights and activations in BF16.
//
// conv1 is written as C'[co][px] = sum_k W'[co][k] P[k][px] over a 4x4 input
// window per output pixel: the crop is stored in LDS space-to-depth (2x2
// blocks of 8 bytes), so the window of pixel (y, x) is the four blocks at
// block rows y-1, y and block columns x-1, x, and a lane's eight k values are
// two adjacent blocks (two 8-byte reads).  k = 8r + 4c + 2dy + dx addresses
// block row r, block column c and the element (dy, dx) inside it, which is
// input row 2y - 2 + 2r + dy, i.e. tap ky = 2r + dy - 1 (likewise kx); taps
// outside 0..2 carry a zero weight.  The transposed product hands each lane
// four consecutive channels of one pixel, one 8-byte LDS store.
//
// conv2 is C[pos][co] = sum_k col[pos][k] W2[k][co] with k = tap*16 + ci
// (K = 144 padded to 160): a lane's eight k values are eight channels of one
// a1 pixel, one 16-byte LDS read; the weights stay in registers for the
// workgroup's lifetime.  Each lane then holds four consecutive positions of
// one output channel, one 8-byte store into a2[b][co*256 + pos].
//
// Split precision (PREC): every operand v of both convolutions is carried as
// two BF16 numbers, hi = bf16(v) and lo = bf16(v - hi) (16 significant bits;
// the crop L/256 is exact), and each product is hi*hi + hi*lo + lo*hi on
// MFMA (the lo*lo term is below FP32 resolution of the sum), so the ReLU
// pre-activations are FP32-accurate and a ReLU sees the sign the exact
// network gives; the outputs (a1 and the FC1 input) are stored as hi and lo.
#pragma once

#include "policy_kernels.h"

namespace aslam {
namespace pol {

using gemm::bf16x8;
using gemm::f32x4;

constexpr int kBlk = 33;                 // crop 2x2 blocks per row and column, plus the zero block -1
constexpr int kA1Row = 33;               // a1 pixels per row and column, plus the zero pixel -1
constexpr int kCropLds = kBlk * kBlk * 4;            // BF16 elements
constexpr int kA1Lds = kA1Row * kA1Row * kC1;        // BF16 elements

// a1 pixel (y, x), x, y in [-1, 31], of the forward kernel's LDS copy: rows of 33
// pixel slots with even x + 1 in slots 0..16 and odd x + 1 in slots 17..32, so
// that conv2's stride-2 reads along x hit consecutive slots (different banks).
__device__ __forceinline__ int a1_slot(int y, int x) {
  return (y + 1) * kA1Row + ((x + 1) & 1) * 17 + ((x + 1) >> 1);
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
}

// hi = bf16(v), or with LO the remainder bf16(v - hi).
template <bool LO>
__device__ __forceinline__ uint16_t bf16_part(float v) {
  const uint16_t h = f2bf(v);
  return LO ? f2bf(v - bf2f(h)) : h;
}

// conv1 weights as the A operand: lane supplies W'[co = lane % 16][k = 8 (lane / 16) + j].
template <bool LO = false>
__device__ __forceinline__ bf16x8 conv1_weight_frag(const float* w1, int lr, int lg) {
  uint16_t v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * lg + j;
    const int r = k >> 3, c = (k >> 2) & 1, dy = (k >> 1) & 1, dx = k & 1;
    const int ky = 2 * r + dy - 1, kx = 2 * c + dx - 1;
    v[j] = (lg < 2 && ky >= 0 && kx >= 0) ? bf16_part<LO>(w1[lr * 9 + ky * 3 + kx]) : (uint16_t)0;
  }
  uint4 u;
  u.x = v[0] | ((uint32_t)v[1] << 16);
  u.y = v[2] | ((uint32_t)v[3] << 16);
  u.z = v[4] | ((uint32_t)v[5] << 16);
  u.w = v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}

// conv2 weights as the B operand: lane supplies W2[k = 32 s + 8 (lane / 16) + j][co], k = tap*16 + ci.
template <bool LO = false>
__device__ __forceinline__ bf16x8 conv2_weight_frag(const float* w2, int co, int s, int lg) {
  uint16_t v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 32 * s + 8 * lg + j, tap = k >> 4, ci = k & 15;
    v[j] = tap < 9 ? bf16_part<LO>(w2[(co * kC1 + ci) * 9 + tap]) : (uint16_t)0;
  }
  uint4 u;
  u.x = v[0] | ((uint32_t)v[1] << 16);
  u.y = v[2] | ((uint32_t)v[3] << 16);
  u.z = v[4] | ((uint32_t)v[5] << 16);
  u.w = v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}

// The forward's weight fragments, formed once per parameter update: fragment f < 11 of lane l at
// frag[64 f + l]; f = 0 is conv1's A operand, f = 1 + 5 nt + s is conv2's B operand for output
// channels 16 nt .. 16 nt + 15 and k slice s (the values conv1_weight_frag / conv2_weight_frag give).
// With LO the same fragments of the weights' lo parts, written from frag[64 kConvLoFrag] on.
constexpr int kConvFrags = 11;

template <bool LO = false>
__device__ __forceinline__ void conv_frag_elem(const float* prm, const Offsets& o, uint4* frag, int idx) {
  const int f = idx >> 6, lane = idx & 63, lr = lane & 15, lg = lane >> 4;
  bf16x8 v;
  if (f == 0) {
    v = conv1_weight_frag<LO>(prm + o.c1w, lr, lg);
  } else {
    const int nt = (f - 1) / 5, s = (f - 1) % 5;
    v = conv2_weight_frag<LO>(prm + o.c2w, 16 * nt + lr, s, lg);
  }
  frag[idx] = __builtin_bit_cast(uint4, v);
}

template <bool LO = false>
__global__ __launch_bounds__(64 * kConvFrags) void k_conv_frags(const float* prm, Offsets o, uint4* frag) {
  conv_frag_elem<LO>(prm, o, frag, threadIdx.x);
}

// A 64x64 int16 crop is 512 vectors of eight cells (row y = v / 8, columns
// 8 (v % 8) .. + 7); a workgroup of NT threads holds 512 / NT of them per
// thread in registers, so the next sample's crop can be in flight while the
// current one is processed.
template <int NT>
struct CropRegs {
  static constexpr int kPer = kCrop * kCrop / 8 / NT;
  int4 v[kPer];
};

template <int NT>
__device__ __forceinline__ void load_crop(const int16_t* src, CropRegs<NT>& r) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
#pragma unroll
  for (int i = 0; i < CropRegs<NT>::kPer; ++i) r.v[i] = s4[threadIdx.x + i * NT];
}

// Crop registers into LDS, space-to-depth, as BF16(L / 256) (with LO its lo part).  Block (Y, X)
// sits at ((Y + 1) * 33 + X + 1) * 4; the row and column of index 0 are the
// zero padding and are never written here.
template <int NT, bool LO = false>
__device__ __forceinline__ void store_crop(const CropRegs<NT>& r, uint16_t* s_crop) {
#pragma unroll
  for (int i = 0; i < CropRegs<NT>::kPer; ++i) {
    const int v = threadIdx.x + i * NT;
    const int y = v >> 3, x0 = (v & 7) * 8;
    const int32_t w[4] = {r.v[i].x, r.v[i].y, r.v[i].z, r.v[i].w};
    const int Y = y >> 1, dy = y & 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float lo = (float)(int16_t)(w[q] & 0xffff) * (1.0f / 256.0f);
      const float hi = (float)(int16_t)(w[q] >> 16) * (1.0f / 256.0f);
      const int X = (x0 >> 1) + q;
      *reinterpret_cast<uint32_t*>(s_crop + ((Y + 1) * kBlk + X + 1) * 4 + 2 * dy) =
          (uint32_t)bf16_part<LO>(lo) | ((uint32_t)bf16_part<LO>(hi) << 16);
    }
  }
}

// conv1 window operand of pixel px (lanes with lg >= 2 supply zeros) from a space-to-depth crop.
__device__ __forceinline__ uint4 conv1_window(const uint16_t* s_crop, int px, int lg) {
  const int y = px >> 5, x = px & 31;
  if (lg >= 2) return make_uint4(0u, 0u, 0u, 0u);
  const uint16_t* q = s_crop + ((y + lg) * kBlk + x) * 4;
  const uint2 a = *reinterpret_cast<const uint2*>(q);
  const uint2 c = *reinterpret_cast<const uint2*>(q + 4);
  return make_uint4(a.x, a.y, c.x, c.y);
}

// Four ReLU outputs packed as BF16 (hi parts, or with LO the lo parts).
template <bool LO>
__device__ __forceinline__ uint2 pack_relu4(const f32x4& acc, const float b[4]) {
  uint16_t h[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) h[e] = bf16_part<LO>(fmaxf(acc[e] + b[e], 0.0f));
  return make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
}

// conv1 + ReLU of the staged crop into s_a1 (pixel (y, x) at a1_slot(y, x) * 16): 64 tiles of 16 pixels
// over the NW waves, four at a time so that their operand reads are in flight together; PREC: the
// crop's and the weights' lo parts enter the product too, and a1's lo part goes to s_a1l.  The wave's
// tiles' LDS offsets are formed once for all samples: tile j of the wave is wave + NW j, win[j] the
// element offset of its window operand in the crop (-1: the lanes with lg >= 2, which supply zeros)
// and slot[j] that of its output in a1.
template <bool PREC, int NW>
__device__ __forceinline__ void conv1_lds_at(const uint16_t* s_crop, const uint16_t* s_cropl, uint16_t* s_a1,
                                             uint16_t* s_a1l, const bf16x8& w1f, const bf16x8& w1fl, const float b1[4],
                                             const int (&win)[kA1 * kA1 / 16 / NW],
                                             const int (&slot)[kA1 * kA1 / 16 / NW]) {
  constexpr int kT = kA1 * kA1 / 16 / NW;
  auto window = [&](const uint16_t* c, int off) -> uint4 {
    if (off < 0) return make_uint4(0u, 0u, 0u, 0u);
    const uint2 a = *reinterpret_cast<const uint2*>(c + off);
    const uint2 d = *reinterpret_cast<const uint2*>(c + off + 4);
    return make_uint4(a.x, a.y, d.x, d.y);
  };
#pragma unroll
  for (int j0 = 0; j0 < kT; j0 += 4) {
    uint4 u[4], ul[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      u[i] = window(s_crop, win[j0 + i]);
      if (PREC) ul[i] = window(s_cropl, win[j0 + i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f, __builtin_bit_cast(bf16x8, u[i]),
                                                         f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      if (PREC) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f, __builtin_bit_cast(bf16x8, ul[i]), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1fl, __builtin_bit_cast(bf16x8, u[i]), acc, 0, 0, 0);
      }
      *reinterpret_cast<uint2*>(s_a1 + slot[j0 + i]) = pack_relu4<false>(acc, b1);
      if (PREC) *reinterpret_cast<uint2*>(s_a1l + slot[j0 + i]) = pack_relu4<true>(acc, b1);
    }
  }
}

// Encoder forward: a2[b * lda2 + co*256 + oy*16 + ox] = bf16(relu(conv2(relu(conv1(crop_b))))), and
// the rest of the FC1 input row: a2[b * lda2 + 8192 + j] = bf16(scan_b[j]), then bf16(state_b), then
// zeros up to lda2.  Input row b is rows[b] of crop / scan / state (b itself when rows is NULL).
// The workgroup loops over samples; the next sample's crop and the first 512 elements of its
// scan / state tail are loaded into registers while the current one is processed, so no global read
// is waited on inside a sample (a longer tail, R > 500, reads its remainder directly).
constexpr int kConvFwdTailPre = 2;   // tail elements per thread held in registers

// The lo fragments of the split-precision path start at fragment kConvLoFrag (after the backward's).
constexpr int kConvLoFrag = 20;

// PREC: a2lo receives the lo parts of the same row (conv features and the scan / state tail), the
// products are split as described at the top, and the workgroup holds the crop and a1 twice (87 KB of
// LDS: one workgroup per CU, of NT = 512 threads so that eight waves share the CU).
template <bool PREC, int NT = 256>
__global__ __launch_bounds__(NT) void k_conv_fwd(const float* __restrict__ prm, Offsets o,
                                                  const uint4* __restrict__ frag, const int16_t* __restrict__ crop,
                                                  const float* __restrict__ scan, const float* __restrict__ state,
                                                  int R, const int32_t* __restrict__ rows, uint16_t* __restrict__ a2,
                                                  uint16_t* __restrict__ a2lo, int64_t lda2, int B) {
  constexpr int kCopies = PREC ? 2 : 1;
  __shared__ __align__(16) uint16_t s_crop[kCopies * kCropLds];
  __shared__ __align__(16) uint16_t s_a1[kCopies * kA1Lds];
  uint16_t* const s_cropl = s_crop + (PREC ? kCropLds : 0);
  uint16_t* const s_a1l = s_a1 + (PREC ? kA1Lds : 0);
  constexpr int NW = NT / 64;
  static_assert(NW == 4 || NW == 8, "four or eight waves");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  {
    uint4* z = reinterpret_cast<uint4*>(s_crop);
    for (int i = threadIdx.x; i < kCopies * kCropLds / 8; i += NT) z[i] = make_uint4(0u, 0u, 0u, 0u);
    z = reinterpret_cast<uint4*>(s_a1);
    for (int i = threadIdx.x; i < kCopies * kA1Lds / 8; i += NT) z[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  const bf16x8 w1f = __builtin_bit_cast(bf16x8, frag[lane]);
  const bf16x8 w1fl = PREC ? __builtin_bit_cast(bf16x8, frag[64 * kConvLoFrag + lane]) : w1f;
  float b1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) b1[i] = prm[o.c1b + 4 * lg + i];
  bf16x8 w2f[2][5], w2fl[2][5];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      w2f[nt][s] = __builtin_bit_cast(bf16x8, frag[64 * (1 + 5 * nt + s) + lane]);
      if (PREC) w2fl[nt][s] = __builtin_bit_cast(bf16x8, frag[64 * (kConvLoFrag + 1 + 5 * nt + s) + lane]);
    }
  const float b2[2] = {prm[o.c2b + lr], prm[o.c2b + 16 + lr]};
  const int tail = (int)(lda2 - kFeat);
  auto src = [&](int b) -> int64_t { return rows ? (int64_t)rows[b] : (int64_t)b; };
  auto tail_value = [&](int64_t sb, int j) -> float {
    return j < R ? scan[sb * R + j] : (j < R + 12 ? state[sb * 12 + (j - R)] : 0.0f);
  };
  CropRegs<NT> cr;
  float tv[kConvFwdTailPre];
  auto load_sample = [&](int b) {
    const int64_t sb = src(b);
    load_crop<NT>(crop + sb * kCrop * kCrop, cr);
#pragma unroll
    for (int i = 0; i < kConvFwdTailPre; ++i) {
      const int j = threadIdx.x + NT * i;
      tv[i] = j < tail ? tail_value(sb, j) : 0.0f;
    }
  };
  // the LDS offsets of the wave's conv1 tiles and conv2 operands are the same for every sample
  constexpr int kT1 = kA1 * kA1 / 16 / NW, kR2 = kA2 / NW;
  int c1_win[kT1], c1_slot[kT1], c2_off[kR2][5];
#pragma unroll
  for (int j = 0; j < kT1; ++j) {
    const int px = (wave + NW * j) * 16 + lr, y = px >> 5, x = px & 31;
    c1_win[j] = lg < 2 ? ((y + lg) * kBlk + x) * 4 : -1;
    c1_slot[j] = a1_slot(y, x) * kC1 + 4 * lg;
  }
#pragma unroll
  for (int i = 0; i < kR2; ++i)
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const int oy = wave + NW * i, k0 = 32 * s + 8 * lg, tap = k0 >> 4, ci0 = k0 & 15;
      c2_off[i][s] = tap < 9 ? a1_slot(2 * oy + tap / 3 - 1, 2 * lr + tap % 3 - 1) * kC1 + ci0 : -1;
    }
  auto col_frag = [&](const uint16_t* a, int off) -> bf16x8 {
    return __builtin_bit_cast(bf16x8, off < 0 ? make_uint4(0u, 0u, 0u, 0u) : *reinterpret_cast<const uint4*>(a + off));
  };
  if (blockIdx.x < B) load_sample(blockIdx.x);
  __syncthreads();
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    store_crop<NT>(cr, s_crop);
    if (PREC) store_crop<NT, true>(cr, s_cropl);
    uint16_t* row = a2 + (int64_t)b * lda2 + kFeat;
    uint16_t* rowl = PREC ? a2lo + (int64_t)b * lda2 + kFeat : row;
#pragma unroll
    for (int i = 0; i < kConvFwdTailPre; ++i) {
      const int j = threadIdx.x + NT * i;
      if (j < tail) {
        row[j] = j < R + 12 ? f2bf(tv[i]) : (uint16_t)0;
        if (PREC) rowl[j] = j < R + 12 ? bf16_part<true>(tv[i]) : (uint16_t)0;
      }
    }
    for (int j = threadIdx.x + NT * kConvFwdTailPre; j < tail; j += NT) {
      const float v = j < R + 12 ? tail_value(src(b), j) : 0.0f;
      row[j] = f2bf(v);
      if (PREC) rowl[j] = bf16_part<true>(v);
    }
    __syncthreads();
    // the next sample's crop and tail are loaded while this one is processed
    if (b + (int)gridDim.x < B) load_sample(b + gridDim.x);
    conv1_lds_at<PREC, NW>(s_crop, s_cropl, s_a1, s_a1l, w1f, w1fl, b1, c1_win, c1_slot);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kR2; ++i) {
      const int oy = wave + NW * i;
      f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        const bf16x8 af = col_frag(s_a1, c2_off[i][s]);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, w2f[0][s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, w2f[1][s], acc1, 0, 0, 0);
        if (PREC) {
          const bf16x8 afl = col_frag(s_a1l, c2_off[i][s]);
          acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, w2fl[0][s], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, w2fl[1][s], acc1, 0, 0, 0);
          acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl, w2f[0][s], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl, w2f[1][s], acc1, 0, 0, 0);
        }
      }
      const int64_t off = (int64_t)b * lda2 + oy * kA2 + 4 * lg;
      const float bb0[4] = {b2[0], b2[0], b2[0], b2[0]}, bb1[4] = {b2[1], b2[1], b2[1], b2[1]};
      *reinterpret_cast<uint2*>(a2 + off + lr * 256) = pack_relu4<false>(acc0, bb0);
      *reinterpret_cast<uint2*>(a2 + off + (16 + lr) * 256) = pack_relu4<false>(acc1, bb1);
      if (PREC) {
        *reinterpret_cast<uint2*>(a2lo + off + lr * 256) = pack_relu4<true>(acc0, bb0);
        *reinterpret_cast<uint2*>(a2lo + off + (16 + lr) * 256) = pack_relu4<true>(acc1, bb1);
      }
    }
    __syncthreads();
  }
}

}  // namespace pol
}  // namespace aslam

namespace aslam {
namespace pol {

// ------------------------------------------------------------ encoder backward
//
// One kernel for everything below the FC1 input gradient, per sample b:
//   conv1 is recomputed from the crop; with dz2 = dL/d(conv2 pre-activation)
//   (BF16 [b][co][pos], already masked by conv2's ReLU),
//   dW2[co][ci][tap] += sum_pos dz2[co][pos] a1[ci][pixel(pos, tap)]
//   da1[ci][y][x]     = sum_{co, tap} W2[co][ci][tap] dz2[co][pos(y, x, tap)]
//   dz1 = bf16(da1) * [a1 > 0]
//   dW1[co][tap]     += sum_px dz1[co][px] in[pixel(px, tap)]
//   db1 += sum dz1,  db2 += sum dz2.
// The workgroup (8 waves) keeps its gradient sums over all its samples and
// writes them once, as partials [gridDim.x][kConvPart], reduced afterwards in
// a fixed order.
//
// LDS layouts (BF16):
//   crop   space-to-depth, as in the forward kernel (conv1's operand);
//   inq    the crop again as five column-residue planes, inq[p][y+1][X] =
//          in[y][4X + p] for p < 4 and inq[4][y+1][X] = in[y][4X - 1] (row 0 and
//          inq[4][.][0] zero): the operand of the dW1 product, where a lane
//          needs the input under one tap at four pixels 2 apart, i.e. four
//          input columns 4 apart -- four consecutive elements of one plane;
//   a1x    [kx][ci][y+1][ox] = a1[ci][y][2 ox + kx - 1] (channels padded by 8
//          elements against bank conflicts): for a fixed tap, eight
//          consecutive output columns are eight consecutive elements, so the
//          im2col operand of the dW2 product is one 16-byte read; y = -1 and
//          x = -1 are zero;
//   dzT    [co][pos], rows padded to 264 elements: the dW2 operand is one
//          16-byte read (eight positions of one channel);
//   dz     [oy][ox][co] over 17 x 17 positions (row and column 16 zero),
//          positions padded to 40 elements so that eight lanes' 16-byte
//          accesses cover all banks: the operand of the input-gradient
//          product (eight channels of one position per read), transposed
//          from dzT once per sample.
// da1 is computed one sub-pixel phase (y % 2, x % 2) at a time: the input
// pixels of a phase form a 16 x 16 grid that receives taps ky = 1 (y even) or
// ky in {0, 2} (y odd), likewise kx, each from the output position
// (qy + (py + 1 - ky) / 2, qx + (px + 1 - kx) / 2).  K = 32 channels per tap.
// dz1 = bf16(da1) * [a1 > 0] never leaves registers: a lane holds channel
// lr at the pixels 4 lg + i of the phase rows qy = wave and wave + 8, and
// those eight values are exactly its A operand of one dW1 MFMA (K = the
// wave's 32 pixels of the phase), so dW1 is accumulated right after each
// phase's two da1 products.
constexpr int kConvPartW2 = kC2 * 144;          // [co][tap*16 + ci]
constexpr int kConvPartW1 = kC1 * 16;           // [co][tap], taps padded to 16
constexpr int kConvPart = kConvPartW2 + kConvPartW1 + kC1 + kC2;
constexpr int kA1xRow = 16, kA1xRows = 33;
constexpr int kA1xCi = kA1xRows * kA1xRow + 8;         // one channel's rows, padded against bank conflicts
constexpr int kA1xLds = 3 * kC1 * kA1xCi;               // BF16 elements
constexpr int kDzRow = 256 + 8;
constexpr int kDzLds = kC2 * kDzRow;
constexpr int kDzSide = 17, kDzPos = 40;
constexpr int kDzPLds = kDzSide * kDzSide * kDzPos;
constexpr int kInqRow = kCrop / 4, kInqPlane = (kCrop + 1) * kInqRow;   // 16 columns, 65 rows (row 0 zero)
constexpr int kInqLds = 5 * kInqPlane;
constexpr int kBwdThreads = 512;

struct PhaseTaps {
  int n;                 // taps of the phase (1, 2 or 4)
  int ky[4], kx[4], dy[4], dx[4];
};

__device__ __forceinline__ PhaseTaps phase_taps(int py, int px) {
  PhaseTaps t;
  const int nky = py ? 2 : 1, nkx = px ? 2 : 1;
  t.n = nky * nkx;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int iy = j / nkx, ix = j % nkx;
    const int ky = py ? 2 * iy : 1, kx = px ? 2 * ix : 1;
    t.ky[j] = ky; t.kx[j] = kx;
    t.dy[j] = (py + 1 - ky) / 2; t.dx[j] = (px + 1 - kx) / 2;
  }
  return t;
}

// B operand of the phase product for k-step (phase, j): lane supplies
// W2[co = 8 lg + e][ci = lr][ky_j][kx_j], e < 8.
__device__ __forceinline__ bf16x8 phase_weight_frag(const float* w2, int ky, int kx, int lr, int lg) {
  uint16_t v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = f2bf(w2[((8 * lg + e) * kC1 + lr) * 9 + ky * 3 + kx]);
  uint4 u;
  u.x = v[0] | ((uint32_t)v[1] << 16);
  u.y = v[2] | ((uint32_t)v[3] << 16);
  u.z = v[4] | ((uint32_t)v[5] << 16);
  u.w = v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}

// The backward's phase weight fragments, formed once per parameter update after the forward's
// kConvFrags: fragment kConvFrags + q of lane l at frag[64 (kConvFrags + q) + l], q enumerating the
// (phase, tap) pairs in phase order (9 in all).
constexpr int kConvPhaseFrags = 9;
static_assert(kConvLoFrag == kConvFrags + kConvPhaseFrags, "lo fragments follow the backward's");

__device__ __forceinline__ void conv_bwd_frag_elem(const float* prm, const Offsets& o, uint4* frag, int idx) {
  const int f = idx >> 6, lane = idx & 63, lr = lane & 15, lg = lane >> 4;
  int q = 0;
#pragma unroll
  for (int ph = 0; ph < 4; ++ph) {
    const PhaseTaps t = phase_taps(ph >> 1, ph & 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j < t.n) {
        if (q == f)
          frag[64 * (kConvFrags + q) + lane] =
              __builtin_bit_cast(uint4, phase_weight_frag(prm + o.c2w, t.ky[j], t.kx[j], lr, lg));
        ++q;
      }
    }
  }
}

__global__ __launch_bounds__(64 * kConvPhaseFrags) void k_conv_bwd_frags(const float* prm, Offsets o, uint4* frag) {
  conv_bwd_frag_elem(prm, o, frag, threadIdx.x);
}

// PREC: conv1 is recomputed with split operands (the crop's lo part staged beside it), so its ReLU
// mask is the one the split forward applied; the products of the backward stay BF16.
template <bool PREC>
__global__ __launch_bounds__(kBwdThreads) void k_conv_bwd(const float* __restrict__ prm, Offsets o,
                                                          const uint4* __restrict__ frag,
                                                          const int16_t* __restrict__ crop,
                                                          const int32_t* __restrict__ rows,
                                                          const uint16_t* __restrict__ dz2c, int B,
                                                          float* __restrict__ part) {
  __shared__ __align__(16) uint16_t s_crop[(PREC ? 2 : 1) * kCropLds];
  uint16_t* const s_cropl = s_crop + (PREC ? kCropLds : 0);
  __shared__ __align__(16) uint16_t s_a1x[kA1xLds];
  __shared__ __align__(16) uint16_t s_dz[kDzLds];
  __shared__ __align__(16) uint16_t s_dzp[kDzPLds];
  __shared__ __align__(16) uint16_t s_inq[kInqLds];
  __shared__ float s_red[8][kC1 * 16];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  {
    uint4* z = reinterpret_cast<uint4*>(s_crop);
    for (int i = threadIdx.x; i < (PREC ? 2 : 1) * kCropLds / 8; i += kBwdThreads) z[i] = make_uint4(0u, 0u, 0u, 0u);
    z = reinterpret_cast<uint4*>(s_a1x);
    for (int i = threadIdx.x; i < kA1xLds / 8; i += kBwdThreads) z[i] = make_uint4(0u, 0u, 0u, 0u);
    z = reinterpret_cast<uint4*>(s_dzp);
    for (int i = threadIdx.x; i < kDzPLds / 8; i += kBwdThreads) z[i] = make_uint4(0u, 0u, 0u, 0u);
    z = reinterpret_cast<uint4*>(s_inq);
    for (int i = threadIdx.x; i < kInqLds / 8; i += kBwdThreads) z[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  // registers that live for the whole workgroup
  // conv1's weights as the B operand: the same values as the forward's A fragment (W'[k][co] at co = lane % 16)
  const bf16x8 w1f = __builtin_bit_cast(bf16x8, frag[lane]);
  const bf16x8 w1fl = PREC ? __builtin_bit_cast(bf16x8, frag[64 * kConvLoFrag + lane]) : w1f;
  const float b1c = prm[o.c1b + lr];
  // phase weights: this wave's qy rows are {wave, wave + 8}; all four phases, 9 k-steps
  bf16x8 wph[kConvPhaseFrags];
#pragma unroll
  for (int q = 0; q < kConvPhaseFrags; ++q) wph[q] = __builtin_bit_cast(bf16x8, frag[64 * (kConvFrags + q) + lane]);
  // accumulators: every dW2 tile (nt = tap, mt = output-channel half) over this wave's k-step
  // (positions 32 wave .. 32 wave + 31) of every sample
  f32x4 gw2[9][2];
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) gw2[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 gw1 = {0.f, 0.f, 0.f, 0.f};
  float gb1 = 0.0f, gb2[2] = {0.f, 0.f};
  // the sample's crop and dz2 in registers; the next sample's are loaded while this one is processed
  CropRegs<kBwdThreads> cr;
  uint4 dzr[2];
  auto load_sample = [&](int bb) {
    load_crop<kBwdThreads>(crop + (rows ? (int64_t)rows[bb] : (int64_t)bb) * kCrop * kCrop, cr);
    const uint4* src = reinterpret_cast<const uint4*>(dz2c + (int64_t)bb * kFeat);
    dzr[0] = src[threadIdx.x];
    dzr[1] = src[threadIdx.x + kBwdThreads];
  };
  if (blockIdx.x < B) load_sample(blockIdx.x);
  __syncthreads();

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    // ---- stage the crop and dz2 ([co][pos]); db2 from the same values
    store_crop<kBwdThreads>(cr, s_crop);
    if (PREC) store_crop<kBwdThreads, true>(cr, s_cropl);
    {
      // the thread's eight cells: row y = v / 8, columns 8 (v % 8) + j, i.e. X = 2 (v % 8) + (j >= 4)
      // and residue j % 4
      static_assert(CropRegs<kBwdThreads>::kPer == 1, "one crop vector per thread");
      const int v = threadIdx.x, y = v >> 3, X0 = 2 * (v & 7);
      const int32_t w[4] = {cr.v[0].x, cr.v[0].y, cr.v[0].z, cr.v[0].w};
      uint16_t c[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        c[j] = f2bf((float)(int16_t)(w[j >> 1] >> ((j & 1) * 16)) * (1.0f / 256.0f));
      uint16_t* rowp = s_inq + (y + 1) * kInqRow + X0;
#pragma unroll
      for (int p = 0; p < 4; ++p)
        *reinterpret_cast<uint32_t*>(rowp + p * kInqPlane) = (uint32_t)c[p] | ((uint32_t)c[4 + p] << 16);
      rowp[4 * kInqPlane + 1] = c[3];
      if (X0 + 2 < kInqRow) rowp[4 * kInqPlane + 2] = c[7];
    }
    {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int v = threadIdx.x + r * kBwdThreads;   // vector of 8 positions of channel co
        const int co = v >> 5, p0 = (v & 31) * 8;
        const uint4 u = dzr[r];
        *reinterpret_cast<uint4*>(s_dz + co * kDzRow + p0) = u;
        float e[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        add_bf16x8(e, u);
        gb2[r] += ((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]));
      }
    }
    __syncthreads();
    if (b + (int)gridDim.x < B) load_sample(b + gridDim.x);
    // ---- conv1 recompute: C[px][co], lane gets pixels 16 t + 4 lg + i of channel lr; the wave's
    // eight tiles t = wave + 8 m are taken four at a time so that their operand reads overlap
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint4 u[4], ul[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = wave + 8 * (4 * h + i);
        u[i] = conv1_window(s_crop, t * 16 + lr, lg);
        if (PREC) ul[i] = conv1_window(s_cropl, t * 16 + lr, lg);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = wave + 8 * (4 * h + i);
        f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, u[i]), w1f,
                                                           f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        if (PREC) {
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ul[i]), w1f, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, u[i]), w1fl, acc, 0, 0, 0);
        }
        const int px0 = t * 16 + 4 * lg, y = px0 >> 5, x0 = px0 & 31;   // x0 = 0 mod 4
        uint16_t hv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) hv[e] = f2bf(fmaxf(acc[e] + b1c, 0.0f));
        uint16_t* row = s_a1x + lr * kA1xCi + (y + 1) * kA1xRow;    // kx plane 0
        const int plane = kC1 * kA1xCi;
        // even x -> kx = 1 at ox = x / 2; odd x -> kx = 0 at (x + 1) / 2 and kx = 2 at (x - 1) / 2
        *reinterpret_cast<uint32_t*>(row + plane + (x0 >> 1)) = (uint32_t)hv[0] | ((uint32_t)hv[2] << 16);
        *reinterpret_cast<uint32_t*>(row + 2 * plane + (x0 >> 1)) = (uint32_t)hv[1] | ((uint32_t)hv[3] << 16);
        row[(x0 >> 1) + 1] = hv[1];
        if ((x0 >> 1) + 2 < kA1xRow) row[(x0 >> 1) + 2] = hv[3];
      }
    }
    // dz2 [co][pos] -> [pos][co]: thread takes position v % 256 and channels 8 (v / 256) .. + 7
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int v = threadIdx.x + r * kBwdThreads;
      const int pos = v & 255, cg = v >> 8;
      uint16_t g[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) g[e] = s_dz[(8 * cg + e) * kDzRow + pos];
      *reinterpret_cast<uint4*>(s_dzp + ((pos >> 4) * kDzSide + (pos & 15)) * kDzPos + 8 * cg) = pack8(g);
    }
    __syncthreads();
    // ---- dW2: the wave's k-step (positions p0 = 32 wave + 8 lg .. + 7 of the lane) for all nine taps;
    // the dz operand is read once and serves every tap
    {
      const int p0 = 32 * wave + 8 * lg, oy = p0 >> 4, ox0 = p0 & 15;
      bf16x8 af[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        af[mt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(s_dz + (16 * mt + lr) * kDzRow + p0));
#pragma unroll
      for (int nt = 0; nt < 9; ++nt) {
        const int ky = nt / 3, kx = nt % 3;
        const int yy = 2 * oy + ky - 1;
        const bf16x8 bf = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(s_a1x + (kx * kC1 + lr) * kA1xCi + (yy + 1) * kA1xRow + ox0));
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          gw2[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bf, gw2[nt][mt], 0, 0, 0);
      }
    }
    // ---- da1 by phases -> dz1 (masked, BF16, in registers); db1; dW1 per phase
    {
      int q = 0;
#pragma unroll
      for (int ph = 0; ph < 4; ++ph) {
        const int py = ph >> 1, px = ph & 1;
        const PhaseTaps t = phase_taps(py, px);
        uint32_t dpk[4];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
          const int qy = wave + 8 * rr;
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j >= t.n) break;
            const int oy = qy + t.dy[j], ox = lr + t.dx[j];
            const bf16x8 af = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4*>(s_dzp + (oy * kDzSide + ox) * kDzPos + 8 * lg));
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, wph[q + j], acc, 0, 0, 0);
          }
          // lane: input pixels (2 qy + py, 2 (4 lg + i) + px), channel lr
          const int y = 2 * qy + py;
          const uint2 m = *reinterpret_cast<const uint2*>(
              s_a1x + ((1 + px) * kC1 + lr) * kA1xCi + (y + 1) * kA1xRow + 4 * lg);
          const uint32_t mw[2] = {m.x, m.y};
          uint16_t d[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint16_t a = (uint16_t)(mw[i >> 1] >> ((i & 1) * 16));
            d[i] = bf2f(a) > 0.0f ? f2bf(acc[i]) : (uint16_t)0;
            gb1 += bf2f(d[i]);
          }
          dpk[2 * rr] = (uint32_t)d[0] | ((uint32_t)d[1] << 16);
          dpk[2 * rr + 1] = (uint32_t)d[2] | ((uint32_t)d[3] << 16);
        }
        q += t.n;
        // dW1: C[co][tap] += sum_k dz1[co][k] in(k, tap) over the wave's 32 pixels of the phase, k = 8 lg
        // + 4 rr + i <-> pixel (2 (wave + 8 rr) + py, 2 (4 lg + i) + px).  B: lane (tap = lr, lg) reads
        // in[4 qy + 2 py + ky - 1][16 lg + 4 i + r], r = 2 px + kx - 1, i < 4: plane r (plane 4 for
        // r = -1), four consecutive elements from column 4 lg.
        uint2 bw[2] = {make_uint2(0u, 0u), make_uint2(0u, 0u)};
        if (lr < 9) {
          const int ky = lr / 3, kx = lr % 3, r = 2 * px + kx - 1;
          const uint16_t* pl = s_inq + (r < 0 ? 4 : r) * kInqPlane + 4 * lg;
#pragma unroll
          for (int rr = 0; rr < 2; ++rr) {
            const int row = 4 * (wave + 8 * rr) + 2 * py + ky - 1;
            bw[rr] = *reinterpret_cast<const uint2*>(pl + (row + 1) * kInqRow);
          }
        }
        const uint4 au = make_uint4(dpk[0], dpk[1], dpk[2], dpk[3]);
        const uint4 bu = make_uint4(bw[0].x, bw[0].y, bw[1].x, bw[1].y);
        gw1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, au), __builtin_bit_cast(bf16x8, bu),
                                                      gw1, 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ---- write the workgroup's partial sums (fixed order everywhere)
  float* out = part + (int64_t)blockIdx.x * kConvPart;
  float* st = reinterpret_cast<float*>(s_a1x);   // free after the sample loop
  // dW2 [co][nt*16 + ci]: lane value C[4 lg + i][lr] of tile (nt, mt) = (co = 16 mt + 4 lg + i, ci = lr), the
  // eight waves' k-step partials summed in wave order, three taps at a time through LDS
#pragma unroll
  for (int g = 0; g < 3; ++g) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) st[((wave * 3 + j) * 32 + 16 * mt + 4 * lg + i) * 16 + lr] = gw2[3 * g + j][mt][i];
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * 512; e += kBwdThreads) {
      const int j = e >> 9, r = e & 511;
      float sum = 0.0f;
      for (int w = 0; w < 8; ++w) sum += st[(w * 3 + j) * 512 + r];
      out[(r >> 4) * 144 + (3 * g + j) * 16 + (r & 15)] = sum;
    }
    __syncthreads();
  }
  // dW1 tile: C[4 lg + i][lr] = (co = 4 lg + i, tap = lr), summed over the waves in wave order
#pragma unroll
  for (int i = 0; i < 4; ++i) s_red[wave][(4 * lg + i) * 16 + lr] = gw1[i];
  __syncthreads();
  for (int e = threadIdx.x; e < kC1 * 16; e += kBwdThreads) {
    float sum = 0.0f;
    for (int w = 0; w < 8; ++w) sum += s_red[w][e];
    out[kConvPartW2 + e] = sum;
  }
  __syncthreads();
  {
    // db1: lane lr of each wave holds a channel-lr sum; db2: thread t holds channels t / 32 and t / 32 + 16
    st[threadIdx.x] = gb1;
    st[kBwdThreads + threadIdx.x] = gb2[0];
    st[2 * kBwdThreads + threadIdx.x] = gb2[1];
    __syncthreads();
    if (threadIdx.x < kC1) {
      float s = 0.0f;
      for (int t = 0; t < kBwdThreads; ++t)
        if ((t & 15) == threadIdx.x) s += st[t];
      out[kConvPartW2 + kConvPartW1 + threadIdx.x] = s;
    } else if (threadIdx.x >= 64 && threadIdx.x < 64 + kC2) {
      const int co = threadIdx.x - 64, r = co >> 4, t0 = (co & 15) * 32;
      float s = 0.0f;
      for (int t = t0; t < t0 + 32; ++t) s += st[(1 + r) * kBwdThreads + t];
      out[kConvPartW2 + kConvPartW1 + kC1 + co] = s;
    }
  }
}

}  // namespace pol
}  // namespace aslam
