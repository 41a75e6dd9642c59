// gru_kernels.h -- the recurrent actor-critic's GRU layer on gfx950 (library-internal).
//
// A single-layer GRU of 256 units (arXiv 2603.25834, Sec. III-F, "Recurrent Layer") sits between
// FC1 and the heads.  Gate rows of the weights are ordered reset / update / new:
//   r = sigmoid(W_ir x + b_ir + W_hr h + b_hr),  z = sigmoid(W_iz x + b_iz + W_hz h + b_hz),
//   n = tanh(W_in x + b_in + r (W_hn h + b_hn)),  h' = (1 - z) n + z h,
// with the state zeroed before a step that starts an episode.  The products run on MFMA with BF16
// operands (FC1 output, weights, the state fed to W_hh) and FP32 accumulation; the gate math and
// the state itself are FP32.
//
// One workgroup (4 waves) owns a tile of 16 rows.  Wave w owns units 64 w .. 64 w + 63 of every gate,
// so each lane ends up holding r, z and both halves of n's pre-activation for the same (row, unit)
// pairs and forms h' in registers.
#pragma once

#include "policy_kernels.h"

namespace aslam {
namespace pol {

constexpr int kGruRows = 16;
constexpr int kGruLdX = kHid + 8;    // BF16 rows in LDS, padded
constexpr int kGruLdF = kHid + 4;    // FP32 rows in LDS, padded
constexpr int kGruLdG = kGates + 8;  // BF16 gate-gradient rows in LDS, padded

struct GruFwdArgs {
  const float* prm;
  Offsets o;
  int rows;              // rows of this step
  int64_t s0;            // their first index in the minibatch-wide buffers (training; 0 in a rollout)
  const float* part;     // FC1 split-K partial sums (S > 0): slice z, row i at (z * part_rows + s0 + i) * 256
  int S;
  int64_t part_rows;
  const uint16_t* h1;    // else the BF16 FC1 output, row s0 + i
  const uint16_t* wih;   // BF16 [768][256]
  const uint16_t* whh;   // BF16 [768][256]
  const float* hp;       // entering state: row hp_map[i] (or i)
  const int32_t* hp_map;
  const uint8_t* first;  // episode start flag of row first_map[i] (or i); NULL = none
  const int32_t* first_map;
  float* h_out;          // new state, row s0 + i
  // training: what the backward reads, rows s0 + i
  float *g_r, *g_z, *g_n, *g_ghn, *hp_used;
  uint16_t* hp_bf;
  // rollout: heads and the Gaussian sample, row i
  float* mu;
  float* value;
  const float* eps;
  float* act;
  float* logp;
};

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

template <bool ROLLOUT>
__global__ __launch_bounds__(256) void k_gru_fwd(GruFwdArgs a) {
  __shared__ __align__(16) uint16_t s_x[kGruRows * kGruLdX];
  __shared__ __align__(16) uint16_t s_hb[kGruRows * kGruLdX];
  __shared__ __align__(16) float s_hp[kGruRows * kGruLdF];
  __shared__ __align__(16) float s_h[kGruRows * kGruLdF];
  const int row0 = blockIdx.x * kGruRows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const Offsets& o = a.o;
  const float* b1 = a.prm + o.f1b;
  // FC1 output (split-K sum + bias + ReLU -> BF16, or the stored rows) and the entering state
  for (int g = threadIdx.x; g < kGruRows * (kHid / 8); g += 256) {
    const int r = g / (kHid / 8), n0 = (g % (kHid / 8)) * 8;
    const int i = row0 + r;
    uint4 vx = make_uint4(0u, 0u, 0u, 0u);
    float hv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < a.rows) {
      const int64_t s = a.s0 + i;
      if (a.S > 0) {
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        sum_slices8(a.part + s * kHid + n0, a.S, a.part_rows * kHid, acc);
        uint16_t h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) h[j] = f2bf(fmaxf(acc[j] + b1[n0 + j], 0.0f));
        vx = pack8(h);
      } else {
        vx = *reinterpret_cast<const uint4*>(a.h1 + s * kHid + n0);
      }
      const bool reset = a.first && a.first[a.first_map ? a.first_map[i] : i];
      if (!reset) {
        const float* q = a.hp + (int64_t)(a.hp_map ? a.hp_map[i] : i) * kHid + n0;
        const float4 lo = *reinterpret_cast<const float4*>(q), hi = *reinterpret_cast<const float4*>(q + 4);
        hv[0] = lo.x; hv[1] = lo.y; hv[2] = lo.z; hv[3] = lo.w;
        hv[4] = hi.x; hv[5] = hi.y; hv[6] = hi.z; hv[7] = hi.w;
      }
    }
    *reinterpret_cast<uint4*>(s_x + r * kGruLdX + n0) = vx;
    uint16_t hb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      s_hp[r * kGruLdF + n0 + j] = hv[j];
      hb[j] = f2bf(hv[j]);
    }
    *reinterpret_cast<uint4*>(s_hb + r * kGruLdX + n0) = pack8(hb);
  }
  __syncthreads();
  // gate products: r and z accumulate the input and the state part in one accumulator; n keeps them apart
  gemm::f32x4 ar[4], az[4], an[4], ahn[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ar[j] = az[j] = an[j] = ahn[j] = gemm::f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const int ub = 64 * wave + lr;
#pragma unroll 2
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    const int kk = k0 + 8 * lg;
    const gemm::bf16x8 ax = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_x + lr * kGruLdX + kk));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t u = ub + 16 * j;
      const auto wr = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.wih + u * kHid + kk));
      const auto wz = __builtin_bit_cast(gemm::bf16x8,
                                         *reinterpret_cast<const uint4*>(a.wih + (u + kHid) * kHid + kk));
      const auto wn = __builtin_bit_cast(gemm::bf16x8,
                                         *reinterpret_cast<const uint4*>(a.wih + (u + 2 * kHid) * kHid + kk));
      ar[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, wr, ar[j], 0, 0, 0);
      az[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, wz, az[j], 0, 0, 0);
      an[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, wn, an[j], 0, 0, 0);
    }
  }
#pragma unroll 2
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    const int kk = k0 + 8 * lg;
    const gemm::bf16x8 ah = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_hb + lr * kGruLdX + kk));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t u = ub + 16 * j;
      const auto wr = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.whh + u * kHid + kk));
      const auto wz = __builtin_bit_cast(gemm::bf16x8,
                                         *reinterpret_cast<const uint4*>(a.whh + (u + kHid) * kHid + kk));
      const auto wn = __builtin_bit_cast(gemm::bf16x8,
                                         *reinterpret_cast<const uint4*>(a.whh + (u + 2 * kHid) * kHid + kk));
      ar[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wr, ar[j], 0, 0, 0);
      az[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wz, az[j], 0, 0, 0);
      ahn[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wn, ahn[j], 0, 0, 0);
    }
  }
  // gates and the new state: lane holds units ub + 16 j of rows 4 lg + e
  const float* bi = a.prm + o.gbi;
  const float* bh = a.prm + o.gbh;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int u = ub + 16 * j;
    const float bir = bi[u], biz = bi[u + kHid], bin = bi[u + 2 * kHid];
    const float bhr = bh[u], bhz = bh[u + kHid], bhn = bh[u + 2 * kHid];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 4 * lg + e;
      const float rg = sigmoidf_((ar[j][e] + bir) + bhr);
      const float zg = sigmoidf_((az[j][e] + biz) + bhz);
      const float ghn = ahn[j][e] + bhn;
      const float ng = tanhf((an[j][e] + bin) + rg * ghn);
      const float hpv = s_hp[r * kGruLdF + u];
      const float h = (1.0f - zg) * ng + zg * hpv;
      s_h[r * kGruLdF + u] = h;
      const int i = row0 + r;
      if (i < a.rows) {
        const int64_t q = (a.s0 + i) * kHid + u;
        a.h_out[q] = h;
        if (!ROLLOUT) {
          a.g_r[q] = rg;
          a.g_z[q] = zg;
          a.g_n[q] = ng;
          a.g_ghn[q] = ghn;
          a.hp_used[q] = hpv;
          a.hp_bf[q] = s_hb[r * kGruLdX + u];
        }
      }
    }
  }
  if (!ROLLOUT) return;
  __syncthreads();
  // heads on the new state (no ReLU): wave w takes rows 4 w .. 4 w + 3, lane l columns 4 l .. 4 l + 3
  const float* prm = a.prm;
  float wmu0[4], wmu1[4], wv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    wmu0[e] = prm[o.muw + lane * 4 + e];
    wmu1[e] = prm[o.muw + kHid + lane * 4 + e];
    wv[e] = prm[o.vw + lane * 4 + e];
  }
  const float bmu0 = prm[o.mub], bmu1 = prm[o.mub + 1], bv = prm[o.vb];
  for (int rr = 0; rr < kGruRows / 4; ++rr) {
    const int r = 4 * wave + rr;
    const int64_t row = row0 + r;
    if (row >= a.rows) break;
    const float4 hh = *reinterpret_cast<const float4*>(s_h + r * kGruLdF + lane * 4);
    const float hv[4] = {hh.x, hh.y, hh.z, hh.w};
    float s0 = 0, s1 = 0, sv = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      s0 += wmu0[e] * hv[e];
      s1 += wmu1[e] * hv[e];
      sv += wv[e] * hv[e];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
      sv += __shfl_xor(sv, off, 64);
    }
    if (lane == 0) {
      const float m0 = s0 + bmu0, m1 = s1 + bmu1;
      if (a.mu) {
        a.mu[2 * row] = m0;
        a.mu[2 * row + 1] = m1;
      }
      a.value[row] = sv + bv;
      const float ls0 = prm[o.lstd], ls1 = prm[o.lstd + 1];
      const float e0 = a.eps[2 * row], e1 = a.eps[2 * row + 1];
      a.act[2 * row] = m0 + expf(ls0) * e0;
      a.act[2 * row + 1] = m1 + expf(ls1) * e1;
      a.logp[row] = -0.5f * (e0 * e0 + e1 * e1) - (ls0 + ls1) - 1.8378770664093453f;
    }
  }
}

// Training forward step: as k_gru_fwd<false>, with the 256 units split over gridDim.y = 4 workgroups
// per row tile (64 units each, 16 per wave), so a workgroup reads a quarter of the weights and a step
// of a few hundred rows still spreads over many CUs.  Values and accumulation order per unit are
// those of k_gru_fwd.
constexpr int kGruSlices = 4;

__global__ __launch_bounds__(256) void k_gru_fwd_train(GruFwdArgs a) {
  __shared__ __align__(16) uint16_t s_x[kGruRows * kGruLdX];
  __shared__ __align__(16) uint16_t s_hb[kGruRows * kGruLdX];
  __shared__ __align__(16) float s_hp[kGruRows * kGruLdF];
  const int row0 = blockIdx.x * kGruRows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const Offsets& o = a.o;
  for (int g = threadIdx.x; g < kGruRows * (kHid / 8); g += 256) {
    const int r = g / (kHid / 8), n0 = (g % (kHid / 8)) * 8;
    const int i = row0 + r;
    uint4 vx = make_uint4(0u, 0u, 0u, 0u);
    float hv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < a.rows) {
      vx = *reinterpret_cast<const uint4*>(a.h1 + (a.s0 + i) * kHid + n0);
      const bool reset = a.first && a.first[a.first_map ? a.first_map[i] : i];
      if (!reset) {
        const float* q = a.hp + (int64_t)(a.hp_map ? a.hp_map[i] : i) * kHid + n0;
        const float4 lo = *reinterpret_cast<const float4*>(q), hi = *reinterpret_cast<const float4*>(q + 4);
        hv[0] = lo.x; hv[1] = lo.y; hv[2] = lo.z; hv[3] = lo.w;
        hv[4] = hi.x; hv[5] = hi.y; hv[6] = hi.z; hv[7] = hi.w;
      }
    }
    *reinterpret_cast<uint4*>(s_x + r * kGruLdX + n0) = vx;
    uint16_t hb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      s_hp[r * kGruLdF + n0 + j] = hv[j];
      hb[j] = f2bf(hv[j]);
    }
    *reinterpret_cast<uint4*>(s_hb + r * kGruLdX + n0) = pack8(hb);
  }
  __syncthreads();
  const int64_t u = 64 * blockIdx.y + 16 * wave + lr;
  gemm::f32x4 ar = {0.f, 0.f, 0.f, 0.f}, az = ar, an = ar, ahn = ar;
#pragma unroll
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    const int kk = k0 + 8 * lg;
    const auto ax = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_x + lr * kGruLdX + kk));
    ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        ax, __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.wih + u * kHid + kk)), ar, 0, 0, 0);
    az = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        ax, __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.wih + (u + kHid) * kHid + kk)), az,
        0, 0, 0);
    an = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        ax, __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.wih + (u + 2 * kHid) * kHid + kk)),
        an, 0, 0, 0);
  }
#pragma unroll
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    const int kk = k0 + 8 * lg;
    const auto ah = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_hb + lr * kGruLdX + kk));
    ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        ah, __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.whh + u * kHid + kk)), ar, 0, 0, 0);
    az = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        ah, __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.whh + (u + kHid) * kHid + kk)), az,
        0, 0, 0);
    ahn = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        ah, __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.whh + (u + 2 * kHid) * kHid + kk)),
        ahn, 0, 0, 0);
  }
  const float* bi = a.prm + o.gbi;
  const float* bh = a.prm + o.gbh;
  const float bir = bi[u], biz = bi[u + kHid], bin = bi[u + 2 * kHid];
  const float bhr = bh[u], bhz = bh[u + kHid], bhn = bh[u + 2 * kHid];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = 4 * lg + e, i = row0 + r;
    if (i >= a.rows) continue;
    const float rg = sigmoidf_((ar[e] + bir) + bhr);
    const float zg = sigmoidf_((az[e] + biz) + bhz);
    const float ghn = ahn[e] + bhn;
    const float ng = tanhf((an[e] + bin) + rg * ghn);
    const float hpv = s_hp[r * kGruLdF + u];
    const int64_t q = (a.s0 + i) * kHid + u;
    a.h_out[q] = (1.0f - zg) * ng + zg * hpv;
    a.g_r[q] = rg;
    a.g_z[q] = zg;
    a.g_n[q] = ng;
    a.g_ghn[q] = ghn;
    a.hp_used[q] = hpv;
    a.hp_bf[q] = s_hb[r * kGruLdX + u];
  }
}

// One step of backpropagation through time, rows s0 + i (i < rows) of step t:
//   dh = dh_head + dh_next (the gradient reaching h_t from the heads and from step t + 1),
//   gate pre-activation gradients dgi = [dr', dz', dn'], dgh = [dr', dz', dn' r] (BF16, the operands
//   of the weight-gradient and input-gradient GEMMs), and the gradient reaching h_{t-1}:
//   dh_prev = z dh + dgh W_hh, zero where step t starts an episode.
struct GruBwdArgs {
  int rows;
  int64_t s0;
  const float* dh_head;            // [B][256], row s0 + i
  const float* dh_next;            // [rows][256] or NULL
  const float *g_r, *g_z, *g_n, *g_ghn, *hp_used;   // row s0 + i
  const uint8_t* first;            // flag of row first_map[i]; NULL = none
  const int32_t* first_map;
  const uint16_t* whht;            // W_hh transposed: BF16 [256][768]
  uint16_t* dgi;                   // [B][768], row s0 + i
  uint16_t* dgh;
  float* dh_prev;                  // [rows][256]
};

// gridDim.y = kGruSlices workgroups share a row tile: each forms the tile's gate gradients (slice 0
// alone writes them out) and the state gradient for its 64 columns.
__global__ __launch_bounds__(256) void k_gru_bwd_step(GruBwdArgs a) {
  __shared__ __align__(16) uint16_t s_g[kGruRows * kGruLdG];
  __shared__ __align__(16) float s_d[kGruRows * kGruLdF];
  const int row0 = blockIdx.x * kGruRows;
  const int u = threadIdx.x;   // one unit per thread
  for (int r = 0; r < kGruRows; ++r) {
    const int i = row0 + r;
    float dr = 0.f, dz = 0.f, dn = 0.f, dnr = 0.f, dd = 0.f;
    if (i < a.rows) {
      const int64_t q = (a.s0 + i) * kHid + u;
      const float dh = a.dh_head[q] + (a.dh_next ? a.dh_next[(int64_t)i * kHid + u] : 0.0f);
      const float rg = a.g_r[q], zg = a.g_z[q], ng = a.g_n[q], ghn = a.g_ghn[q], hp = a.hp_used[q];
      dd = dh * zg;
      const float dn_pre = (dh * (1.0f - zg)) * (1.0f - ng * ng);
      dz = (dh * (hp - ng)) * (zg * (1.0f - zg));
      dr = (dn_pre * ghn) * (rg * (1.0f - rg));
      dn = dn_pre;
      dnr = dn_pre * rg;
      if (blockIdx.y == 0) {
        const int64_t g = (a.s0 + i) * kGates + u;
        a.dgi[g] = f2bf(dr);
        a.dgi[g + kHid] = f2bf(dz);
        a.dgi[g + 2 * kHid] = f2bf(dn);
        a.dgh[g] = f2bf(dr);
        a.dgh[g + kHid] = f2bf(dz);
        a.dgh[g + 2 * kHid] = f2bf(dnr);
      }
    }
    s_g[r * kGruLdG + u] = f2bf(dr);
    s_g[r * kGruLdG + u + kHid] = f2bf(dz);
    s_g[r * kGruLdG + u + 2 * kHid] = f2bf(dnr);
    s_d[r * kGruLdF + u] = dd;
  }
  __syncthreads();
  // dgh [16 x 768] x W_hh [768 x 256]: this workgroup's columns 64 y .. 64 y + 63, 16 per wave
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int64_t n = 64 * blockIdx.y + 16 * wave + lr;
  gemm::f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
  for (int k0 = 0; k0 < kGates; k0 += 32) {
    const int kk = k0 + 8 * lg;
    const gemm::bf16x8 ag = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_g + lr * kGruLdG + kk));
    const auto wb = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.whht + n * kGates + kk));
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ag, wb, acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = 4 * lg + e, i = row0 + r;
    if (i >= a.rows) continue;
    const bool reset = a.first && a.first[a.first_map ? a.first_map[i] : i];
    a.dh_prev[(int64_t)i * kHid + n] = reset ? 0.0f : s_d[r * kGruLdF + n] + acc[e];
  }
}

// Column sums of a BF16 [rows][ch] tensor into per-block partials [gridDim.x][ch] (fixed order:
// each block sums a contiguous row range in order; thread c takes columns c, c + 256, ...).
__global__ __launch_bounds__(256) void k_colsum_bf16(const uint16_t* src, int64_t rows, int ch, float* part) {
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t beg = (int64_t)blockIdx.x * per, end = min(rows, beg + per);
  for (int c = threadIdx.x; c < ch; c += 256) {
    float t = 0.0f;
    for (int64_t r = beg; r < end; ++r) t += bf2f(src[r * ch + c]);
    part[(int64_t)blockIdx.x * ch + c] = t;
  }
}

// Minibatch rows of a sequence minibatch: sample s = t * nb + i is rollout row t * N + robots[i].
__global__ void k_seq_rows(const int32_t* robots, int nb, int T, int N, int32_t* rows) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= T * nb) return;
  const int t = s / nb, i = s - t * nb;
  rows[s] = t * N + robots[i];
}

}  // namespace pol
}  // namespace aslam
