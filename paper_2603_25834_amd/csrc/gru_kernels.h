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
// A step runs as a grid of 16-row tiles x kGruSlices workgroups: each workgroup (4 waves) stages its
// rows' FC1 output and entering state, and owns 64 of the 256 units (16 per wave) of every gate, so
// each lane ends up holding r, z and both halves of n's pre-activation for the same (row, unit) pairs
// and forms h' in registers; a workgroup reads a quarter of the weights, and a step of a few hundred
// rows spreads over many CUs.
#pragma once

#include "policy_kernels.h"

namespace aslam {
namespace pol {

constexpr int kGruRows = 16;
constexpr int kGruLdX = kHid + 8;    // BF16 rows in LDS, padded
constexpr int kGruLdF = kHid + 4;    // FP32 rows in LDS, padded
constexpr int kGruLdG = kGates + 8;  // BF16 gate-gradient rows in LDS, padded

constexpr int kGruSlices = 4;

struct GruFwdArgs {
  const float* prm;
  Offsets o;
  int rows;              // rows of this step
  int64_t s0;            // their first index in the minibatch-wide buffers (training; 0 in a rollout)
  const uint16_t* h1;    // the BF16 FC1 output, row s0 + i
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
};

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// One GRU step over rows s0 .. s0 + rows - 1; with TRAIN also the gate values the backward reads.
// h_out must not alias hp (other workgroups of the tile still read the entering state).
// The lane's weight fragments (unit u, gate g, k-step s) of a [768][256] BF16 matrix, all loads
// issued together: the step is latency-bound, so its 24 fragments cost one memory round trip.
__device__ __forceinline__ void gru_weight_frags(const uint16_t* w, int64_t u, int lg, gemm::bf16x8 (&f)[3][8]) {
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s)
      f[g][s] = __builtin_bit_cast(gemm::bf16x8,
                                   *reinterpret_cast<const uint4*>(w + (u + g * kHid) * kHid + 32 * s + 8 * lg));
}

template <bool TRAIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_gru_fwd(GruFwdArgs a) {
  __shared__ __align__(16) uint16_t s_x[kGruRows * kGruLdX];
  __shared__ __align__(16) uint16_t s_hb[kGruRows * kGruLdX];
  __shared__ __align__(16) float s_hp[kGruRows * kGruLdF];
  const int row0 = blockIdx.x * kGruRows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const Offsets& o = a.o;
  const int64_t u = 64 * blockIdx.y + 16 * wave + lr;
  gemm::bf16x8 wi[3][8], wh[3][8];
  gru_weight_frags(a.wih, u, lg, wi);
  gru_weight_frags(a.whh, u, lg, wh);
#pragma unroll
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
  // r and z accumulate the input and the state part in one accumulator (input first); n keeps them apart
  gemm::f32x4 ar = {0.f, 0.f, 0.f, 0.f}, az = ar, an = ar, ahn = ar;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const auto ax =
        __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_x + lr * kGruLdX + 32 * s + 8 * lg));
    ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, wi[0][s], ar, 0, 0, 0);
    az = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, wi[1][s], az, 0, 0, 0);
    an = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, wi[2][s], an, 0, 0, 0);
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const auto ah =
        __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_hb + lr * kGruLdX + 32 * s + 8 * lg));
    ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wh[0][s], ar, 0, 0, 0);
    az = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wh[1][s], az, 0, 0, 0);
    ahn = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wh[2][s], ahn, 0, 0, 0);
  }
  // gates and the new state: lane holds unit u of rows 4 lg + e
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
    if (TRAIN) {
      a.g_r[q] = rg;
      a.g_z[q] = zg;
      a.g_n[q] = ng;
      a.g_ghn[q] = ghn;
      a.hp_used[q] = hpv;
      a.hp_bf[q] = s_hb[r * kGruLdX + u];
    }
  }
}

// Rollout heads on the new state (no ReLU) and the Gaussian sample, one wave per row (lane l holds
// units 4 l .. 4 l + 3); also copies the state to h_out (which may alias the step's entering state,
// read completely by the step kernel before this one runs).
__global__ __launch_bounds__(256) void k_gru_heads(const float* prm, Offsets o, const float* h, int rows,
                                                   float* h_out, float* mu, float* value, ActDraws eps,
                                                   float* act, float* logp) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= rows) return;
  const float4 hh = *reinterpret_cast<const float4*>(h + row * kHid + lane * 4);
  if (h_out != h) *reinterpret_cast<float4*>(h_out + row * kHid + lane * 4) = hh;
  const float hv[4] = {hh.x, hh.y, hh.z, hh.w};
  float s0 = 0, s1 = 0, sv = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    s0 += prm[o.muw + lane * 4 + e] * hv[e];
    s1 += prm[o.muw + kHid + lane * 4 + e] * hv[e];
    sv += prm[o.vw + lane * 4 + e] * hv[e];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
    sv += __shfl_xor(sv, off, 64);
  }
  // the row's two normals on lanes 0 and 1 at once (a library draw is a long dependent chain)
  const float ed = lane < 2 ? eps(row, lane) : 0.0f;
  const float e1 = __shfl(ed, 1, 64);
  if (lane == 0) {
    const float m0 = s0 + prm[o.mub], m1 = s1 + prm[o.mub + 1];
    if (mu) {
      mu[2 * row] = m0;
      mu[2 * row + 1] = m1;
    }
    value[row] = sv + prm[o.vb];
    const float ls0 = prm[o.lstd], ls1 = prm[o.lstd + 1];
    const float e0 = ed;
    act[2 * row] = m0 + expf(ls0) * e0;
    act[2 * row + 1] = m1 + expf(ls1) * e1;
    logp[row] = -0.5f * (e0 * e0 + e1 * e1) - (ls0 + ls1) - 1.8378770664093453f;
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
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_gru_bwd_step(GruBwdArgs a) {
  __shared__ __align__(16) uint16_t s_g[kGruRows * kGruLdG];
  __shared__ __align__(16) float s_d[kGruRows * kGruLdF];
  const int row0 = blockIdx.x * kGruRows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  // W_hh^T fragments of this lane's output column n (k-steps of 32 over the 768 gate rows), loaded
  // first so that they arrive while the gate gradients are formed
  const int64_t n = 64 * blockIdx.y + 16 * wave + lr;
  gemm::bf16x8 wf[kGates / 32];
#pragma unroll
  for (int s = 0; s < kGates / 32; ++s)
    wf[s] = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(a.whht + n * kGates + 32 * s + 8 * lg));
  const int u = threadIdx.x;   // one unit per thread
  // the rows four at a time, so that their loads are in flight together
#pragma unroll
  for (int r0 = 0; r0 < kGruRows; r0 += 4) {
    float dh[4], rg[4], zg[4], ng[4], ghn[4], hp[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = row0 + r0 + e;
      dh[e] = rg[e] = zg[e] = ng[e] = ghn[e] = hp[e] = 0.0f;
      if (i < a.rows) {
        const int64_t q = (a.s0 + i) * kHid + u;
        dh[e] = a.dh_head[q] + (a.dh_next ? a.dh_next[(int64_t)i * kHid + u] : 0.0f);
        rg[e] = a.g_r[q]; zg[e] = a.g_z[q]; ng[e] = a.g_n[q]; ghn[e] = a.g_ghn[q]; hp[e] = a.hp_used[q];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = r0 + e, i = row0 + r;
      float dr = 0.f, dz = 0.f, dn = 0.f, dnr = 0.f, dd = 0.f;
      if (i < a.rows) {
        dd = dh[e] * zg[e];
        const float dn_pre = (dh[e] * (1.0f - zg[e])) * (1.0f - ng[e] * ng[e]);
        dz = (dh[e] * (hp[e] - ng[e])) * (zg[e] * (1.0f - zg[e]));
        dr = (dn_pre * ghn[e]) * (rg[e] * (1.0f - rg[e]));
        dn = dn_pre;
        dnr = dn_pre * rg[e];
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
  }
  __syncthreads();
  // dgh [16 x 768] x W_hh [768 x 256]: this workgroup's columns 64 y .. 64 y + 63, 16 per wave
  gemm::f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < kGates / 32; ++s) {
    const gemm::bf16x8 ag =
        __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_g + lr * kGruLdG + 32 * s + 8 * lg));
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ag, wf[s], acc, 0, 0, 0);
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
