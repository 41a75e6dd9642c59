// policy_kernels.h -- PPO actor-critic forward / backward, GAE and Adam on gfx950.
//
// Method: arXiv 2603.25834, Sec. III-F.  The policy is trained with PPO's
// clipped surrogate (Eqs. 18-20) on advantages from Generalized Advantage
// Estimation.  The network is the workload's actor-critic: conv 1->16 and
// 16->32 (3x3, stride 2, padding 1, ReLU) on a 64x64 belief crop, the 8192
// features concatenated with the normalised scan (R) and the 12-float state,
// FC 256 and FC 256 (ReLU), a Gaussian mean head (2), a value head (1) and a
// state-independent log standard deviation (2).
//
// Precision: GEMM operands are rounded to BF16 (round to nearest even) and
// accumulated in FP32 on MFMA; activations between layers are stored as BF16;
// biases, heads, the loss and every reduction are FP32.  Parameters and
// gradients are FP32 in the flat layout documented in include/aslam.h.
//
// Backward recomputes the forward activations of the minibatch (only the
// inputs are kept across the rollout); weight gradients are formed by split-K
// GEMMs whose partial sums are reduced in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "aslam.h"
#include "gemm_bf16.h"
#include "rng.h"

namespace aslam {
namespace pol {

using gemm::bf2f;
using gemm::f2bf;

constexpr int kCrop = 64, kA1 = 32, kA2 = 16, kC1 = 16, kC2 = 32, kHid = 256, kFeat = kC2 * kA2 * kA2;

constexpr int kGates = 3 * kHid;   // GRU gate rows: reset, update, new

struct Offsets {
  int64_t c1w, c1b, c2w, c2b, f1w, f1b, f2w, f2b, muw, mub, vw, vb, lstd, total;
  int64_t gih, ghh, gbi, gbh;   // recurrent layout: GRU weights [768][256] and biases [768]; -1 otherwise
  int32_t k1;  // FC1 input width = 8192 + R + 12
  int32_t recurrent;
};

// Flat parameter layout: the feed-forward network, or with `recurrent` the GRU in place of FC2.
inline Offsets offsets(int32_t n_scan, bool recurrent = false) {
  Offsets o;
  o.k1 = kFeat + n_scan + 12;
  o.recurrent = recurrent ? 1 : 0;
  int64_t p = 0;
  o.c1w = p; p += kC1 * 9;
  o.c1b = p; p += kC1;
  o.c2w = p; p += kC2 * kC1 * 9;
  o.c2b = p; p += kC2;
  o.f1w = p; p += (int64_t)kHid * o.k1;
  o.f1b = p; p += kHid;
  if (recurrent) {
    o.f2w = o.f2b = -1;
    o.gih = p; p += (int64_t)kGates * kHid;
    o.ghh = p; p += (int64_t)kGates * kHid;
    o.gbi = p; p += kGates;
    o.gbh = p; p += kGates;
  } else {
    o.gih = o.ghh = o.gbi = o.gbh = -1;
    o.f2w = p; p += kHid * kHid;
    o.f2b = p; p += kHid;
  }
  o.muw = p; p += 2 * kHid;
  o.mub = p; p += 2;
  o.vw = p; p += kHid;
  o.vb = p; p += 1;
  o.lstd = p; p += 2;
  o.total = p;
  return o;
}

// ------------------------------------------------------------------ loaders

__device__ __forceinline__ uint4 pack8(const uint16_t v[8]) {
  return make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16), v[4] | ((uint32_t)v[5] << 16),
                    v[6] | ((uint32_t)v[7] << 16));
}

// BF16 matrix, element (i, k) at p[i*ld + k]; contiguous along k.
struct LdBF16K {
  static constexpr bool kMajor = true;
  const uint16_t* p; int64_t ld; int rows, cols;
  __device__ uint4 fetch(int i, int k) const {
    if (i >= rows || k >= cols) return make_uint4(0u, 0u, 0u, 0u);
    const uint16_t* q = p + (int64_t)i * ld + k;
    if (k + 8 <= cols && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) return *reinterpret_cast<const uint4*>(q);
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (k + j < cols) ? q[j] : (uint16_t)0;
    return pack8(v);
  }
};

// BF16 matrix, element (i, k) at p[k*ld + i]; contiguous along i.
struct LdBF16I {
  static constexpr bool kMajor = false;
  const uint16_t* p; int64_t ld; int rows, cols;
  __device__ uint4 fetch(int i, int k) const {
    if (i >= rows || k >= cols) return make_uint4(0u, 0u, 0u, 0u);
    const uint16_t* q = p + (int64_t)k * ld + i;
    if (i + 8 <= rows && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) return *reinterpret_cast<const uint4*>(q);
    uint16_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (i + j < rows) ? q[j] : (uint16_t)0;
    return pack8(v);
  }
};

// ---------------------------------------------------------------- epilogues
// store8(m, n0, v, nvalid): row m, columns n0 .. n0 + nvalid - 1 (n0 multiple of 8).
// kSliced: the epilogue stores a split-K slice and takes its index (store8z(z, ...)).

struct EpiBiasReluBF16 {
  uint16_t* out; const float* bias; int64_t ld;
  static constexpr bool kPrefetch = false, kSliced = false;
  __device__ void store8(int m, int n0, const float* v, int nvalid) const {
    uint16_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = j < nvalid ? f2bf(fmaxf(v[j] + bias[n0 + j], 0.0f)) : (uint16_t)0;
    uint16_t* q = out + (int64_t)m * ld + n0;
    if (nvalid == 8 && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) {
      *reinterpret_cast<uint4*>(q) = pack8(h);
    } else {
      for (int j = 0; j < nvalid; ++j) q[j] = h[j];
    }
  }
};

struct EpiBiasF32 {
  float* out; const float* bias; int64_t ld;
  static constexpr bool kPrefetch = false, kSliced = false;
  __device__ void store8(int m, int n0, const float* v, int nvalid) const {
    float* q = out + (int64_t)m * ld + n0;
    if (nvalid == 8 && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) {
      *reinterpret_cast<float4*>(q) = make_float4(v[0] + bias[n0], v[1] + bias[n0 + 1], v[2] + bias[n0 + 2],
                                                  v[3] + bias[n0 + 3]);
      *reinterpret_cast<float4*>(q + 4) = make_float4(v[4] + bias[n0 + 4], v[5] + bias[n0 + 5],
                                                      v[6] + bias[n0 + 6], v[7] + bias[n0 + 7]);
    } else {
      for (int j = 0; j < nvalid; ++j) q[j] = v[j] + bias[n0 + j];
    }
  }
};

// Split-K partial sums: slice z of a [splits][M][N] FP32 buffer.
struct EpiPartial {
  float* part; int64_t ld; int64_t slice;
  static constexpr bool kPrefetch = false, kSliced = true;
  __device__ void store8z(int z, int m, int n0, const float* v, int nvalid) const {
    float* q = part + (int64_t)z * slice + (int64_t)m * ld + n0;
    if (nvalid == 8 && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) {
      *reinterpret_cast<float4*>(q) = make_float4(v[0], v[1], v[2], v[3]);
      *reinterpret_cast<float4*>(q + 4) = make_float4(v[4], v[5], v[6], v[7]);
    } else {
      for (int j = 0; j < nvalid; ++j) q[j] = v[j];
    }
  }
};

// Gradient through a ReLU whose output (BF16) is `act`: out = bf16(act > 0 ? v : 0).
struct EpiReluGradBF16 {
  uint16_t* out; const uint16_t* act; int64_t ld, ld_act;
  // the engine loads the mask at kernel start (fetch) and hands it to store8_pre
  static constexpr bool kPrefetch = true, kSliced = false;
  __device__ bool vec_ok(int m, int n0, int nvalid) const {
    return nvalid == 8 && ((((int64_t)m * ld + n0) & 7) == 0) && ((((int64_t)m * ld_act + n0) & 7) == 0);
  }
  __device__ uint4 fetch(int m, int n0, int nvalid) const {
    return vec_ok(m, n0, nvalid) ? *reinterpret_cast<const uint4*>(act + (int64_t)m * ld_act + n0)
                                 : make_uint4(0u, 0u, 0u, 0u);
  }
  __device__ void store8_pre(int m, int n0, const float* v, int nvalid, const uint4& a) const {
    if (vec_ok(m, n0, nvalid)) {
      uint16_t h[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) h[j] = bf2f(gemm::lane16(a, j)) > 0.0f ? f2bf(v[j]) : (uint16_t)0;
      *reinterpret_cast<uint4*>(out + (int64_t)m * ld + n0) = pack8(h);
    } else {
      store8(m, n0, v, nvalid);
    }
  }
  __device__ void store8(int m, int n0, const float* v, int nvalid) const {
    const int64_t o = (int64_t)m * ld + n0, oa = (int64_t)m * ld_act + n0;
    if (nvalid == 8 && ((o & 7) == 0) && ((oa & 7) == 0)) {
      const uint4 a = *reinterpret_cast<const uint4*>(act + oa);
      uint16_t h[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) h[j] = bf2f(gemm::lane16(a, j)) > 0.0f ? f2bf(v[j]) : (uint16_t)0;
      *reinterpret_cast<uint4*>(out + o) = pack8(h);
    } else {
      for (int j = 0; j < nvalid; ++j) out[o + j] = bf2f(act[oa + j]) > 0.0f ? f2bf(v[j]) : (uint16_t)0;
    }
  }
};

// ---------------------------------------------------------------- kernels

struct LossCoef {
  float eps, c_v, c_e, inv_b;
};

// Heads (FP32): one wave per row.  h2 = relu(z2); mu = Wmu h2 + bmu; V = wv h2 + bv.
// With `grad`: the PPO loss of the row and its gradient, written as
// dz2 = (dmu Wmu + dV wv) * [z2 > 0] (BF16), plus per-workgroup partial sums of
// the head parameter gradients, dlog_std and the loss terms, in `part`:
// [Wmu 512 | bmu 2 | wv 256 | bv 1 | dlogstd 2 | db2 256 | loss 4] floats.
constexpr int kHeadPart = 512 + 2 + 256 + 1 + 2 + 256 + 4;
constexpr int kHeadRows = 64;   // rows per workgroup (16 per wave)

// RECUR: the heads read the GRU state directly (no ReLU) and, with GRAD, write its gradient dh (FP32)
// to dh_out instead of the masked BF16 dz2.
template <bool GRAD, bool RECUR = false>
__global__ __launch_bounds__(256) void k_heads(const float* prm, Offsets o, const float* z2, int B, float* mu_out,
                                               float* v_out, const float* act, const float* old_logp,
                                               const float* adv, const float* ret, const int32_t* rows, LossCoef lc,
                                               uint16_t* dz2, float* part, float* dh_out = nullptr) {
  __shared__ float acc[4][kHeadPart];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float wmu0[4], wmu1[4], wv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    wmu0[e] = prm[o.muw + lane * 4 + e];
    wmu1[e] = prm[o.muw + kHid + lane * 4 + e];
    wv[e] = prm[o.vw + lane * 4 + e];
  }
  const float bmu0 = prm[o.mub], bmu1 = prm[o.mub + 1], bv = prm[o.vb];
  const float ls0 = prm[o.lstd], ls1 = prm[o.lstd + 1];
  float gw0[4] = {0, 0, 0, 0}, gw1[4] = {0, 0, 0, 0}, gwv[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0};
  float gbm0 = 0, gbm1 = 0, gbv = 0, gls0 = 0, gls1 = 0, lclip = 0, lval = 0;
  const float log2pi = 1.8378770664093453f;
  // the wave's 16 rows: lane j < 16 fetches row j's rollout data up front (handed out by shuffles), and
  // all 16 rows of z2 are loaded up front (one memory round trip for the wave)
  constexpr int kWaveRows = kHeadRows / 4;
  const int wrow0 = blockIdx.x * kHeadRows + wave * kWaveRows;
  float q_a0 = 0.f, q_a1 = 0.f, q_olp = 0.f, q_adv = 0.f, q_ret = 0.f;
  if (GRAD && lane < kWaveRows && wrow0 + lane < B) {
    const int64_t sr = rows ? (int64_t)rows[wrow0 + lane] : (int64_t)(wrow0 + lane);
    q_a0 = act[2 * sr];
    q_a1 = act[2 * sr + 1];
    q_olp = old_logp[sr];
    q_adv = adv[sr];
    q_ret = ret[sr];
  }
  float4 zr[kWaveRows];
#pragma unroll
  for (int rr = 0; rr < kWaveRows; ++rr)
    zr[rr] = *reinterpret_cast<const float4*>(z2 + (int64_t)min(wrow0 + rr, B - 1) * kHid + lane * 4);
#pragma unroll
  for (int rr = 0; rr < kWaveRows; ++rr) {
    const int row = wrow0 + rr;
    if (row >= B) break;
    const float4 zz = zr[rr];
    const float z[4] = {zz.x, zz.y, zz.z, zz.w};
    float h[4], s0 = 0, s1 = 0, sv = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      h[e] = RECUR ? z[e] : fmaxf(z[e], 0.0f);
      s0 += wmu0[e] * h[e];
      s1 += wmu1[e] * h[e];
      sv += wv[e] * h[e];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
      sv += __shfl_xor(sv, off, 64);
    }
    const float m0 = s0 + bmu0, m1 = s1 + bmu1, val = sv + bv;
    if (!GRAD) {
      if (lane == 0) {
        mu_out[2 * (int64_t)row] = m0;
        mu_out[2 * (int64_t)row + 1] = m1;
        v_out[row] = val;
      }
      continue;
    }
    // PPO loss of this row (Eqs. 18-20) with value and entropy terms; its rollout data (row rows[row])
    const float a0 = __shfl(q_a0, rr, 64), a1 = __shfl(q_a1, rr, 64), olp = __shfl(q_olp, rr, 64);
    const float A = __shfl(q_adv, rr, 64), rt = __shfl(q_ret, rr, 64);
    const float is0 = expf(-ls0), is1 = expf(-ls1);
    const float u0 = (a0 - m0) * is0, u1 = (a1 - m1) * is1;
    const float logp = -0.5f * (u0 * u0 + u1 * u1) - (ls0 + ls1) - log2pi;
    const float ratio = expf(logp - olp);
    const float clipped = fminf(fmaxf(ratio, 1.0f - lc.eps), 1.0f + lc.eps);
    const float surr = fminf(ratio * A, clipped * A);
    // d(-surr)/dlogp is -A*ratio when the unclipped term is the minimum, else 0
    const bool active = ratio * A <= clipped * A;
    const float g_logp = active ? -A * ratio * lc.inv_b : 0.0f;
    const float dm0 = g_logp * (u0 * is0), dm1 = g_logp * (u1 * is1);
    const float dV = lc.c_v * 2.0f * (val - rt) * lc.inv_b;
    if (lane == 0) {
      gls0 += g_logp * (u0 * u0 - 1.0f);
      gls1 += g_logp * (u1 * u1 - 1.0f);
      gbm0 += dm0;
      gbm1 += dm1;
      gbv += dV;
      lclip += -surr * lc.inv_b;
      lval += (val - rt) * (val - rt) * lc.inv_b;
    }
    uint32_t dzp[2];
    float dhv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      gw0[e] += dm0 * h[e];
      gw1[e] += dm1 * h[e];
      gwv[e] += dV * h[e];
      const float dh = dm0 * wmu0[e] + dm1 * wmu1[e] + dV * wv[e];
      dhv[e] = dh;
      const float dz = z[e] > 0.0f ? dh : 0.0f;
      const uint32_t bits = f2bf(dz);
      gb2[e] += bf2f((uint16_t)bits);  // the bias gradient sums the same BF16 values the GEMMs consume
      if (e & 1) dzp[e >> 1] |= bits << 16; else dzp[e >> 1] = bits;
    }
    if (RECUR)
      *reinterpret_cast<float4*>(dh_out + (int64_t)row * kHid + lane * 4) = make_float4(dhv[0], dhv[1], dhv[2], dhv[3]);
    else
      *reinterpret_cast<uint2*>(dz2 + (int64_t)row * kHid + lane * 4) = make_uint2(dzp[0], dzp[1]);
  }
  if (!GRAD) return;
  float* a = acc[wave];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    a[lane * 4 + e] = gw0[e];
    a[kHid + lane * 4 + e] = gw1[e];
    a[514 + lane * 4 + e] = gwv[e];
    a[773 + lane * 4 + e] = gb2[e];
  }
  if (lane == 0) {
    a[512] = gbm0; a[513] = gbm1; a[770] = gbv; a[771] = gls0; a[772] = gls1;
    a[1029] = lclip; a[1030] = lval; a[1031] = 0.0f; a[1032] = 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHeadPart; i += 256)
    part[(int64_t)blockIdx.x * kHeadPart + i] = acc[0][i] + acc[1][i] + acc[2][i] + acc[3][i];
}

// Sum of split-K partials part[z * slice + i], z < S, in a fixed order, added
// into dst[map(i)].  A workgroup covers 4*CX consecutive outputs (CX groups of four)
// and splits S over 256/CX lanes; each lane sums its share with four loads in
// flight, then one lane per group adds the lanes' sums in lane order.
// map: 0 identity, 1 conv2 weight
// (k' = tap*16 + ci -> ci*9 + tap within each co row of 144), 2 conv1 weight
// (partial [16][16] tap-padded -> [16][9]).
constexpr int kReduceThreads = 256;

__device__ __forceinline__ int64_t reduce_dst(int map, int64_t i, bool& skip) {
  skip = false;
  if (map == 1) {
    const int co = (int)(i / 144), kk = (int)(i % 144), tap = kk >> 4, ci = kk & 15;
    return (int64_t)co * 144 + ci * 9 + tap;
  }
  if (map == 2) {
    const int co = (int)(i / 16), tap = (int)(i % 16);
    skip = tap >= 9;
    return (int64_t)co * 9 + tap;
  }
  return i;
}

// The sum over the S slices of the four outputs i0 .. i0 + 3 of this thread's group, in a fixed order:
// true (and the sums in tv) for the thread that holds the group's result.
__device__ __forceinline__ bool reduce_group(const float* part, int S, int64_t count, int64_t slice, int cx_log2,
                                             float4* red, float (&tv)[4], int64_t& i0) {
  const int CX = 1 << cx_log2, LY = kReduceThreads >> cx_log2;
  const int cx = threadIdx.x & (CX - 1), ly = threadIdx.x >> cx_log2;
  i0 = ((int64_t)blockIdx.x * CX + cx) * 4;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i0 < count) {
    if (i0 + 3 < count && (slice & 3) == 0) {
      int z = ly;
      for (; z + 3 * LY < S; z += 4 * LY) {
        const float4 v0 = *reinterpret_cast<const float4*>(part + (int64_t)z * slice + i0);
        const float4 v1 = *reinterpret_cast<const float4*>(part + (int64_t)(z + LY) * slice + i0);
        const float4 v2 = *reinterpret_cast<const float4*>(part + (int64_t)(z + 2 * LY) * slice + i0);
        const float4 v3 = *reinterpret_cast<const float4*>(part + (int64_t)(z + 3 * LY) * slice + i0);
        acc.x += v0.x; acc.y += v0.y; acc.z += v0.z; acc.w += v0.w;
        acc.x += v1.x; acc.y += v1.y; acc.z += v1.z; acc.w += v1.w;
        acc.x += v2.x; acc.y += v2.y; acc.z += v2.z; acc.w += v2.w;
        acc.x += v3.x; acc.y += v3.y; acc.z += v3.z; acc.w += v3.w;
      }
      for (; z < S; z += LY) {
        const float4 v = *reinterpret_cast<const float4*>(part + (int64_t)z * slice + i0);
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
      }
    } else {
      for (int z = ly; z < S; z += LY) {
        const float* q = part + (int64_t)z * slice + i0;
        acc.x += q[0];
        if (i0 + 1 < count) acc.y += q[1];
        if (i0 + 2 < count) acc.z += q[2];
        if (i0 + 3 < count) acc.w += q[3];
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (ly != 0 || i0 >= count) return false;
  float4 t = red[cx];
  for (int y = 1; y < LY; ++y) {
    const float4 v = red[y * CX + cx];
    t.x += v.x; t.y += v.y; t.z += v.z; t.w += v.w;
  }
  tv[0] = t.x; tv[1] = t.y; tv[2] = t.z; tv[3] = t.w;
  return true;
}

__global__ __launch_bounds__(kReduceThreads) void k_reduce(const float* part, int S, int64_t count, float* dst,
                                                           int map, int64_t slice, int cx_log2) {
  __shared__ float4 red[kReduceThreads];
  float tv[4];
  int64_t i0;
  if (!reduce_group(part, S, count, slice, cx_log2, red, tv, i0)) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = i0 + e;
    if (i >= count) break;
    bool skip;
    const int64_t d = reduce_dst(map, i, skip);
    if (skip) continue;
    dst[d] += tv[e];
  }
}

// Up to four consecutive output segments of one partial layout in one launch: segment k holds n[k]
// outputs (multiples of four) added into grads + off[k] through map[k] (0, 1 or 2 of reduce_dst).
struct ReduceSegs {
  int32_t n[4];
  int32_t map[4];
  int64_t off[4];
};

__global__ __launch_bounds__(kReduceThreads) void k_reduce_segs(const float* part, int S, int64_t count,
                                                                float* grads, ReduceSegs sg, int64_t slice,
                                                                int cx_log2) {
  __shared__ float4 red[kReduceThreads];
  float tv[4];
  int64_t i0;
  if (!reduce_group(part, S, count, slice, cx_log2, red, tv, i0)) return;
  int k = 0;
  int64_t j0 = i0;
  while (k < 3 && j0 >= sg.n[k]) j0 -= sg.n[k++];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (i0 + e >= count) break;
    bool skip;
    const int64_t d = reduce_dst(sg.map[k], j0 + e, skip);
    if (!skip) grads[sg.off[k] + d] += tv[e];
  }
}

// a[j] += q[z * stride + j] for z = 0 .. S-1 in order, j < 8.  The loads of eight slices are issued
// before their adds, so the slices cost one memory round trip per eight, not one each; the additions
// keep the order of z.
__device__ __forceinline__ void sum_slices8(const float* q, int S, int64_t stride, float a[8]) {
  int z = 0;
  for (; z + 8 <= S; z += 8) {
    float4 lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      lo[u] = *reinterpret_cast<const float4*>(q + (int64_t)(z + u) * stride);
      hi[u] = *reinterpret_cast<const float4*>(q + (int64_t)(z + u) * stride + 4);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[0] += lo[u].x; a[1] += lo[u].y; a[2] += lo[u].z; a[3] += lo[u].w;
      a[4] += hi[u].x; a[5] += hi[u].y; a[6] += hi[u].z; a[7] += hi[u].w;
    }
  }
  for (; z < S; ++z) {
    const float4 lo = *reinterpret_cast<const float4*>(q + (int64_t)z * stride);
    const float4 hi = *reinterpret_cast<const float4*>(q + (int64_t)z * stride + 4);
    a[0] += lo.x; a[1] += lo.y; a[2] += lo.z; a[3] += lo.w;
    a[4] += hi.x; a[5] += hi.y; a[6] += hi.z; a[7] += hi.w;
  }
}

// Eight ReLU outputs relu(a + bias) as BF16 into out (hi parts) and, when out_lo is given, their
// lo parts into out_lo (the split operand of the next layer).
__device__ __forceinline__ void store_relu8(const float a[8], const float* bias, int n0, uint16_t* out,
                                            uint16_t* out_lo, int64_t o) {
  uint16_t h[8], l[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float v = fmaxf(a[j] + bias[n0 + j], 0.0f);
    h[j] = f2bf(v);
    l[j] = f2bf(v - bf2f(h[j]));
  }
  *reinterpret_cast<uint4*>(out + o) = pack8(h);
  if (out_lo) *reinterpret_cast<uint4*>(out_lo + o) = pack8(l);
}

// Split-K finish of a GEMM with a bias + ReLU + BF16 epilogue: out[m][n] =
// bf16(relu(bias[n] + sum_z part[z][m][n])), z in order; 8 columns per thread (N % 8 == 0);
// out_lo (may be NULL) receives the lo parts.
__global__ void k_reduce_bias_relu_bf16(const float* part, int S, int M, int N, const float* bias, uint16_t* out,
                                        int64_t ldo, uint16_t* out_lo = nullptr) {
  const int64_t groups = (int64_t)M * (N / 8);
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = g / (N / 8);
    const int n0 = (int)(g - m * (N / 8)) * 8;
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = 0.0f;
    sum_slices8(part + m * N + n0, S, (int64_t)M * N, a);
    store_relu8(a, bias, n0, out, out_lo, m * ldo + n0);
  }
}

// The same for many slices (a small batch split many ways): each wave sums a quarter of the slices
// for 64 consecutive 8-column groups, and wave 0 adds the four quarters in order.
__global__ __launch_bounds__(256) void k_reduce_bias_relu_bf16_q(const float* part, int S, int M, int N,
                                                                 const float* bias, uint16_t* out, int64_t ldo,
                                                                 uint16_t* out_lo = nullptr) {
  __shared__ float s_q[3][64][9];
  const int64_t groups = (int64_t)M * (N / 8);
  const int64_t g = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6, sq = (S + 3) / 4;
  const int z0 = min(S, q * sq), z1 = min(S, z0 + sq);
  const int64_t m = g / (N / 8);
  const int n0 = (int)(g - m * (N / 8)) * 8;
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 0.0f;
  if (g < groups) sum_slices8(part + (int64_t)z0 * M * N + m * N + n0, z1 - z0, (int64_t)M * N, a);
  if (q > 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) s_q[q - 1][threadIdx.x & 63][j] = a[j];
  }
  __syncthreads();
  if (q == 0 && g < groups) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] += s_q[r][threadIdx.x][j];
    store_relu8(a, bias, n0, out, out_lo, m * ldo + n0);
  }
}

// Launch helper: outputs in groups of four, S split over the remaining lanes.  Large outputs
// (at least 2048 workgroups with every lane on its own group) give each lane a group and all the
// slices, so a wave reads 1 KB contiguous per slice; otherwise 16 groups x 16 lanes, fewer groups
// for tiny outputs.
inline int64_t reduce_shape(int64_t count, int& cx_log2) {
  const int64_t groups = (count + 3) / 4;
  cx_log2 = groups >= 2048LL * kReduceThreads ? 8 : 4;
  while (cx_log2 > 0 && (1LL << (cx_log2 - 1)) >= groups) --cx_log2;
  return (groups + (1LL << cx_log2) - 1) >> cx_log2;
}

inline hipError_t launch_reduce(const float* part, int S, int64_t count, float* dst, int map, int64_t slice,
                                hipStream_t st) {
  int cx_log2;
  const int64_t blocks = reduce_shape(count, cx_log2);
  k_reduce<<<(unsigned)blocks, kReduceThreads, 0, st>>>(part, S, count, dst, map, slice, cx_log2);
  return hipGetLastError();
}

inline hipError_t launch_reduce_segs(const float* part, int S, float* grads, const ReduceSegs& sg, int64_t slice,
                                     hipStream_t st) {
  const int64_t count = (int64_t)sg.n[0] + sg.n[1] + sg.n[2] + sg.n[3];
  int cx_log2;
  const int64_t blocks = reduce_shape(count, cx_log2);
  k_reduce_segs<<<(unsigned)blocks, kReduceThreads, 0, st>>>(part, S, count, grads, sg, slice, cx_log2);
  return hipGetLastError();
}

// Head sum i (of kHeadPart) -> its gradient entry or loss term.
__device__ __forceinline__ void scatter_head(int i, float s, float* grad, const Offsets& o, float* loss, float c_e) {
  if (i < 512) grad[o.muw + i] += s;
  else if (i < 514) grad[o.mub + (i - 512)] += s;
  else if (i < 770) grad[o.vw + (i - 514)] += s;
  else if (i == 770) grad[o.vb] += s;
  else if (i < 773) grad[o.lstd + (i - 771)] += s - c_e;  // entropy term: -c_e dH/dlog_std
  else if (i < 1029) { if (o.f2b >= 0) grad[o.f2b + (i - 773)] += s; }
  else if (i == 1029) loss[1] = s;
  else if (i == 1030) loss[2] = s;
}


__device__ __forceinline__ void loss_total(const float* prm, const Offsets& o, float* loss, float c_v, float c_e) {
  const float h = (prm[o.lstd] + prm[o.lstd + 1]) + 2.0f * 1.4189385332046727f;  // 0.5*log(2*pi*e) per dim
  loss[3] = h;
  loss[0] = loss[1] + c_v * loss[2] - c_e * h;
}

// The head partials' reduction, their scatter into the gradient and the loss total in one launch
// (the sums as the reduction forms them; the thread holding sums 1028 .. 1031 writes both loss terms
// and then the total).
static_assert(kHeadPart > 1030 && 1028 % 4 == 0, "the loss terms share one group of four sums");

__global__ __launch_bounds__(kReduceThreads) void k_reduce_heads(const float* part, int S, const float* prm,
                                                                 Offsets o, float* grad, float* loss, float c_v,
                                                                 float c_e, int cx_log2) {
  __shared__ float4 red[kReduceThreads];
  float tv[4];
  int64_t i0;
  if (!reduce_group(part, S, kHeadPart, kHeadPart, cx_log2, red, tv, i0)) return;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < kHeadPart) scatter_head((int)i0 + e, tv[e], grad, o, loss, c_e);
  if (i0 == 1028) loss_total(prm, o, loss, c_v, c_e);
}

inline hipError_t launch_reduce_heads(const float* part, int S, const float* prm, const Offsets& o, float* grad,
                                      float* loss, float c_v, float c_e, hipStream_t st) {
  int cx_log2;
  const int64_t blocks = reduce_shape(kHeadPart, cx_log2);
  k_reduce_heads<<<(unsigned)blocks, kReduceThreads, 0, st>>>(part, S, prm, o, grad, loss, c_v, c_e, cx_log2);
  return hipGetLastError();
}

// Bias gradients: column sums of a BF16 [rows][ch] tensor (ch divides 2048,
// rows * ch a multiple of 8) into per-block partials [gridDim.x][ch].  Thread t
// reads the 16-byte vectors t, t + 256, ... of its block's range; 256 vectors
// span 2048 elements, so a thread always sees the same eight channels.  Four
// loads are kept in flight; every sum is taken in a fixed order.
constexpr int kBiasBlocks = 512;

__device__ __forceinline__ void add_bf16x8(float* a, const uint4& v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    a[2 * j] += __uint_as_float(w[j] << 16);
    a[2 * j + 1] += __uint_as_float(w[j] & 0xffff0000u);
  }
}

__global__ __launch_bounds__(256) void k_bias_rows(const uint16_t* src, int64_t rows, int ch, float* part) {
  __shared__ float sacc[256 * 8];
  const int64_t nvec = rows * ch / 8;
  const int64_t per = ((nvec + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
  const int64_t beg = (int64_t)blockIdx.x * per, end = min(nvec, beg + per);
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int64_t i = beg + threadIdx.x;
  for (; i + 3 * 256 < end; i += 4 * 256) {
    const uint4 v0 = s4[i], v1 = s4[i + 256], v2 = s4[i + 512], v3 = s4[i + 768];
    add_bf16x8(a, v0);
    add_bf16x8(a, v1);
    add_bf16x8(a, v2);
    add_bf16x8(a, v3);
  }
  for (; i < end; i += 256) add_bf16x8(a, s4[i]);
#pragma unroll
  for (int j = 0; j < 8; ++j) sacc[threadIdx.x * 8 + j] = a[j];
  __syncthreads();
  if (threadIdx.x < ch) {
    const int c = threadIdx.x, step = ch / 8;
    float t = 0.0f;
    for (int tt = (c >> 3); tt < 256; tt += step) t += sacc[tt * 8 + (c & 7)];
    part[(int64_t)blockIdx.x * ch + c] = t;
  }
}

// BF16 copies of FP32 weight matrices for the GEMMs (rounded to nearest even).
// k_convert_bf16: dst[r][c] = bf16(src[r][c]) for c < cols, 0 for cols <= c < ld_dst; with dst_lo
// also the remainder dst_lo[r][c] = bf16(src[r][c] - bf16(src[r][c])) (the split operand's lo part).
// (one workgroup's share: workgroup blk of nblk, blockDim threads)
__device__ __forceinline__ void convert_bf16_part(const float* src, int64_t ld_src, int rows, int cols, uint16_t* dst,
                                                  int64_t ld_dst, uint16_t* dst_lo, int blk, int nblk) {
  const int64_t total = (int64_t)rows * ld_dst;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < total; i += (int64_t)nblk * blockDim.x) {
    const int64_t r = i / ld_dst, c = i - r * ld_dst;
    const float v = c < cols ? src[r * ld_src + c] : 0.0f;
    const uint16_t h = f2bf(v);
    dst[i] = h;
    if (dst_lo) dst_lo[i] = f2bf(v - bf2f(h));
  }
}

__global__ void k_convert_bf16(const float* src, int64_t ld_src, int rows, int cols, uint16_t* dst,
                               int64_t ld_dst, uint16_t* dst_lo = nullptr) {
  convert_bf16_part(src, ld_src, rows, cols, dst, ld_dst, dst_lo, blockIdx.x, gridDim.x);
}

// k_transpose_bf16: dst[c][r] = bf16(src[r][c]) through 32 x 32 LDS tiles (256 threads).
// (tile (bx, by) with 256 threads and a [32][33] LDS tile)
__device__ __forceinline__ void transpose_bf16_tile(const float* src, int64_t ld_src, int rows, int cols,
                                                    uint16_t* dst, int64_t ld_dst, float (*tile)[33], int bx, int by) {
  const int c0 = bx * 32, r0 = by * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < rows && c < cols) ? src[(int64_t)r * ld_src + c] : 0.0f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (c < cols && r < rows) dst[(int64_t)c * ld_dst + r] = f2bf(tile[tx][k]);
  }
}

__global__ __launch_bounds__(256) void k_transpose_bf16(const float* src, int64_t ld_src, int rows, int cols,
                                                        uint16_t* dst, int64_t ld_dst) {
  __shared__ float tile[32][33];
  transpose_bf16_tile(src, ld_src, rows, cols, dst, ld_dst, tile, blockIdx.x, blockIdx.y);
}

// Forward tail of a tile of kTailRows rows, for the forward-only calls: the FC1 split-K sum (slices in
// order) + bias + ReLU rounded to BF16 (or the BF16 h1 rows when S == 0), FC2 on MFMA with the k
// chunks in the GEMM engine's order, + bias, then the heads and, when eps is given, the Gaussian
// action sample.  Every value is formed by the same operations in the same order as the unfused
// sequence (split-K reduce, FC2 GEMM, k_heads, k_sample), so the outputs are bit-identical to it.
// Standard normals of the Gaussian action sample: the caller's eps [B,2], or the library's own draw
// of row b, dimension d at counter (counter, b, d) under key (seed, action domain).
struct ActDraws {
  const float* eps;
  uint64_t seed, counter;
  __device__ __forceinline__ float operator()(int64_t b, int d) const {
    return eps ? eps[2 * b + d] : rng::normal(seed, rng::kDomainAction, counter, (uint64_t)b, (uint64_t)d);
  }
};

constexpr int kTailRows = 16;
constexpr int kTailLdH = kHid + 8;   // BF16 h1 rows in LDS, padded
constexpr int kTailLdZ = kHid + 4;   // FP32 z2 rows in LDS, padded

//
// PREC (split operands): h1's lo parts ride along (h1lo rows, or formed from the slice sums) and FC2 is
// h1_hi W2_hi + h1_hi W2_lo + h1_lo W2_hi (w2lo the lo parts of the weights), k step by k step.
template <bool PREC>
__global__ __launch_bounds__(256) void k_fwd_tail(const float* prm, Offsets o, const float* part, int S,
                                                  const uint16_t* h1, const uint16_t* h1lo, const uint16_t* w2b,
                                                  const uint16_t* w2lo, int B, float* mu_out, float* v_out,
                                                  bool sample, ActDraws eps, float* act, float* logp) {
  __shared__ __align__(16) uint16_t s_h[(PREC ? 2 : 1) * kTailRows * kTailLdH];
  __shared__ __align__(16) float s_z[kTailRows * kTailLdZ];
  uint16_t* const s_hl = s_h + (PREC ? kTailRows * kTailLdH : 0);
  const int row0 = blockIdx.x * kTailRows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const float* b1 = prm + o.f1b;
  // the sample's normals of the wave's rows (4 w .. 4 w + 3, two each), one per lane 0..7, drawn up
  // front: a library draw is a long dependent chain that the loads and MFMAs below can hide
  float my_eps = 0.0f;
  if (sample && lane < 8 && row0 + 4 * wave + (lane >> 1) < B) my_eps = eps(row0 + 4 * wave + (lane >> 1), lane & 1);
  for (int g = threadIdx.x; g < kTailRows * (kHid / 8); g += 256) {
    const int r = g / (kHid / 8), n0 = (g % (kHid / 8)) * 8;
    const int64_t m = row0 + r;
    uint4 v = make_uint4(0u, 0u, 0u, 0u), vl = v;
    if (m < B) {
      if (S > 0) {
        float a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = 0.0f;
        sum_slices8(part + m * kHid + n0, S, (int64_t)B * kHid, a);
        uint16_t h[8], l[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float y = fmaxf(a[j] + b1[n0 + j], 0.0f);
          h[j] = f2bf(y);
          l[j] = f2bf(y - bf2f(h[j]));
        }
        v = pack8(h);
        vl = pack8(l);
      } else {
        v = *reinterpret_cast<const uint4*>(h1 + m * kHid + n0);
        if (PREC) vl = *reinterpret_cast<const uint4*>(h1lo + m * kHid + n0);
      }
    }
    *reinterpret_cast<uint4*>(s_h + r * kTailLdH + n0) = v;
    if (PREC) *reinterpret_cast<uint4*>(s_hl + r * kTailLdH + n0) = vl;
  }
  __syncthreads();
  // FC2: wave w owns columns 64 w .. 64 w + 63 (four 16-column fragments)
  gemm::f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = gemm::f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    const gemm::bf16x8 af =
        __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_h + lr * kTailLdH + k0 + 8 * lg));
    gemm::bf16x8 afl = af;
    if (PREC)
      afl = __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(s_hl + lr * kTailLdH + k0 + 8 * lg));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = 64 * wave + 16 * j + lr;
      const gemm::bf16x8 bf =
          __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(w2b + (int64_t)n * kHid + k0 + 8 * lg));
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[j], 0, 0, 0);
      if (PREC) {
        const gemm::bf16x8 bfl =
            __builtin_bit_cast(gemm::bf16x8, *reinterpret_cast<const uint4*>(w2lo + (int64_t)n * kHid + k0 + 8 * lg));
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfl, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl, bf, acc[j], 0, 0, 0);
      }
    }
  }
  const float* b2 = prm + o.f2b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 64 * wave + 16 * j + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i) s_z[(4 * lg + i) * kTailLdZ + c] = acc[j][i] + b2[c];
  }
  __syncthreads();
  // heads: wave w takes rows 4 w .. 4 w + 3, lane l holds z2 columns 4 l .. 4 l + 3 (as k_heads)
  float wmu0[4], wmu1[4], wv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    wmu0[e] = prm[o.muw + lane * 4 + e];
    wmu1[e] = prm[o.muw + kHid + lane * 4 + e];
    wv[e] = prm[o.vw + lane * 4 + e];
  }
  const float bmu0 = prm[o.mub], bmu1 = prm[o.mub + 1], bv = prm[o.vb];
  for (int rr = 0; rr < kTailRows / 4; ++rr) {
    const int r = 4 * wave + rr;
    const int64_t row = row0 + r;
    if (row >= B) break;
    const float4 zz = *reinterpret_cast<const float4*>(s_z + r * kTailLdZ + lane * 4);
    const float z[4] = {zz.x, zz.y, zz.z, zz.w};
    float s0 = 0, s1 = 0, sv = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float h = fmaxf(z[e], 0.0f);
      s0 += wmu0[e] * h;
      s1 += wmu1[e] * h;
      sv += wv[e] * h;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
      sv += __shfl_xor(sv, off, 64);
    }
    const float e0 = __shfl(my_eps, 2 * rr, 64), e1 = __shfl(my_eps, 2 * rr + 1, 64);
    if (lane == 0) {
      const float m0 = s0 + bmu0, m1 = s1 + bmu1;
      if (mu_out) {
        mu_out[2 * row] = m0;
        mu_out[2 * row + 1] = m1;
      }
      v_out[row] = sv + bv;
      if (sample) {
        const float ls0 = prm[o.lstd], ls1 = prm[o.lstd + 1];
        act[2 * row] = m0 + expf(ls0) * e0;
        act[2 * row + 1] = m1 + expf(ls1) * e1;
        logp[row] = -0.5f * (e0 * e0 + e1 * e1) - (ls0 + ls1) - 1.8378770664093453f;
      }
    }
  }
}

// Gaussian action sampling: act = mu + exp(log_std) eps, logp = log N(act; mu, exp(log_std)).
__global__ void k_sample(const float* prm, Offsets o, const float* mu, ActDraws eps, int B, float* act,
                         float* logp) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float ls0 = prm[o.lstd], ls1 = prm[o.lstd + 1];
  const float e0 = eps(b, 0), e1 = eps(b, 1);
  act[2 * (int64_t)b] = mu[2 * (int64_t)b] + expf(ls0) * e0;
  act[2 * (int64_t)b + 1] = mu[2 * (int64_t)b + 1] + expf(ls1) * e1;
  logp[b] = -0.5f * (e0 * e0 + e1 * e1) - (ls0 + ls1) - 1.8378770664093453f;
}

// Keyed permutation of [0, n): out[j] = the image of j (rng::permute), each lane walking its own
// cycle through Feistel evaluations.
__global__ void k_permutation(int32_t n, int h, uint64_t seed, uint64_t counter, int32_t* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = rng::permute((int32_t)j, n, h, seed, counter);
}

// The same permutation in two passes: the Feistel image of every point of the 2^(2h) domain (one
// evaluation per lane, all lanes busy), then each j < n follows its cycle through that table, so the
// walk past images >= n costs a load per hop instead of eight Philox blocks.
__global__ void k_feistel_table(int h, uint64_t seed, uint64_t counter, uint32_t* tab) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < (1ull << (2 * h))) tab[v] = (uint32_t)rng::feistel(v, h, seed, counter);
}

__global__ void k_permutation_walk(int32_t n, const uint32_t* __restrict__ tab, int32_t* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t y = tab[j];
  while (y >= (uint32_t)n) y = tab[y];   // ends: j's cycle returns to j < n
  out[j] = (int32_t)y;
}

// dst row i = src row idx[i]; rows of `words` 32-bit words, 16-byte vectors when `vec`.
__global__ void k_gather_rows(const uint32_t* src, int64_t words, const int32_t* idx, int n, uint32_t* dst,
                              int vec) {
  const int64_t total = vec ? (int64_t)n * (words >> 2) : (int64_t)n * words;
  const int64_t per = vec ? (words >> 2) : words;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / per, c = i - r * per;
    const int64_t s = idx[r];
    if (vec) {
      reinterpret_cast<uint4*>(dst)[r * per + c] = reinterpret_cast<const uint4*>(src)[s * per + c];
    } else {
      dst[r * per + c] = src[s * per + c];
    }
  }
}

__global__ void k_gae(const float* rew, const float* val, const uint8_t* done, const float* last, int T, int N,
                      float gamma, float lam, float* adv, float* ret) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float nxt = last[n], acc = 0.0f;
  for (int t = T - 1; t >= 0; --t) {
    const int64_t i = (int64_t)t * N + n;
    const float nonterm = done[i] ? 0.0f : 1.0f;
    const float delta = rew[i] + gamma * nxt * nonterm - val[i];
    acc = delta + gamma * lam * nonterm * acc;
    adv[i] = acc;
    ret[i] = acc + val[i];
    nxt = val[i];
  }
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

}  // namespace pol
}  // namespace aslam
