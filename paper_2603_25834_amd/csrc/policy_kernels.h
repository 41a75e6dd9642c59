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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "aslam.h"
#include "gemm_bf16.h"

namespace aslam {
namespace pol {

using gemm::bf2f;
using gemm::f2bf;

constexpr int kCrop = 64, kA1 = 32, kA2 = 16, kC1 = 16, kC2 = 32, kHid = 256, kFeat = kC2 * kA2 * kA2;

struct Offsets {
  int64_t c1w, c1b, c2w, c2b, f1w, f1b, f2w, f2b, muw, mub, vw, vb, lstd, total;
  int32_t k1;  // FC1 input width = 8192 + R + 12
};

inline Offsets offsets(int32_t n_scan) {
  Offsets o;
  o.k1 = kFeat + n_scan + 12;
  int64_t p = 0;
  o.c1w = p; p += kC1 * 9;
  o.c1b = p; p += kC1;
  o.c2w = p; p += kC2 * kC1 * 9;
  o.c2b = p; p += kC2;
  o.f1w = p; p += (int64_t)kHid * o.k1;
  o.f1b = p; p += kHid;
  o.f2w = p; p += kHid * kHid;
  o.f2b = p; p += kHid;
  o.muw = p; p += 2 * kHid;
  o.mub = p; p += 2;
  o.vw = p; p += kHid;
  o.vb = p; p += 1;
  o.lstd = p; p += 2;
  o.total = p;
  return o;
}

// ------------------------------------------------------------------ loaders

__device__ __forceinline__ void zero8(uint16_t v[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = 0;
}

__device__ __forceinline__ void unpack8(const uint4 w, uint16_t v[8]) {
  v[0] = w.x & 0xffff; v[1] = w.x >> 16; v[2] = w.y & 0xffff; v[3] = w.y >> 16;
  v[4] = w.z & 0xffff; v[5] = w.z >> 16; v[6] = w.w & 0xffff; v[7] = w.w >> 16;
}

// BF16 matrix, element (i, k) at p[i*ld + k]; contiguous along k.
struct LdBF16K {
  static constexpr bool kMajor = true;
  const uint16_t* p; int64_t ld; int rows, cols;
  __device__ void fetch(int i, int k, uint16_t v[8]) const {
    if (i >= rows || k >= cols) { zero8(v); return; }
    const uint16_t* q = p + (int64_t)i * ld + k;
    if (k + 8 <= cols && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) {
      unpack8(*reinterpret_cast<const uint4*>(q), v);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (k + j < cols) ? q[j] : (uint16_t)0;
    }
  }
};

// BF16 matrix, element (i, k) at p[k*ld + i]; contiguous along i.
struct LdBF16I {
  static constexpr bool kMajor = false;
  const uint16_t* p; int64_t ld; int rows, cols;
  __device__ void fetch(int i, int k, uint16_t v[8]) const {
    if (i >= rows || k >= cols) { zero8(v); return; }
    const uint16_t* q = p + (int64_t)k * ld + i;
    if (i + 8 <= rows && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) {
      unpack8(*reinterpret_cast<const uint4*>(q), v);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (i + j < rows) ? q[j] : (uint16_t)0;
    }
  }
};

// FP32 matrix rounded to BF16 on load, element (i, k) at p[i*ld + k].
struct LdF32K {
  static constexpr bool kMajor = true;
  const float* p; int64_t ld; int rows, cols;
  __device__ void fetch(int i, int k, uint16_t v[8]) const {
    if (i >= rows || k >= cols) { zero8(v); return; }
    const float* q = p + (int64_t)i * ld + k;
    if (k + 8 <= cols && ((reinterpret_cast<uintptr_t>(q) & 15) == 0)) {
      const float4 a = *reinterpret_cast<const float4*>(q);
      const float4 b = *reinterpret_cast<const float4*>(q + 4);
      v[0] = f2bf(a.x); v[1] = f2bf(a.y); v[2] = f2bf(a.z); v[3] = f2bf(a.w);
      v[4] = f2bf(b.x); v[5] = f2bf(b.y); v[6] = f2bf(b.z); v[7] = f2bf(b.w);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (k + j < cols) ? f2bf(q[j]) : (uint16_t)0;
    }
  }
};

// FP32 matrix rounded to BF16 on load, element (i, k) at p[k*ld + i].
struct LdF32I {
  static constexpr bool kMajor = false;
  const float* p; int64_t ld; int rows, cols;
  __device__ void fetch(int i, int k, uint16_t v[8]) const {
    if (i >= rows || k >= cols) { zero8(v); return; }
    const float* q = p + (int64_t)k * ld + i;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (i + j < rows) ? f2bf(q[j]) : (uint16_t)0;
  }
};

// FC1 input X[b][k] = [a2 (BF16, 8192) | scan (FP32, R) | state (FP32, 12)].
struct XSrc {
  const uint16_t* a2; const float* scan; const float* state; int R; int B; int k1;
  __device__ __forceinline__ uint16_t at(int b, int k) const {
    if (k < kFeat) return a2[(int64_t)b * kFeat + k];
    if (k < kFeat + R) return f2bf(scan[(int64_t)b * R + (k - kFeat)]);
    if (k < k1) return f2bf(state[(int64_t)b * 12 + (k - kFeat - R)]);
    return 0;
  }
};

// A operand of FC1 forward: (i = b, k).
struct LdXK {
  static constexpr bool kMajor = true;
  XSrc x;
  __device__ void fetch(int i, int k, uint16_t v[8]) const {
    if (i >= x.B) { zero8(v); return; }
    if (k + 8 <= kFeat) {
      unpack8(*reinterpret_cast<const uint4*>(x.a2 + (int64_t)i * kFeat + k), v);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = x.at(i, k + j);
    }
  }
};

// B operand of the FC1 weight gradient: B(k = b, n = i) = X[b][i], contiguous along i.
struct LdXI {
  static constexpr bool kMajor = false;
  XSrc x;
  __device__ void fetch(int i, int k, uint16_t v[8]) const {
    if (k >= x.B || i >= x.k1) { zero8(v); return; }
    if (i + 8 <= kFeat) {
      unpack8(*reinterpret_cast<const uint4*>(x.a2 + (int64_t)k * kFeat + i), v);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = x.at(k, i + j);
    }
  }
};

// conv2 input as im2col rows: A(m = b*256 + p, k = tap*16 + ci) from a1 [b][32][32][16] (BF16).
struct LdIm2colK {
  static constexpr bool kMajor = true;
  const uint16_t* a1; int M;
  __device__ void fetch(int m, int k, uint16_t v[8]) const {
    const int tap = k >> 4, ci0 = k & 15;
    if (m >= M || tap >= 9) { zero8(v); return; }
    const int b = m >> 8, p = m & 255;
    const int y = 2 * (p >> 4) + tap / 3 - 1, x = 2 * (p & 15) + tap % 3 - 1;
    if (y < 0 || y >= kA1 || x < 0 || x >= kA1) { zero8(v); return; }
    unpack8(*reinterpret_cast<const uint4*>(a1 + (((int64_t)b * kA1 + y) * kA1 + x) * kC1 + ci0), v);
  }
};

// conv2 weights as B(k = tap*16 + ci, n = co) = W2[co][ci][tap] (FP32 params -> BF16).
struct LdW2K {
  static constexpr bool kMajor = true;
  const float* w;  // [32][16][9]
  __device__ void fetch(int co, int k, uint16_t v[8]) const {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kk = k + j, tap = kk >> 4, ci = kk & 15;
      v[j] = (co < kC2 && tap < 9) ? f2bf(w[(co * kC1 + ci) * 9 + tap]) : (uint16_t)0;
    }
  }
};

// conv2 weight gradient: A(m = co, k = b*256 + p) = dz2c[b][co*256 + p] (contiguous along k).
struct LdDz2cK {
  static constexpr bool kMajor = true;
  const uint16_t* d; int K;
  __device__ void fetch(int co, int k, uint16_t v[8]) const {
    if (co >= kC2 || k >= K) { zero8(v); return; }
    const int b = k >> 8, p = k & 255;
    unpack8(*reinterpret_cast<const uint4*>(d + (int64_t)b * kFeat + co * 256 + p), v);
  }
};

// conv2 weight gradient: B(k = b*256 + p, n = tap*16 + ci) = im2col(a1), contiguous along n.
struct LdIm2colI {
  static constexpr bool kMajor = false;
  const uint16_t* a1; int K;
  __device__ void fetch(int n, int k, uint16_t v[8]) const {
    const int tap = n >> 4, ci0 = n & 15;
    if (k >= K || tap >= 9) { zero8(v); return; }
    const int b = k >> 8, p = k & 255;
    const int y = 2 * (p >> 4) + tap / 3 - 1, x = 2 * (p & 15) + tap % 3 - 1;
    if (y < 0 || y >= kA1 || x < 0 || x >= kA1) { zero8(v); return; }
    unpack8(*reinterpret_cast<const uint4*>(a1 + (((int64_t)b * kA1 + y) * kA1 + x) * kC1 + ci0), v);
  }
};

// Input gradient of conv2 for one sub-pixel phase (ry, rx) of the 32x32 grid:
// input pixel (2qy+ry, 2qx+rx) receives tap (ky, kx) of output pixel
// (qy + (ry+1-ky)/2, qx + (rx+1-kx)/2) when ky = ry+1 (mod 2) and kx = rx+1 (mod 2).
struct Phase {
  int ry, rx, nty, ntx;
  int ky[2], kx[2];
};

__host__ __device__ inline Phase make_phase(int ry, int rx) {
  Phase ph;
  ph.ry = ry; ph.rx = rx;
  if (ry == 0) { ph.nty = 1; ph.ky[0] = 1; ph.ky[1] = 1; } else { ph.nty = 2; ph.ky[0] = 0; ph.ky[1] = 2; }
  if (rx == 0) { ph.ntx = 1; ph.kx[0] = 1; ph.kx[1] = 1; } else { ph.ntx = 2; ph.kx[0] = 0; ph.kx[1] = 2; }
  return ph;
}

// A(m = b*256 + qy*16 + qx, k = j*32 + co) = dz2c[b][co][py][px] for the phase's tap j.
struct LdPhaseA {
  static constexpr bool kMajor = false;
  const uint16_t* d; int M; Phase ph;
  __device__ void fetch(int m, int k, uint16_t v[8]) const {
    const int j = k >> 5, co = k & 31;
    if (m >= M || j >= ph.nty * ph.ntx) { zero8(v); return; }
    const int ky = ph.ky[j / ph.ntx], kx = ph.kx[j % ph.ntx];
    const int b = m >> 8, qy = (m >> 4) & 15, qx0 = m & 15;
    const int py = qy + (ph.ry + 1 - ky) / 2;
    const int dx = (ph.rx + 1 - kx) / 2;
    const uint16_t* row = d + (int64_t)b * kFeat + co * 256 + py * 16;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int px = qx0 + t + dx;
      v[t] = (py < kA2 && px < kA2) ? row[px] : (uint16_t)0;
    }
  }
};

// B(k = j*32 + co, n = ci) = W2[co][ci][ky_j][kx_j].
struct LdPhaseB {
  static constexpr bool kMajor = true;
  const float* w; Phase ph;
  __device__ void fetch(int ci, int k, uint16_t v[8]) const {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = k + t, j = kk >> 5, co = kk & 31;
      if (ci >= kC1 || j >= ph.nty * ph.ntx) { v[t] = 0; continue; }
      const int ky = ph.ky[j / ph.ntx], kx = ph.kx[j % ph.ntx];
      v[t] = f2bf(w[(co * kC1 + ci) * 9 + ky * 3 + kx]);
    }
  }
};

// conv1 weight gradient: A(m = co, k = b*1024 + y*32 + x) = dz1c[b][y][x][co] (contiguous along m).
struct LdDz1cI {
  static constexpr bool kMajor = false;
  const uint16_t* d; int K;
  __device__ void fetch(int co, int k, uint16_t v[8]) const {
    if (k >= K || co >= kC1) { zero8(v); return; }
    unpack8(*reinterpret_cast<const uint4*>(d + (int64_t)k * kC1 + co), v);
  }
};

__device__ __forceinline__ uint16_t crop_in(const int16_t* crop, int b, int y, int x) {
  if (y < 0 || y >= kCrop || x < 0 || x >= kCrop) return 0;
  return f2bf((float)crop[((int64_t)b * kCrop + y) * kCrop + x] * (1.0f / 256.0f));
}

// conv1 weight gradient: B(k = b*1024 + y*32 + x, n = tap) = input (2y+ky-1, 2x+kx-1).
struct LdCropTapK {
  static constexpr bool kMajor = true;
  const int16_t* crop; int K;
  __device__ void fetch(int tap, int k, uint16_t v[8]) const {
    if (tap >= 9) { zero8(v); return; }
    const int ky = tap / 3, kx = tap % 3;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = k + t;
      if (kk >= K) { v[t] = 0; continue; }
      const int b = kk >> 10, y = (kk >> 5) & 31, x = kk & 31;
      v[t] = crop_in(crop, b, 2 * y + ky - 1, 2 * x + kx - 1);
    }
  }
};

// ---------------------------------------------------------------- epilogues

struct EpiConv2 {  // a2[b][co*256 + p] = bf16(relu(v + bias))
  uint16_t* a2; const float* bias;
  __device__ void store(int m, int n, float v, bool ok) const {
    if (!ok) return;
    a2[(int64_t)(m >> 8) * kFeat + n * 256 + (m & 255)] = f2bf(fmaxf(v + bias[n], 0.0f));
  }
};

struct EpiBiasReluBF16 {
  uint16_t* out; const float* bias; int64_t ld;
  __device__ void store(int m, int n, float v, bool ok) const {
    if (ok) out[(int64_t)m * ld + n] = f2bf(fmaxf(v + bias[n], 0.0f));
  }
};

struct EpiBiasF32 {
  float* out; const float* bias; int64_t ld;
  __device__ void store(int m, int n, float v, bool ok) const {
    if (ok) out[(int64_t)m * ld + n] = v + bias[n];
  }
};

// Split-K partial sums: slice blockIdx.z of a [splits][M][N] FP32 buffer.
struct EpiPartial {
  float* part; int64_t ld; int64_t slice;
  __device__ void store(int m, int n, float v, bool ok) const {
    if (ok) part[(int64_t)blockIdx.z * slice + (int64_t)m * ld + n] = v;
  }
};

// Gradient through a ReLU whose output (BF16) is `act`: out = bf16(act > 0 ? v : 0).
struct EpiReluGradBF16 {
  uint16_t* out; const uint16_t* act; int64_t ld;
  __device__ void store(int m, int n, float v, bool ok) const {
    if (!ok) return;
    const int64_t o = (int64_t)m * ld + n;
    out[o] = bf2f(act[o]) > 0.0f ? f2bf(v) : (uint16_t)0;
  }
};

// Input gradient of conv2 for one phase, masked by conv1's ReLU: dz1c[b][y][x][ci] (BF16).
struct EpiPhase {
  uint16_t* dz1c; const uint16_t* a1; int ry, rx;
  __device__ void store(int m, int n, float v, bool ok) const {
    if (!ok) return;
    const int b = m >> 8, y = 2 * ((m >> 4) & 15) + ry, x = 2 * (m & 15) + rx;
    const int64_t o = (((int64_t)b * kA1 + y) * kA1 + x) * kC1 + n;
    dz1c[o] = bf2f(a1[o]) > 0.0f ? f2bf(v) : (uint16_t)0;
  }
};

// ---------------------------------------------------------------- kernels

// conv1 (1 -> 16, 3x3, stride 2, pad 1) + ReLU for one sample per workgroup:
// a1[b][y][x][co] = bf16(relu(b1[co] + sum_tap bf16(w1[co][tap]) * bf16(L/256))).
__global__ __launch_bounds__(256) void k_conv1(const float* prm, Offsets o, const int16_t* crop, uint16_t* a1,
                                               int B) {
  __shared__ float w[kC1 * 9];
  __shared__ float bias[kC1];
  __shared__ float in[kCrop * kCrop];
  for (int i = threadIdx.x; i < kC1 * 9; i += 256) w[i] = bf2f(f2bf(prm[o.c1w + i]));
  if (threadIdx.x < kC1) bias[threadIdx.x] = prm[o.c1b + threadIdx.x];
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    __syncthreads();
    for (int i = threadIdx.x; i < kCrop * kCrop; i += 256)
      in[i] = bf2f(f2bf((float)crop[(int64_t)b * kCrop * kCrop + i] * (1.0f / 256.0f)));
    __syncthreads();
    for (int px = threadIdx.x; px < kA1 * kA1; px += 256) {
      const int y = px >> 5, x = px & 31;
      float t[9];
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int iy = 2 * y + ky - 1, ix = 2 * x + kx - 1;
          t[ky * 3 + kx] = (iy >= 0 && iy < kCrop && ix >= 0 && ix < kCrop) ? in[iy * kCrop + ix] : 0.0f;
        }
      uint32_t packed[8];
#pragma unroll
      for (int c = 0; c < kC1; c += 2) {
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          s0 += w[c * 9 + k] * t[k];
          s1 += w[(c + 1) * 9 + k] * t[k];
        }
        packed[c / 2] = (uint32_t)f2bf(fmaxf(s0 + bias[c], 0.0f)) |
                        ((uint32_t)f2bf(fmaxf(s1 + bias[c + 1], 0.0f)) << 16);
      }
      uint4* dst = reinterpret_cast<uint4*>(a1 + ((int64_t)b * kA1 * kA1 + px) * kC1);
      dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
      dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
    }
  }
}

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

template <bool GRAD>
__global__ __launch_bounds__(256) void k_heads(const float* prm, Offsets o, const float* z2, int B, float* mu_out,
                                               float* v_out, const float* act, const float* old_logp,
                                               const float* adv, const float* ret, LossCoef lc, uint16_t* dz2,
                                               float* part) {
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
  for (int rr = 0; rr < kHeadRows / 4; ++rr) {
    const int row = blockIdx.x * kHeadRows + wave * (kHeadRows / 4) + rr;
    if (row >= B) break;
    const float4 zz = *reinterpret_cast<const float4*>(z2 + (int64_t)row * kHid + lane * 4);
    const float z[4] = {zz.x, zz.y, zz.z, zz.w};
    float h[4], s0 = 0, s1 = 0, sv = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      h[e] = fmaxf(z[e], 0.0f);
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
    // PPO loss of this row (Eqs. 18-20) with value and entropy terms
    const float is0 = expf(-ls0), is1 = expf(-ls1);
    const float u0 = (act[2 * (int64_t)row] - m0) * is0, u1 = (act[2 * (int64_t)row + 1] - m1) * is1;
    const float logp = -0.5f * (u0 * u0 + u1 * u1) - (ls0 + ls1) - log2pi;
    const float ratio = expf(logp - old_logp[row]);
    const float A = adv[row];
    const float clipped = fminf(fmaxf(ratio, 1.0f - lc.eps), 1.0f + lc.eps);
    const float surr = fminf(ratio * A, clipped * A);
    // d(-surr)/dlogp is -A*ratio when the unclipped term is the minimum, else 0
    const bool active = ratio * A <= clipped * A;
    const float g_logp = active ? -A * ratio * lc.inv_b : 0.0f;
    const float dm0 = g_logp * (u0 * is0), dm1 = g_logp * (u1 * is1);
    const float dV = lc.c_v * 2.0f * (val - ret[row]) * lc.inv_b;
    if (lane == 0) {
      gls0 += g_logp * (u0 * u0 - 1.0f);
      gls1 += g_logp * (u1 * u1 - 1.0f);
      gbm0 += dm0;
      gbm1 += dm1;
      gbv += dV;
      lclip += -surr * lc.inv_b;
      lval += (val - ret[row]) * (val - ret[row]) * lc.inv_b;
    }
    uint32_t dzp[2];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      gw0[e] += dm0 * h[e];
      gw1[e] += dm1 * h[e];
      gwv[e] += dV * h[e];
      const float dh = dm0 * wmu0[e] + dm1 * wmu1[e] + dV * wv[e];
      const float dz = z[e] > 0.0f ? dh : 0.0f;
      const uint32_t bits = f2bf(dz);
      gb2[e] += bf2f((uint16_t)bits);  // the bias gradient sums the same BF16 values the GEMMs consume
      if (e & 1) dzp[e >> 1] |= bits << 16; else dzp[e >> 1] = bits;
    }
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

// Sum of split-K partials [S][count] in a fixed order, added into dst[map(i)].
// map: 0 identity; 1 conv2 weight (k' = tap*16 + ci -> ci*9 + tap within each co row of 144);
//      2 conv1 weight (partial [16][16] tap-padded -> [16][9]).
__global__ void k_reduce(const float* part, int S, int64_t count, float* dst, int map, int64_t slice) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * slice + i];
    int64_t d = i;
    if (map == 1) {
      const int co = (int)(i / 144), kk = (int)(i % 144), tap = kk >> 4, ci = kk & 15;
      d = (int64_t)co * 144 + ci * 9 + tap;
    } else if (map == 2) {
      const int co = (int)(i / 16), tap = (int)(i % 16);
      if (tap >= 9) continue;
      d = (int64_t)co * 9 + tap;
    }
    dst[d] += s;
  }
}

// Head partials [nb][kHeadPart] -> gradient vector and loss terms.
__global__ void k_reduce_heads(const float* part, int nb, float* grad, Offsets o, float* loss, float c_e,
                               float c_v) {
  for (int i = threadIdx.x; i < kHeadPart; i += blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < nb; ++z) s += part[(int64_t)z * kHeadPart + i];
    if (i < 512) grad[o.muw + i] += s;
    else if (i < 514) grad[o.mub + (i - 512)] += s;
    else if (i < 770) grad[o.vw + (i - 514)] += s;
    else if (i == 770) grad[o.vb] += s;
    else if (i < 773) grad[o.lstd + (i - 771)] += s - c_e;  // entropy term: -c_e dH/dlog_std
    else if (i < 1029) grad[o.f2b + (i - 773)] += s;
    else if (i == 1029) loss[1] = s;
    else if (i == 1030) loss[2] = s;
  }
}

__global__ void k_loss_total(const float* prm, Offsets o, float* loss, float c_v, float c_e) {
  const float h = (prm[o.lstd] + prm[o.lstd + 1]) + 2.0f * 1.4189385332046727f;  // 0.5*log(2*pi*e) per dim
  loss[3] = h;
  loss[0] = loss[1] + c_v * loss[2] - c_e * h;
}

// Bias gradients: column sums of a BF16 [rows][ch] tensor (ch divides 256)
// into per-block partials [gridDim.x][ch]; thread t always sees channel t % ch.
__global__ __launch_bounds__(256) void k_bias_rows(const uint16_t* src, int64_t rows, int ch, float* part) {
  __shared__ float sacc[256];
  const int64_t total = rows * ch;
  const int64_t per = ((total + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
  const int64_t beg = (int64_t)blockIdx.x * per, end = min(total, beg + per);
  float s = 0.0f;
  for (int64_t i = beg + threadIdx.x; i < end; i += 256) s += bf2f(src[i]);
  sacc[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < ch) {  // fixed summation order: deterministic
    float t = 0.0f;
    for (int j = threadIdx.x; j < 256; j += ch) t += sacc[j];
    part[(int64_t)blockIdx.x * ch + threadIdx.x] = t;
  }
}

// conv2 bias gradient: sums of dz2c[b][co][p] over b and p; thread t owns co = t / 8.
__global__ __launch_bounds__(256) void k_bias_c2(const uint16_t* dz2c, int B, float* part) {
  __shared__ float sacc[256];
  const int co = threadIdx.x >> 3, sub = threadIdx.x & 7;
  const int per = (B + gridDim.x - 1) / gridDim.x;
  const int b0 = blockIdx.x * per, b1 = min(B, b0 + per);
  float s = 0.0f;
  for (int b = b0; b < b1; ++b) {
    const uint16_t* row = dz2c + (int64_t)b * kFeat + co * 256;
    for (int p = sub; p < 256; p += 8) s += bf2f(row[p]);
  }
  sacc[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < kC2) {  // fixed summation order: deterministic
    float t = 0.0f;
    for (int j = 0; j < 8; ++j) t += sacc[threadIdx.x * 8 + j];
    part[(int64_t)blockIdx.x * kC2 + threadIdx.x] = t;
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
