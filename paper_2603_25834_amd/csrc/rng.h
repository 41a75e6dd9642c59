// rng.h -- counter-based random numbers of the library (device side).
//
// The workload's odometry and loop-closure noise, the paper's range noise
// (Sec. IV-A: Gaussian, 0.01 m) and PPO's Gaussian action samples (Sec. III-F)
// are standard normals; PPO also shuffles its minibatches.  Every draw is a
// pure function of (key, counter), so any thread computes its own draw with
// no state to carry between launches and a replayed step draws the same
// numbers as the first run:
//   * the block generator is Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
//     "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
//     two 64x64->128-bit products over a 4-word counter, the 2-word key
//     bumped by the two Weyl increments between rounds;
//   * one normal per block: the Irwin-Hall sum of its twelve 21-bit fields
//     (bits 63..43, 42..22 and 21..1 of each word), centred on 6 (2^21 - 1)
//     and scaled by 2^-21 -- exact in FP32, mean 0, variance 1 - 2^-42,
//     support [-6, 6];
//   * a keyed permutation of [0, n): an 8-round balanced Feistel network on
//     the smallest even bit width b >= 2 with 2^b >= n, round function = the
//     low b/2 bits of word 0 of the block at counter (counter, right half,
//     round, 0) under key (seed, kDomainPerm), walked along its cycle until
//     the image falls below n.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aslam {
namespace rng {

constexpr uint64_t kDomainEnv = 1;     // env step: counter (robot's step count, robot, draw index)
constexpr uint64_t kDomainAction = 2;  // action sampling: counter (caller's counter, row, dimension)
constexpr uint64_t kDomainPerm = 3;    // minibatch permutations

struct Block {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1) {
  constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;   // multiplies counter word 0
  constexpr uint64_t kMulB = 0xCA5A826395121157ull;   // multiplies counter word 2
  constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;  // key word 0 increment
  constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;  // key word 1 increment
#pragma unroll
  for (int rd = 0; rd < 10; ++rd) {
    const uint64_t a_lo = kMulA * c0, a_hi = __umul64hi(kMulA, c0);
    const uint64_t b_lo = kMulB * c2, b_hi = __umul64hi(kMulB, c2);
    const uint64_t n0 = b_hi ^ c1 ^ k0;
    const uint64_t n2 = a_hi ^ c3 ^ k1;
    c0 = n0;
    c1 = b_lo;
    c2 = n2;
    c3 = a_lo;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  return Block{c0, c1, c2, c3};
}

__device__ __forceinline__ int32_t fields21(uint64_t w) {
  constexpr uint64_t m = (1ull << 21) - 1;
  return (int32_t)((w >> 43) & m) + (int32_t)((w >> 22) & m) + (int32_t)((w >> 1) & m);
}

// Standard normal at counter (c0, c1, c2, 0) under key (seed, domain).
__device__ __forceinline__ float normal(uint64_t seed, uint64_t domain, uint64_t c0, uint64_t c1, uint64_t c2) {
  const Block b = philox4x64_10(c0, c1, c2, 0ull, seed, domain);
  const int32_t s = fields21(b.w0) + fields21(b.w1) + fields21(b.w2) + fields21(b.w3);   // < 2^25
  return (float)(s - 6 * ((1 << 21) - 1)) * (1.0f / 2097152.0f);
}

// Feistel image of v (2h bits) under (seed, counter).
__device__ __forceinline__ uint64_t feistel(uint64_t v, int h, uint64_t seed, uint64_t counter) {
  const uint64_t mask = (1ull << h) - 1ull;
  uint64_t left = v >> h, right = v & mask;
  for (uint64_t rd = 0; rd < 8; ++rd) {
    const Block b = philox4x64_10(counter, right, rd, 0ull, seed, kDomainPerm);
    const uint64_t f = left ^ (b.w0 & mask);
    left = right;
    right = f;
  }
  return (left << h) | right;
}

// Half width h of the Feistel domain of a permutation of [0, n), n >= 1.
__host__ __device__ inline int perm_half_bits(int64_t n) {
  int b = 2;
  while ((1ll << b) < n) b += 2;
  return b >> 1;
}

// Image of j < n under the permutation keyed by (seed, counter): cycle walking from j's Feistel
// image; it ends because j's cycle returns to j.
__device__ __forceinline__ int32_t permute(int32_t j, int32_t n, int h, uint64_t seed, uint64_t counter) {
  uint64_t y = feistel((uint64_t)j, h, seed, counter);
  while (y >= (uint64_t)n) y = feistel(y, h, seed, counter);
  return (int32_t)y;
}

}  // namespace rng
}  // namespace aslam
