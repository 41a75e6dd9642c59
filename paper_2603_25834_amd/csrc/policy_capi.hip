// policy_capi.hip -- C-ABI of the PPO actor-critic (declared in include/aslam.h).
//
// The handle owns the minibatch workspaces (activations recomputed per
// minibatch, gradient partial sums), allocated once at create time for
// `max_batch` samples; forward and backward allocate nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "aslam.h"
#include "policy_kernels.h"
#include "conv_fused.h"
#include "gru_kernels.h"

using namespace aslam;
using namespace aslam::pol;

// Error messages of the policy calls are reported through aslam_last_error.
namespace aslam {
void set_last_error(const std::string& msg);
}  // namespace aslam

namespace {
int pfail(int code, const std::string& m) {
  aslam::set_last_error(m);
  return code;
}
}  // namespace

struct aslam_policy {
  aslam_policy_config cfg{};
  Offsets off{};
  int64_t max_b = 0;
  uint16_t *x = nullptr;   // FC1 input [B][k1p]: conv features (8192) | scan | state | zero pad, BF16
  uint16_t *h1 = nullptr, *dz2 = nullptr, *dz1 = nullptr, *dz2c = nullptr;
  float *z2 = nullptr, *part = nullptr, *hpart = nullptr;
  uint16_t *w1b = nullptr, *w1t = nullptr, *w2b = nullptr, *w2t = nullptr;   // BF16 weight copies
  uint4* cfrag = nullptr;   // the encoder's weight fragments (k_conv_frags, k_conv_bwd_frags)
  int32_t k1p = 0;   // FC1 input width padded to a multiple of 8
  // split-precision forward (config precision 1): the lo parts of the FC1 input rows, of h1 and of the
  // FC weights (the encoder's lo fragments sit in cfrag from kConvLoFrag on)
  bool prec = false;
  uint16_t *x_lo = nullptr, *h1_lo = nullptr, *w1b_lo = nullptr, *w2b_lo = nullptr;
  int64_t part_floats = 0;
  bool prepared = false;   // w1b / w2b hold the weights of some params (the caller tracks which)
  // recurrent handle: the GRU's weight copies and the sequence minibatch's buffers
  bool rec = false;
  uint16_t *wihb = nullptr, *whhb = nullptr, *wiht = nullptr, *whht = nullptr;
  float *hst = nullptr, *g_r = nullptr, *g_z = nullptr, *g_n = nullptr, *g_ghn = nullptr, *hp_used = nullptr;
  float *dh_head = nullptr, *dh_buf = nullptr;
  uint16_t *hp_bf = nullptr, *dgi = nullptr, *dgh = nullptr;
  int32_t* rows = nullptr;
};

namespace {

constexpr int kConvGrid = 768;     // encoder forward: the resident workgroups (three per CU, LDS-bound), each looping over samples
constexpr int kConvGridPrec = 256; // the split-precision encoder forward holds twice the LDS: one per CU
constexpr int kConvFragsAll = kConvLoFrag + kConvFrags;   // forward, backward phase and lo fragments
constexpr int kConvBwdGrid = 256;  // encoder backward: one 8-wave workgroup per CU (LDS-bound)
constexpr int64_t kFc1Splits = 12, kFc2Splits = 64;
constexpr int kFc1MinBlocks = 512;   // FC1 forward: resident workgroups (two per CU) that its K splits fill

int64_t splits_for(int64_t K, int64_t min_chunk, int64_t max_splits) {
  return std::max<int64_t>(1, std::min<int64_t>(max_splits, K / min_chunk));
}

// K splits of a split-K GEMM with `tiles` output tiles: the count that minimises (rounds of
// `slots` resident workgroups) x (BK steps per workgroup), the smaller on ties.
int64_t splits_balanced(int64_t K, int BK, int64_t tiles, int64_t slots, int64_t max_splits) {
  int64_t best = 1, best_cost = -1;
  for (int64_t s = 1; s <= max_splits; ++s) {
    const int64_t rounds = (tiles * s + slots - 1) / slots;
    const int64_t steps = (K + s * BK - 1) / (s * BK);
    const int64_t cost = rounds * steps;
    if (best_cost < 0 || cost < best_cost) { best = s; best_cost = cost; }
  }
  return best;
}

// Number of K slices gemm::run launches for `splits` requested splits (chunks rounded up to BK).
int slices_used(int64_t K, int64_t splits, int BK) {
  int64_t chunk = (K + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  return (int)((K + chunk - 1) / chunk);
}

int64_t part_need(const aslam_policy* p) {
  const int64_t k1 = p->off.k1;
  int64_t need = kFc1Splits * 256 * k1;                      // FC1 weight partials
  need = std::max<int64_t>(need, kFc2Splits * kHid * kHid);   // FC2 weight partials
  if (p->rec) need = std::max<int64_t>(need, (int64_t)kFc2Splits * kGates * kHid);   // GRU weight partials
  if (p->rec) need = std::max<int64_t>(need, (int64_t)kBiasBlocks * kGates);         // GRU bias partials
  need = std::max<int64_t>(need, (int64_t)kConvBwdGrid * kConvPart);   // encoder backward partials
  need = std::max<int64_t>(need, (int64_t)kBiasBlocks * 256);
  need = std::max<int64_t>(need, (int64_t)kFc1MinBlocks * 64 * kHid);   // FC1 forward split-K: S * B <= 512 * 64
  if (p->prec)   // the three products of a split FC1, over z (S * B <= 512 * 64 each)
    need = std::max<int64_t>(need, 3 * (int64_t)kFc1MinBlocks * 64 * kHid);
  return need;
}

#define PCHK(e)                                                      \
  do {                                                               \
    hipError_t e_ = (e);                                             \
    if (e_ != hipSuccess) return pfail(ASL_EHIP, hipGetErrorString(e_)); \
  } while (0)

// The MLP policy's weight preparation in one launch, the jobs taken by workgroup ranges in this order:
// kPrepW1 workgroups convert W1 (and its lo part), kPrepW2 convert W2, then with `transposed` the
// 32 x 32 tiles of W1's conv-feature columns and of W2 transposed, and the last workgroup forms the
// encoder's fragments (the forward's, with PREC their lo parts, with `transposed` the backward's phase
// fragments).  Each job does what its own kernel (k_convert_bf16, k_transpose_bf16, k_conv_frags,
// k_conv_bwd_frags) does, value for value; one launch instead of up to seven per parameter update.
constexpr int kPrepW1 = 1024, kPrepW2 = 256;
constexpr int kPrepT1 = (kFeat / 32) * (kHid / 32), kPrepT2 = (kHid / 32) * (kHid / 32);

__global__ __launch_bounds__(256) void k_prep_mlp(const float* __restrict__ prm, Offsets o, int k1p,
                                                  uint16_t* w1b, uint16_t* w1b_lo, uint16_t* w2b, uint16_t* w2b_lo,
                                                  uint16_t* w1t, uint16_t* w2t, uint4* cfrag, int transposed) {
  __shared__ float tile[32][33];
  int b = blockIdx.x;
  if (b < kPrepW1) {
    convert_bf16_part(prm + o.f1w, o.k1, kHid, o.k1, w1b, k1p, w1b_lo, b, kPrepW1);
    return;
  }
  b -= kPrepW1;
  if (b < kPrepW2) {
    convert_bf16_part(prm + o.f2w, kHid, kHid, kHid, w2b, kHid, w2b_lo, b, kPrepW2);
    return;
  }
  b -= kPrepW2;
  if (transposed) {
    if (b < kPrepT1) {
      transpose_bf16_tile(prm + o.f1w, o.k1, kHid, kFeat, w1t, kHid, tile, b % (kFeat / 32), b / (kFeat / 32));
      return;
    }
    b -= kPrepT1;
    if (b < kPrepT2) {
      transpose_bf16_tile(prm + o.f2w, kHid, kHid, kHid, w2t, kHid, tile, b % (kHid / 32), b / (kHid / 32));
      return;
    }
  }
  for (int t = threadIdx.x; t < 64 * kConvFrags; t += 256) conv_frag_elem<false>(prm, o, cfrag, t);
  if (w1b_lo)
    for (int t = threadIdx.x; t < 64 * kConvFrags; t += 256) conv_frag_elem<true>(prm, o, cfrag + 64 * kConvLoFrag, t);
  if (transposed)
    for (int t = threadIdx.x; t < 64 * kConvPhaseFrags; t += 256) conv_bwd_frag_elem(prm, o, cfrag, t);
}

// BF16 copies of W1 (rows padded to k1p) and W2 and the encoder's weight fragments that the forward
// reads; with `transposed` also what only the backward reads (the transposes for the input gradients,
// the encoder backward's phase fragments).
int convert_weights(aslam_policy* P, const float* prm, hipStream_t st, bool transposed) {
  const Offsets& o = P->off;
  if (P->rec) {
    k_convert_bf16<<<1024, 256, 0, st>>>(prm + o.f1w, o.k1, kHid, o.k1, P->w1b, P->k1p, P->prec ? P->w1b_lo : nullptr);
    PCHK(hipGetLastError());
    k_convert_bf16<<<768, 256, 0, st>>>(prm + o.gih, kHid, kGates, kHid, P->wihb, kHid);
    PCHK(hipGetLastError());
    k_convert_bf16<<<768, 256, 0, st>>>(prm + o.ghh, kHid, kGates, kHid, P->whhb, kHid);
    PCHK(hipGetLastError());
    k_conv_frags<<<1, 64 * kConvFrags, 0, st>>>(prm, o, P->cfrag);
    PCHK(hipGetLastError());
    if (transposed) {
      k_conv_bwd_frags<<<1, 64 * kConvPhaseFrags, 0, st>>>(prm, o, P->cfrag);
      PCHK(hipGetLastError());
      k_transpose_bf16<<<dim3(kFeat / 32, kHid / 32), 256, 0, st>>>(prm + o.f1w, o.k1, kHid, kFeat, P->w1t, kHid);
      PCHK(hipGetLastError());
      k_transpose_bf16<<<dim3(kHid / 32, kGates / 32), 256, 0, st>>>(prm + o.gih, kHid, kGates, kHid, P->wiht, kGates);
      PCHK(hipGetLastError());
      k_transpose_bf16<<<dim3(kHid / 32, kGates / 32), 256, 0, st>>>(prm + o.ghh, kHid, kGates, kHid, P->whht, kGates);
      PCHK(hipGetLastError());
    }
    P->prepared = true;
    return ASL_OK;
  }
  const int blocks = kPrepW1 + kPrepW2 + (transposed ? kPrepT1 + kPrepT2 : 0) + 1;
  k_prep_mlp<<<blocks, 256, 0, st>>>(prm, o, P->k1p, P->w1b, P->prec ? P->w1b_lo : nullptr, P->w2b,
                                     P->prec ? P->w2b_lo : nullptr, P->w1t, P->w2t, P->cfrag, transposed ? 1 : 0);
  PCHK(hipGetLastError());
  P->prepared = true;
  return ASL_OK;
}

// Encoder (conv features and the scan / state tail into the FC1 input x) and FC1.  Small batches
// split K so that the launch fills the chip: then *S_used split-K slices are left in P->part;
// otherwise FC1 writes h1 = bf16(relu(. + b1)) and *S_used = 0.
int encode_fc1(aslam_policy* P, const float* prm, const int16_t* crop, const float* scan, const float* state,
               const int32_t* rows, int B, hipStream_t st, int* S_used) {
  const Offsets& o = P->off;
  if (P->prec)
    k_conv_fwd<true, 512><<<std::min(B, kConvGridPrec), 512, 0, st>>>(prm, o, P->cfrag, crop, scan, state,
                                                                      P->cfg.n_scan, rows, P->x, P->x_lo, P->k1p, B);
  else
    k_conv_fwd<false><<<std::min(B, kConvGrid), 256, 0, st>>>(prm, o, P->cfrag, crop, scan, state, P->cfg.n_scan,
                                                              rows, P->x, nullptr, P->k1p, B);
  PCHK(hipGetLastError());
  // FC1: [B x k1p] x [k1p x 256] (both operands zero-padded from k1 to k1p)
  const int K1 = P->k1p;
  const LdBF16K xa{P->x, K1, B, K1};
  const LdBF16K wa{P->w1b, K1, kHid, K1};
  // as many K splits as keep the grid within one round of kFc1MinBlocks resident workgroups; with the
  // three split-precision products and few row tiles (a rollout step) a third of that: the products
  // fill the round themselves, and more slices would only add partial-sum traffic (at 750 rows, 32
  // splits of 3 products wrote and re-read 74 MB of partial sums per call)
  const int tiles = ((B + 127) / 128) * (kHid / 128);
  int S = std::max(1, std::min(32, kFc1MinBlocks / tiles));
  if (P->prec && tiles < 32) S = std::max(1, std::min(32, kFc1MinBlocks / (3 * tiles)));
  if (P->prec) {
    // x_hi W_hi, x_hi W_lo and x_lo W_hi, each split S ways, into consecutive groups of slices (one
    // launch, the products over z: product 1 reads W's lo part, product 2 x's)
    const int nz = slices_used(K1, S, 64);
    const int64_t slice = (int64_t)B * kHid;
    PCHK((gemm::run<128, 128, 64, 2, 2>(gemm::HiLo<LdBF16K>{xa, LdBF16K{P->x_lo, K1, B, K1}, 4u},
                                         gemm::HiLo<LdBF16K>{wa, LdBF16K{P->w1b_lo, K1, kHid, K1}, 2u},
                                         EpiPartial{P->part, kHid, slice}, B, kHid, K1, S, st, 3)));
    *S_used = 3 * nz;
  } else if (S == 1) {
    PCHK((gemm::run<128, 128, 64, 2, 2>(xa, wa, EpiBiasReluBF16{P->h1, prm + o.f1b, kHid}, B, kHid, K1, 1, st)));
    *S_used = 0;
  } else {
    *S_used = slices_used(K1, S, 64);
    PCHK((gemm::run<128, 128, 64, 2, 2>(xa, wa, EpiPartial{P->part, kHid, (int64_t)B * kHid}, B, kHid, K1, S,
                                         st)));
  }
  return ASL_OK;
}

// The backward's forward: every weight copy, the encoder, FC1 to h1 and the FC2 pre-activation z2 (FP32).
int forward_core(aslam_policy* P, const float* prm, const int16_t* crop, const float* scan, const float* state,
                 const int32_t* rows, int B, hipStream_t st) {
  const Offsets& o = P->off;
  int rc = convert_weights(P, prm, st, true);
  if (rc) return rc;
  int S = 0;
  rc = encode_fc1(P, prm, crop, scan, state, rows, B, st, &S);
  if (rc) return rc;
  if (S > 0) {
    const int64_t groups = (int64_t)B * (kHid / 8);
    k_reduce_bias_relu_bf16<<<(int)std::min<int64_t>(4096, (groups + 255) / 256), 256, 0, st>>>(
        P->part, S, B, kHid, prm + o.f1b, P->h1, kHid, P->prec ? P->h1_lo : nullptr);
    PCHK(hipGetLastError());
  }
  const LdBF16K ha{P->h1, kHid, B, kHid}, wb{P->w2b, kHid, kHid, kHid};
  if (P->prec) {
    // z2 = h1_hi W2_hi + h1_hi W2_lo + h1_lo W2_hi + b2, the three products in one accumulator
    PCHK((gemm::run<128, 128, 64, 2, 2>(gemm::HiLo<LdBF16K>{ha, LdBF16K{P->h1_lo, kHid, B, kHid}, 4u},
                                       gemm::HiLo<LdBF16K>{wb, LdBF16K{P->w2b_lo, kHid, kHid, kHid}, 2u},
                                       EpiBiasF32{P->z2, prm + o.f2b, kHid}, B, kHid, kHid, 1, st, 3, true)));
    return ASL_OK;
  }
  PCHK((gemm::run<128, 128, 64, 2, 2>(ha, wb, EpiBiasF32{P->z2, prm + o.f2b, kHid}, B, kHid, kHid, 1, st)));
  return ASL_OK;
}

// Forward-only pass: encoder, FC1, then the fused tail (FC2, heads and, with eps, the sample).
int act_core(aslam_policy* P, const float* prm, bool prepared, const int16_t* crop, const float* scan,
             const float* state, int B, bool sample, ActDraws eps, float* mu, float* value, float* act,
             float* logp, hipStream_t st) {
  if (!prepared) {
    int rc = convert_weights(P, prm, st, false);
    if (rc) return rc;
  }
  int S = 0;
  int rc = encode_fc1(P, prm, crop, scan, state, nullptr, B, st, &S);
  if (rc) return rc;
  if (S > 8) {
    // many split-K slices: their sum is spread over the chip first (the tail kernel has B / 16 workgroups)
    const int64_t groups = (int64_t)B * (kHid / 8);
    k_reduce_bias_relu_bf16_q<<<(unsigned)((groups + 63) / 64), 256, 0, st>>>(P->part, S, B, kHid, prm + P->off.f1b,
                                                                              P->h1, kHid, P->prec ? P->h1_lo : nullptr);
    PCHK(hipGetLastError());
    S = 0;
  }
  const int tail_blocks = (B + kTailRows - 1) / kTailRows;
  if (P->prec)
    k_fwd_tail<true><<<tail_blocks, 256, 0, st>>>(prm, P->off, P->part, S, P->h1, P->h1_lo, P->w2b, P->w2b_lo, B, mu,
                                                  value, sample, eps, act, logp);
  else
    k_fwd_tail<false><<<tail_blocks, 256, 0, st>>>(prm, P->off, P->part, S, P->h1, nullptr, P->w2b, nullptr, B, mu,
                                                   value, sample, eps, act, logp);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int backward_fc1_encoder(aslam_policy* P, const float* params, const int16_t* crop, const int32_t* rows, int B,
                         float* grads, hipStream_t st);

}  // namespace

extern "C" {

int64_t aslam_policy_num_params(int32_t n_scan) {
  if (n_scan < 0) return -1;
  return offsets(n_scan).total;
}

int aslam_policy_create(const aslam_policy_config* cfg, aslam_policy** out) {
  if (!cfg || !out) return pfail(ASL_EINVAL, "config or out is NULL");
  *out = nullptr;
  if (cfg->n_scan < 1 || cfg->n_scan > 4096) return pfail(ASL_EINVAL, "n_scan must be in [1, 4096]");
  if (cfg->max_batch < 1 || cfg->max_batch > (1 << 20)) return pfail(ASL_EINVAL, "max_batch must be in [1, 2^20]");
  if (cfg->recurrent != 0 && cfg->recurrent != 1) return pfail(ASL_EINVAL, "recurrent must be 0 or 1");
  if (cfg->precision != 0 && cfg->precision != 1) return pfail(ASL_EINVAL, "precision must be 0 or 1");
  if (cfg->precision == 1 && cfg->recurrent == 1)
    return pfail(ASL_ENOTIMPL, "the split-precision forward is built for the feed-forward policy only");
  aslam_policy* p = new (std::nothrow) aslam_policy();
  if (!p) return pfail(ASL_ENOMEM, "host allocation failed");
  p->cfg = *cfg;
  p->rec = cfg->recurrent == 1;
  p->prec = cfg->precision == 1;
  p->off = offsets(cfg->n_scan, p->rec);
  p->max_b = cfg->max_batch;
  const int64_t Bm = p->max_b;
  p->part_floats = part_need(p);
  p->k1p = (p->off.k1 + 7) / 8 * 8;
  struct A { void** ptr; size_t bytes; } al[] = {
      {(void**)&p->x, 2 * (size_t)Bm * ((p->off.k1 + 7) / 8 * 8)},  {(void**)&p->h1, 2 * (size_t)Bm * kHid},
      {(void**)&p->dz2, 2 * (size_t)Bm * kHid},  {(void**)&p->dz1, 2 * (size_t)Bm * kHid},
      {(void**)&p->dz2c, 2 * (size_t)Bm * kFeat}, {(void**)&p->z2, 4 * (size_t)Bm * kHid},
      {(void**)&p->part, 4 * (size_t)p->part_floats},
      {(void**)&p->hpart, 4 * (size_t)((Bm + kHeadRows - 1) / kHeadRows) * kHeadPart},
      {(void**)&p->w1b, 2 * (size_t)kHid * ((p->off.k1 + 7) / 8 * 8)}, {(void**)&p->w1t, 2 * (size_t)kFeat * kHid},
      {(void**)&p->w2b, 2 * (size_t)kHid * kHid},                        {(void**)&p->w2t, 2 * (size_t)kHid * kHid},
      {(void**)&p->cfrag, sizeof(uint4) * 64 * kConvFragsAll},
  };
  for (auto& a : al) {
    if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
      aslam_policy_destroy(p);
      return pfail(ASL_ENOMEM, "hipMalloc of policy workspace failed");
    }
  }
  if (p->prec) {
    struct A pl[] = {
        {(void**)&p->x_lo, 2 * (size_t)Bm * p->k1p}, {(void**)&p->h1_lo, 2 * (size_t)Bm * kHid},
        {(void**)&p->w1b_lo, 2 * (size_t)kHid * p->k1p}, {(void**)&p->w2b_lo, 2 * (size_t)kHid * kHid},
    };
    for (auto& a : pl) {
      if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
        aslam_policy_destroy(p);
        return pfail(ASL_ENOMEM, "hipMalloc of policy workspace failed");
      }
    }
  }
  if (p->rec) {
    const size_t f = 4 * (size_t)Bm * kHid, h = 2 * (size_t)Bm * kHid, g = 2 * (size_t)Bm * kGates;
    const size_t w = 2 * (size_t)kGates * kHid;
    struct A rl[] = {
        {(void**)&p->wihb, w}, {(void**)&p->whhb, w}, {(void**)&p->wiht, w}, {(void**)&p->whht, w},
        {(void**)&p->hst, f}, {(void**)&p->g_r, f}, {(void**)&p->g_z, f}, {(void**)&p->g_n, f},
        {(void**)&p->g_ghn, f}, {(void**)&p->hp_used, f}, {(void**)&p->dh_head, f}, {(void**)&p->dh_buf, 2 * f},
        {(void**)&p->hp_bf, h}, {(void**)&p->dgi, g}, {(void**)&p->dgh, g},
        {(void**)&p->rows, 4 * (size_t)Bm},
    };
    for (auto& a : rl) {
      if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
        aslam_policy_destroy(p);
        return pfail(ASL_ENOMEM, "hipMalloc of policy workspace failed");
      }
    }
  }
  *out = p;
  return ASL_OK;
}

int64_t aslam_policy_param_count(const aslam_policy_config* cfg) {
  if (!cfg || cfg->n_scan < 0 || (cfg->recurrent != 0 && cfg->recurrent != 1)) return -1;
  return offsets(cfg->n_scan, cfg->recurrent == 1).total;
}

int aslam_policy_destroy(aslam_policy* p) {
  if (!p) return pfail(ASL_EINVAL, "policy is NULL");
  void* ptrs[] = {p->x, p->h1, p->dz2, p->dz1, p->dz2c, p->z2, p->part, p->hpart,
                  p->w1b, p->w1t, p->w2b, p->w2t, p->cfrag,
                  p->wihb, p->whhb, p->wiht, p->whht, p->hst, p->g_r, p->g_z, p->g_n, p->g_ghn, p->hp_used,
                  p->dh_head, p->dh_buf, p->hp_bf, p->dgi, p->dgh, p->rows, p->x_lo, p->h1_lo, p->w1b_lo,
                  p->w2b_lo};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
  return ASL_OK;
}

int aslam_policy_forward(aslam_policy* P, const float* params, const int16_t* crop, const float* scan,
                         const float* state, int32_t batch, float* mu, float* value, aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !mu || !value) return pfail(ASL_EINVAL, "null argument");
  if (batch < 1 || batch > P->max_b) return pfail(ASL_EINVAL, "batch must be in [1, max_batch]");
  if (P->rec) return pfail(ASL_EINVAL, "recurrent policy: use aslam_policy_act_rnn");
  return act_core(P, params, false, crop, scan, state, batch, false, ActDraws{nullptr, 0, 0}, mu, value, nullptr,
                  nullptr, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------------------ forward without allocation
//
// aslam_policy_forward_noalloc keeps what the forward stages between its kernels (the BF16 weight
// copies, the encoder's weight fragments, the FC1 input rows, FC1's split-K partial sums and the
// hidden rows) in one file-scope device array instead of a handle's allocations.  Its layout is fixed
// for the largest scan and batch it accepts.  Host code never passes the array's name to a kernel:
// the device address is looked up once per device with hipGetSymbolAddress and kept.
namespace {
constexpr int64_t kNoAllocMaxScan = 720;
constexpr int64_t kNoAllocMaxBatch = 256;
constexpr int64_t kNoAllocK1p = (kFeat + kNoAllocMaxScan + 12 + 7) / 8 * 8;
constexpr int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }
constexpr int64_t kNaW1b = 0;
constexpr int64_t kNaW2b = kNaW1b + align256(2 * kHid * kNoAllocK1p);
constexpr int64_t kNaFrag = kNaW2b + align256(2 * kHid * kHid);
constexpr int64_t kNaX = kNaFrag + align256(16 * 64 * (kConvFrags + kConvPhaseFrags));
constexpr int64_t kNaH1 = kNaX + align256(2 * kNoAllocMaxBatch * kNoAllocK1p);
constexpr int64_t kNaPart = kNaH1 + align256(2 * kNoAllocMaxBatch * kHid);
constexpr int64_t kNaBytes = kNaPart + align256(4 * 32 * kNoAllocMaxBatch * kHid);   // at most 32 K slices
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_ptr;   // per device: the array's device address, looked up once

int scratch_for_current_device(unsigned char** out) {
  int dev = 0;
  PCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return pfail(ASL_EHIP, "hipGetSymbolAddress returned no address for the forward's scratch");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ASL_OK;
}

}  // namespace

extern "C" {

int64_t aslam_policy_noalloc_limits(int32_t* max_scan, int32_t* max_batch) {
  if (max_scan) *max_scan = (int32_t)kNoAllocMaxScan;
  if (max_batch) *max_batch = (int32_t)kNoAllocMaxBatch;
  return kNaBytes;
}

int aslam_policy_forward_noalloc(const float* params, int32_t n_scan, const int16_t* crop, const float* scan,
                                 const float* state, int32_t batch, float* mu, float* value, aslam_stream_t stream) {
  if (!params || !crop || !scan || !state || !mu || !value) return pfail(ASL_EINVAL, "null argument");
  if (n_scan < 1 || n_scan > kNoAllocMaxScan)
    return pfail(ASL_EINVAL, "forward_noalloc: n_scan must be in [1, " + std::to_string(kNoAllocMaxScan) + "]");
  if (batch < 1 || batch > kNoAllocMaxBatch)
    return pfail(ASL_EINVAL, "forward_noalloc: batch must be in [1, " + std::to_string(kNoAllocMaxBatch) +
                                 "] (the scratch array is sized for that)");
  unsigned char* base = nullptr;
  int rc = scratch_for_current_device(&base);
  if (rc) return rc;
  // a handle on the stack whose workspaces are views of the scratch array: the same kernels as
  // aslam_policy_forward, in the same order, with the same split of FC1's K
  aslam_policy P{};
  P.cfg.n_scan = n_scan;
  P.cfg.max_batch = batch;
  P.off = offsets(n_scan);
  P.max_b = batch;
  P.k1p = (P.off.k1 + 7) / 8 * 8;
  P.w1b = reinterpret_cast<uint16_t*>(base + kNaW1b);
  P.w2b = reinterpret_cast<uint16_t*>(base + kNaW2b);
  P.cfrag = reinterpret_cast<uint4*>(base + kNaFrag);
  P.x = reinterpret_cast<uint16_t*>(base + kNaX);
  P.h1 = reinterpret_cast<uint16_t*>(base + kNaH1);
  P.part = reinterpret_cast<float*>(base + kNaPart);
  return act_core(&P, params, false, crop, scan, state, batch, false, ActDraws{nullptr, 0, 0}, mu, value, nullptr,
                  nullptr, (hipStream_t)stream);
}

int aslam_policy_prepare(aslam_policy* P, const float* params, aslam_stream_t stream) {
  if (!P || !params) return pfail(ASL_EINVAL, "null argument");
  return convert_weights(P, params, (hipStream_t)stream, false);
}

int aslam_policy_act(aslam_policy* P, const float* params, int32_t prepared, const int16_t* crop, const float* scan,
                     const float* state, int32_t batch, const float* eps, uint64_t seed, uint64_t counter, float* mu,
                     float* value, float* act, float* logp, aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !value || !act || !logp)
    return pfail(ASL_EINVAL, "null argument");
  if (batch < 1 || batch > P->max_b) return pfail(ASL_EINVAL, "batch must be in [1, max_batch]");
  if (P->rec) return pfail(ASL_EINVAL, "recurrent policy: use aslam_policy_act_rnn");
  if (prepared && !P->prepared) return pfail(ASL_ESTATE, "act with prepared = 1 before any prepare");
  return act_core(P, params, prepared != 0, crop, scan, state, batch, true, ActDraws{eps, seed, counter}, mu, value,
                  act, logp, (hipStream_t)stream);
}

int aslam_policy_backward(aslam_policy* P, const float* params, const int16_t* crop, const float* scan,
                          const float* state, int32_t batch, const float* act, const float* old_logp,
                          const float* adv, const float* ret, float* grads, float* loss, aslam_stream_t stream) {
  return aslam_policy_backward_rows(P, params, crop, scan, state, nullptr, batch, act, old_logp, adv, ret, grads,
                                    loss, stream);
}

int aslam_policy_backward_rows(aslam_policy* P, const float* params, const int16_t* crop, const float* scan,
                               const float* state, const int32_t* rows, int32_t batch, const float* act,
                               const float* old_logp, const float* adv, const float* ret, float* grads, float* loss,
                               aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !act || !old_logp || !adv || !ret || !grads || !loss)
    return pfail(ASL_EINVAL, "null argument");
  if (batch < 1 || batch > P->max_b) return pfail(ASL_EINVAL, "batch must be in [1, max_batch]");
  if (P->rec) return pfail(ASL_EINVAL, "recurrent policy: use aslam_policy_backward_seq");
  hipStream_t st = (hipStream_t)stream;
  const Offsets& o = P->off;
  const int B = batch;
  int rc = forward_core(P, params, crop, scan, state, rows, B, st);
  if (rc) return rc;
  // heads + loss -> dz2, head / fc2-bias / log-std partial sums
  const int nb = (B + kHeadRows - 1) / kHeadRows;
  LossCoef lc{P->cfg.clip_eps, P->cfg.c_value, P->cfg.c_entropy, 1.0f / (float)B};
  k_heads<true><<<nb, 256, 0, st>>>(params, o, P->z2, B, nullptr, nullptr, act, old_logp, adv, ret, rows, lc, P->dz2,
                                    P->hpart);
  PCHK(hipGetLastError());
  PCHK(launch_reduce_heads(P->hpart, nb, params, o, grads, loss, P->cfg.c_value, P->cfg.c_entropy, st));
  float* part = P->part;
  // FC2 weight: dW2[out][in] = sum_b dz2[b][out] h1[b][in]
  {
    const int64_t S = splits_for(B, 256, kFc2Splits);
    const int S_used = slices_used(B, S, 64);
    PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16I{P->dz2, kHid, kHid, B}, LdBF16I{P->h1, kHid, kHid, B},
                                       EpiPartial{part, kHid, (int64_t)kHid * kHid}, kHid, kHid, B, (int)S, st)));
    PCHK(launch_reduce(part, S_used, (int64_t)kHid * kHid, grads + o.f2w, 0, (int64_t)kHid * kHid, st));
  }
  // dh1 -> dz1 = (dz2 W2) * [h1 > 0]
  PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16K{P->dz2, kHid, B, kHid}, LdBF16K{P->w2t, kHid, kHid, kHid},
                                     EpiReluGradBF16{P->dz1, P->h1, kHid, kHid}, B, kHid, kHid, 1, st)));
  return backward_fc1_encoder(P, params, crop, rows, B, grads, st);
}

}  // extern "C"

namespace {

// Everything below the FC1 output gradient dz1 (BF16, already masked by FC1's ReLU): the FC1 bias and
// weight gradients, the conv-feature gradient and the encoder backward.
int backward_fc1_encoder(aslam_policy* P, const float* params, const int16_t* crop, const int32_t* rows, int B,
                         float* grads, hipStream_t st) {
  const Offsets& o = P->off;
  float* part = P->part;
  // FC1 bias
  k_bias_rows<<<kBiasBlocks, 256, 0, st>>>(P->dz1, B, kHid, part);
  PCHK(hipGetLastError());
  PCHK(launch_reduce(part, kBiasBlocks, kHid, grads + o.f1b, 0, kHid, st));
  // FC1 weight: dW1[out][k] = sum_b dz1[b][out] X[b][k]
  {
    const int64_t S = splits_balanced(B, 64, 2 * (int64_t)((o.k1 + 127) / 128), 512, kFc1Splits);
    const int S_used = slices_used(B, S, 64);
    PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16I{P->dz1, kHid, kHid, B}, LdBF16I{P->x, P->k1p, o.k1, B},
                                       EpiPartial{part, o.k1, (int64_t)kHid * o.k1}, kHid, o.k1, B, (int)S, st)));
    PCHK(launch_reduce(part, S_used, (int64_t)kHid * o.k1, grads + o.f1w, 0, (int64_t)kHid * o.k1, st));
  }
  // dA2 -> dz2c = (dz1 W1[:, :8192]) * [a2 > 0]
  PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16K{P->dz1, kHid, B, kHid}, LdBF16K{P->w1t, kHid, kFeat, kHid},
                                     EpiReluGradBF16{P->dz2c, P->x, kFeat, P->k1p}, B, kFeat, kHid, 1, st)));
  // encoder: conv2 / conv1 weight and bias gradients in one pass over the minibatch
  {
    const int grid = std::min(B, kConvBwdGrid);
    if (P->prec)
      k_conv_bwd<true><<<grid, kBwdThreads, 0, st>>>(params, o, P->cfrag, crop, rows, P->dz2c, B, part);
    else
      k_conv_bwd<false><<<grid, kBwdThreads, 0, st>>>(params, o, P->cfrag, crop, rows, P->dz2c, B, part);
    PCHK(hipGetLastError());
    // the four gradient blocks of the encoder's partials in one reduction
    const ReduceSegs sg{{kConvPartW2, kConvPartW1, kC1, kC2}, {1, 2, 0, 0}, {o.c2w, o.c1w, o.c1b, o.c2b}};
    PCHK(launch_reduce_segs(part, grid, grads, sg, kConvPart, st));
  }
  return ASL_OK;
}

}  // namespace

extern "C" {

int aslam_policy_sample(aslam_policy* P, const float* params, const float* mu, const float* eps, uint64_t seed,
                        uint64_t counter, int32_t batch, float* act, float* logp, aslam_stream_t stream) {
  if (!P || !params || !mu || !act || !logp) return pfail(ASL_EINVAL, "null argument");
  if (batch < 1) return pfail(ASL_EINVAL, "batch must be >= 1");
  k_sample<<<(batch + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, P->off, mu, ActDraws{eps, seed, counter},
                                                                  batch, act, logp);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int64_t aslam_permutation_work_bytes(int32_t n) {
  if (n <= 0) return 0;
  return (int64_t)4 << (2 * rng::perm_half_bits(n));
}

int aslam_permutation(int32_t n, uint64_t seed, uint64_t counter, int32_t* out, void* work, int64_t work_bytes,
                      aslam_stream_t stream) {
  if (n < 0) return pfail(ASL_EINVAL, "n must be >= 0");
  if (n == 0) return ASL_OK;
  if (!out) return pfail(ASL_EINVAL, "null argument");
  const int h = rng::perm_half_bits(n);
  hipStream_t st = (hipStream_t)stream;
  if (!work) {
    k_permutation<<<(n + 255) / 256, 256, 0, st>>>(n, h, seed, counter, out);
  } else {
    const int64_t dom = (int64_t)1 << (2 * h);
    if (work_bytes < 4 * dom) return pfail(ASL_EINVAL, "work_bytes below aslam_permutation_work_bytes(n)");
    if ((uintptr_t)work & 3) return pfail(ASL_EINVAL, "work must be 4-byte aligned");
    uint32_t* tab = static_cast<uint32_t*>(work);
    k_feistel_table<<<(unsigned)((dom + 255) / 256), 256, 0, st>>>(h, seed, counter, tab);
    PCHK(hipGetLastError());
    k_permutation_walk<<<(n + 255) / 256, 256, 0, st>>>(n, tab, out);
  }
  PCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_gather_rows(const void* src, int64_t row_bytes, const int32_t* idx, int32_t n, void* dst,
                      aslam_stream_t stream) {
  if (!src || !idx || !dst) return pfail(ASL_EINVAL, "null argument");
  if (n < 0 || row_bytes < 4 || (row_bytes & 3)) return pfail(ASL_EINVAL, "row_bytes must be a positive multiple of 4");
  if (((uintptr_t)src & 3) || ((uintptr_t)dst & 3)) return pfail(ASL_EINVAL, "src and dst must be 4-byte aligned");
  if (n == 0) return ASL_OK;
  const int vec = ((row_bytes & 15) == 0 && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0) ? 1 : 0;
  const int64_t items = vec ? (int64_t)n * (row_bytes >> 4) : (int64_t)n * (row_bytes >> 2);
  const int blocks = (int)std::min<int64_t>(8192, (items + 255) / 256);
  k_gather_rows<<<blocks, 256, 0, (hipStream_t)stream>>>(static_cast<const uint32_t*>(src), row_bytes >> 2, idx, n,
                                                         static_cast<uint32_t*>(dst), vec);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_gae(const float* rewards, const float* values, const uint8_t* dones, const float* last_value, int32_t T,
              int32_t N, float gamma, float lam, float* adv, float* ret, aslam_stream_t stream) {
  if (!rewards || !values || !dones || !last_value || !adv || !ret) return pfail(ASL_EINVAL, "null argument");
  if (T < 1 || N < 1) return pfail(ASL_EINVAL, "T and N must be >= 1");
  k_gae<<<(N + 255) / 256, 256, 0, (hipStream_t)stream>>>(rewards, values, dones, last_value, T, N, gamma, lam,
                                                           adv, ret);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_adam(float* params, const float* grads, float* m, float* v, int64_t n, int32_t step, float lr,
               float beta1, float beta2, float eps, aslam_stream_t stream) {
  if (!params || !grads || !m || !v) return pfail(ASL_EINVAL, "null argument");
  if (n < 1 || step < 1) return pfail(ASL_EINVAL, "n and step must be >= 1");
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  k_adam<<<blocks, 256, 0, (hipStream_t)stream>>>(params, grads, m, v, n, lr, beta1, beta2, eps, bc1, bc2);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_policy_act_rnn(aslam_policy* P, const float* params, int32_t prepared, const int16_t* crop,
                         const float* scan, const float* state, int32_t batch, const float* h_in, const uint8_t* first,
                         const float* eps, uint64_t seed, uint64_t counter, float* mu, float* value, float* act,
                         float* logp, float* h_out, aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !h_in || !value || !act || !logp || !h_out)
    return pfail(ASL_EINVAL, "null argument");
  if (!P->rec) return pfail(ASL_EINVAL, "feed-forward policy: use aslam_policy_act");
  if (batch < 1 || batch > P->max_b) return pfail(ASL_EINVAL, "batch must be in [1, max_batch]");
  if (prepared && !P->prepared) return pfail(ASL_ESTATE, "act_rnn with prepared = 1 before any prepare");
  hipStream_t st = (hipStream_t)stream;
  if (!prepared) {
    int rc = convert_weights(P, params, st, false);
    if (rc) return rc;
  }
  int S = 0;
  int rc = encode_fc1(P, params, crop, scan, state, nullptr, batch, st, &S);
  if (rc) return rc;
  if (S > 0) {   // the split-K slices summed over the whole chip first (h1 = bf16(relu(. + b1)))
    const int64_t groups = (int64_t)batch * (kHid / 8);
    if (S > 8)
      k_reduce_bias_relu_bf16_q<<<(unsigned)((groups + 63) / 64), 256, 0, st>>>(P->part, S, batch, kHid,
                                                                                params + P->off.f1b, P->h1, kHid);
    else
      k_reduce_bias_relu_bf16<<<(int)std::min<int64_t>(4096, (groups + 255) / 256), 256, 0, st>>>(
          P->part, S, batch, kHid, params + P->off.f1b, P->h1, kHid);
    PCHK(hipGetLastError());
  }
  // the step writes the new state to a workspace (h_out may alias h_in); the heads copy it out
  GruFwdArgs a{};
  a.prm = params; a.o = P->off; a.rows = batch; a.s0 = 0;
  a.h1 = P->h1;
  a.wih = P->wihb; a.whh = P->whhb;
  a.hp = h_in; a.hp_map = nullptr; a.first = first; a.first_map = nullptr;
  a.h_out = P->hst;
  k_gru_fwd<false><<<dim3((batch + kGruRows - 1) / kGruRows, kGruSlices), 256, 0, st>>>(a);
  PCHK(hipGetLastError());
  k_gru_heads<<<(batch + 3) / 4, 256, 0, st>>>(params, P->off, P->hst, batch, h_out, mu, value,
                                                ActDraws{eps, seed, counter}, act, logp);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_policy_backward_seq(aslam_policy* P, const float* params, const int16_t* crop, const float* scan,
                              const float* state, int32_t T, int32_t N, const int32_t* robots, int32_t nb,
                              const float* h0, const uint8_t* first, const float* act, const float* old_logp,
                              const float* adv, const float* ret, float* grads, float* loss, aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !robots || !h0 || !first || !act || !old_logp || !adv || !ret ||
      !grads || !loss)
    return pfail(ASL_EINVAL, "null argument");
  if (!P->rec) return pfail(ASL_EINVAL, "feed-forward policy: use aslam_policy_backward");
  if (T < 1 || N < 1 || nb < 1 || nb > N) return pfail(ASL_EINVAL, "need T >= 1 and 1 <= nb <= N");
  if ((int64_t)T * nb > P->max_b) return pfail(ASL_EINVAL, "T * nb exceeds max_batch");
  hipStream_t st = (hipStream_t)stream;
  const Offsets& o = P->off;
  const int B = T * nb;
  k_seq_rows<<<(B + 255) / 256, 256, 0, st>>>(robots, nb, T, N, P->rows);
  PCHK(hipGetLastError());
  int rc = convert_weights(P, params, st, true);
  if (rc) return rc;
  int S = 0;
  rc = encode_fc1(P, params, crop, scan, state, P->rows, B, st, &S);
  if (rc) return rc;
  if (S > 0) {
    const int64_t groups = (int64_t)B * (kHid / 8);
    k_reduce_bias_relu_bf16<<<(int)std::min<int64_t>(4096, (groups + 255) / 256), 256, 0, st>>>(
        P->part, S, B, kHid, params + o.f1b, P->h1, kHid);
    PCHK(hipGetLastError());
  }
  // the GRU over the T steps, keeping what the backward reads
  const dim3 grid((nb + kGruRows - 1) / kGruRows, kGruSlices);
  for (int t = 0; t < T; ++t) {
    GruFwdArgs a{};
    a.prm = params; a.o = o; a.rows = nb; a.s0 = (int64_t)t * nb;
    a.h1 = P->h1;
    a.wih = P->wihb; a.whh = P->whhb;
    a.hp = t == 0 ? h0 : P->hst + (int64_t)(t - 1) * nb * kHid;
    a.hp_map = t == 0 ? robots : nullptr;
    a.first = first + (int64_t)t * N; a.first_map = robots;
    a.h_out = P->hst;
    a.g_r = P->g_r; a.g_z = P->g_z; a.g_n = P->g_n; a.g_ghn = P->g_ghn; a.hp_used = P->hp_used; a.hp_bf = P->hp_bf;
    k_gru_fwd<true><<<grid, 256, 0, st>>>(a);
    PCHK(hipGetLastError());
  }
  // heads + loss on every sample -> dh (FP32), head / log-std partial sums
  const int nh = (B + kHeadRows - 1) / kHeadRows;
  LossCoef lc{P->cfg.clip_eps, P->cfg.c_value, P->cfg.c_entropy, 1.0f / (float)B};
  k_heads<true, true><<<nh, 256, 0, st>>>(params, o, P->hst, B, nullptr, nullptr, act, old_logp, adv, ret, P->rows,
                                          lc, nullptr, P->hpart, P->dh_head);
  PCHK(hipGetLastError());
  PCHK(launch_reduce_heads(P->hpart, nh, params, o, grads, loss, P->cfg.c_value, P->cfg.c_entropy, st));
  // backpropagation through time
  for (int t = T - 1; t >= 0; --t) {
    GruBwdArgs b{};
    b.rows = nb; b.s0 = (int64_t)t * nb;
    b.dh_head = P->dh_head;
    b.dh_next = t == T - 1 ? nullptr : P->dh_buf + (int64_t)((t + 1) & 1) * nb * kHid;
    b.g_r = P->g_r; b.g_z = P->g_z; b.g_n = P->g_n; b.g_ghn = P->g_ghn; b.hp_used = P->hp_used;
    b.first = first + (int64_t)t * N; b.first_map = robots;
    b.whht = P->whht; b.dgi = P->dgi; b.dgh = P->dgh;
    b.dh_prev = P->dh_buf + (int64_t)(t & 1) * nb * kHid;
    k_gru_bwd_step<<<grid, 256, 0, st>>>(b);
    PCHK(hipGetLastError());
  }
  float* part = P->part;
  // GRU weights: dW_ih = sum_s dgi[s] h1[s]^T, dW_hh = sum_s dgh[s] hp[s]^T; biases: column sums
  {
    const int64_t S2 = splits_for(B, 256, kFc2Splits);
    const int S2u = slices_used(B, S2, 64);
    const int64_t n = (int64_t)kGates * kHid;
    PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16I{P->dgi, kGates, kGates, B}, LdBF16I{P->h1, kHid, kHid, B},
                                       EpiPartial{part, kHid, n}, kGates, kHid, B, (int)S2, st)));
    PCHK(launch_reduce(part, S2u, n, grads + o.gih, 0, n, st));
    PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16I{P->dgh, kGates, kGates, B}, LdBF16I{P->hp_bf, kHid, kHid, B},
                                       EpiPartial{part, kHid, n}, kGates, kHid, B, (int)S2, st)));
    PCHK(launch_reduce(part, S2u, n, grads + o.ghh, 0, n, st));
    k_colsum_bf16<<<kBiasBlocks, 256, 0, st>>>(P->dgi, B, kGates, part);
    PCHK(hipGetLastError());
    PCHK(launch_reduce(part, kBiasBlocks, kGates, grads + o.gbi, 0, kGates, st));
    k_colsum_bf16<<<kBiasBlocks, 256, 0, st>>>(P->dgh, B, kGates, part);
    PCHK(hipGetLastError());
    PCHK(launch_reduce(part, kBiasBlocks, kGates, grads + o.gbh, 0, kGates, st));
  }
  // FC1 output gradient: dz1 = (dgi W_ih) * [h1 > 0]
  PCHK((gemm::run<128, 128, 64, 2, 2>(LdBF16K{P->dgi, kGates, B, kGates}, LdBF16K{P->wiht, kGates, kHid, kGates},
                                     EpiReluGradBF16{P->dz1, P->h1, kHid, kHid}, B, kHid, kGates, 1, st)));
  return backward_fc1_encoder(P, params, crop, P->rows, B, grads, st);
}

}  // extern "C"
