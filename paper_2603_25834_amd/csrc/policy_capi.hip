// policy_capi.hip -- C-ABI of the PPO actor-critic (declared in include/aslam.h).
//
// The handle owns the minibatch workspaces (activations recomputed per
// minibatch, gradient partial sums), allocated once at create time for
// `max_batch` samples; forward and backward allocate nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "aslam.h"
#include "policy_kernels.h"

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
  uint16_t *a1 = nullptr, *a2 = nullptr, *h1 = nullptr, *dz2 = nullptr, *dz1 = nullptr, *dz2c = nullptr,
           *dz1c = nullptr;
  float *z2 = nullptr, *part = nullptr, *hpart = nullptr;
  int64_t part_floats = 0;
};

namespace {

constexpr int kBiasBlocks = 256;

int64_t splits_for(int64_t K, int64_t min_chunk, int64_t max_splits) {
  return std::max<int64_t>(1, std::min<int64_t>(max_splits, K / min_chunk));
}

int64_t part_need(const aslam_policy* p) {
  const int64_t k1 = p->off.k1;
  int64_t need = 4 * 256 * k1;                               // FC1 weight, up to 4 splits
  need = std::max<int64_t>(need, 64LL * kHid * kHid);        // FC2 weight, up to 64 splits
  need = std::max<int64_t>(need, 512LL * kC2 * 144);         // conv2 weight, up to 512 splits
  need = std::max<int64_t>(need, 1024LL * 16 * 16);          // conv1 weight, up to 1024 splits
  need = std::max<int64_t>(need, (int64_t)kBiasBlocks * 256);
  return need;
}

#define PCHK(e)                                                      \
  do {                                                               \
    hipError_t e_ = (e);                                             \
    if (e_ != hipSuccess) return pfail(ASL_EHIP, hipGetErrorString(e_)); \
  } while (0)

int forward_core(aslam_policy* P, const float* prm, const int16_t* crop, const float* scan, const float* state,
                 int B, hipStream_t st) {
  const Offsets& o = P->off;
  const int R = P->cfg.n_scan;
  k_conv1<<<std::min(B, 4096), 256, 0, st>>>(prm, o, crop, P->a1, B);
  PCHK(hipGetLastError());
  // conv2 as an implicit GEMM: [B*256 x 144] x [144 x 32]
  PCHK((gemm::run<128, 32, 4, 1, 1>(LdIm2colK{P->a1, B * 256}, LdW2K{prm + o.c2w},
                                    EpiConv2{P->a2, prm + o.c2b}, B * 256, kC2, 144, 1, st)));
  // FC1: [B x k1] x [k1 x 256]
  XSrc xs{P->a2, scan, state, R, B, o.k1};
  PCHK((gemm::run<128, 128, 2, 2, 1>(LdXK{xs}, LdF32K{prm + o.f1w, o.k1, kHid, o.k1},
                                     EpiBiasReluBF16{P->h1, prm + o.f1b, kHid}, B, kHid, o.k1, 1, st)));
  // FC2 pre-activation (FP32): [B x 256] x [256 x 256]
  PCHK((gemm::run<128, 128, 2, 2, 1>(LdBF16K{P->h1, kHid, B, kHid}, LdF32K{prm + o.f2w, kHid, kHid, kHid},
                                     EpiBiasF32{P->z2, prm + o.f2b, kHid}, B, kHid, kHid, 1, st)));
  return ASL_OK;
}

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
  aslam_policy* p = new (std::nothrow) aslam_policy();
  if (!p) return pfail(ASL_ENOMEM, "host allocation failed");
  p->cfg = *cfg;
  p->off = offsets(cfg->n_scan);
  p->max_b = cfg->max_batch;
  const int64_t Bm = p->max_b;
  p->part_floats = part_need(p);
  struct A { void** ptr; size_t bytes; } al[] = {
      {(void**)&p->a1, 2 * (size_t)Bm * kA1 * kA1 * kC1}, {(void**)&p->a2, 2 * (size_t)Bm * kFeat},
      {(void**)&p->h1, 2 * (size_t)Bm * kHid},            {(void**)&p->dz2, 2 * (size_t)Bm * kHid},
      {(void**)&p->dz1, 2 * (size_t)Bm * kHid},           {(void**)&p->dz2c, 2 * (size_t)Bm * kFeat},
      {(void**)&p->dz1c, 2 * (size_t)Bm * kA1 * kA1 * kC1}, {(void**)&p->z2, 4 * (size_t)Bm * kHid},
      {(void**)&p->part, 4 * (size_t)p->part_floats},
      {(void**)&p->hpart, 4 * (size_t)((Bm + kHeadRows - 1) / kHeadRows) * kHeadPart},
  };
  for (auto& a : al) {
    if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
      aslam_policy_destroy(p);
      return pfail(ASL_ENOMEM, "hipMalloc of policy workspace failed");
    }
  }
  *out = p;
  return ASL_OK;
}

int aslam_policy_destroy(aslam_policy* p) {
  if (!p) return pfail(ASL_EINVAL, "policy is NULL");
  void* ptrs[] = {p->a1, p->a2, p->h1, p->dz2, p->dz1, p->dz2c, p->dz1c, p->z2, p->part, p->hpart};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
  return ASL_OK;
}

int aslam_policy_forward(aslam_policy* P, const float* params, const int16_t* crop, const float* scan,
                         const float* state, int32_t batch, float* mu, float* value, aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !mu || !value) return pfail(ASL_EINVAL, "null argument");
  if (batch < 1 || batch > P->max_b) return pfail(ASL_EINVAL, "batch must be in [1, max_batch]");
  hipStream_t st = (hipStream_t)stream;
  int rc = forward_core(P, params, crop, scan, state, batch, st);
  if (rc) return rc;
  const int nb = (batch + kHeadRows - 1) / kHeadRows;
  k_heads<false><<<nb, 256, 0, st>>>(params, P->off, P->z2, batch, mu, value, nullptr, nullptr, nullptr, nullptr,
                                     LossCoef{0, 0, 0, 0}, nullptr, nullptr);
  PCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_policy_backward(aslam_policy* P, const float* params, const int16_t* crop, const float* scan,
                          const float* state, int32_t batch, const float* act, const float* old_logp,
                          const float* adv, const float* ret, float* grads, float* loss, aslam_stream_t stream) {
  if (!P || !params || !crop || !scan || !state || !act || !old_logp || !adv || !ret || !grads || !loss)
    return pfail(ASL_EINVAL, "null argument");
  if (batch < 1 || batch > P->max_b) return pfail(ASL_EINVAL, "batch must be in [1, max_batch]");
  hipStream_t st = (hipStream_t)stream;
  const Offsets& o = P->off;
  const int B = batch;
  const int R = P->cfg.n_scan;
  int rc = forward_core(P, params, crop, scan, state, B, st);
  if (rc) return rc;
  // heads + loss -> dz2, head / fc2-bias / log-std partial sums
  const int nb = (B + kHeadRows - 1) / kHeadRows;
  LossCoef lc{P->cfg.clip_eps, P->cfg.c_value, P->cfg.c_entropy, 1.0f / (float)B};
  k_heads<true><<<nb, 256, 0, st>>>(params, o, P->z2, B, nullptr, nullptr, act, old_logp, adv, ret, lc, P->dz2,
                                    P->hpart);
  PCHK(hipGetLastError());
  k_reduce_heads<<<1, 256, 0, st>>>(P->hpart, nb, grads, o, loss, P->cfg.c_entropy, P->cfg.c_value);
  PCHK(hipGetLastError());
  k_loss_total<<<1, 1, 0, st>>>(params, o, loss, P->cfg.c_value, P->cfg.c_entropy);
  PCHK(hipGetLastError());
  float* part = P->part;
  // FC2 weight: dW2[out][in] = sum_b dz2[b][out] h1[b][in]
  {
    const int64_t S = splits_for(B, 256, 64);
    const int64_t chunk = ((B + S - 1) / S + 31) / 32 * 32;
    const int S_used = (int)((B + chunk - 1) / chunk);
    PCHK((gemm::run<128, 128, 2, 2, 1>(LdBF16I{P->dz2, kHid, kHid, B}, LdBF16I{P->h1, kHid, kHid, B},
                                       EpiPartial{part, kHid, (int64_t)kHid * kHid}, kHid, kHid, B, (int)S, st)));
    k_reduce<<<256, 256, 0, st>>>(part, S_used, (int64_t)kHid * kHid, grads + o.f2w, 0, (int64_t)kHid * kHid);
    PCHK(hipGetLastError());
  }
  // dh1 -> dz1 = (dz2 W2) * [h1 > 0]
  PCHK((gemm::run<128, 128, 2, 2, 1>(LdBF16K{P->dz2, kHid, B, kHid}, LdF32I{params + o.f2w, kHid, kHid, kHid},
                                     EpiReluGradBF16{P->dz1, P->h1, kHid}, B, kHid, kHid, 1, st)));
  // FC1 bias
  k_bias_rows<<<kBiasBlocks, 256, 0, st>>>(P->dz1, B, kHid, part);
  PCHK(hipGetLastError());
  k_reduce<<<1, 256, 0, st>>>(part, kBiasBlocks, kHid, grads + o.f1b, 0, kHid);
  PCHK(hipGetLastError());
  // FC1 weight: dW1[out][k] = sum_b dz1[b][out] X[b][k]
  XSrc xs{P->a2, scan, state, R, B, o.k1};
  {
    const int64_t S = splits_for(B, 4096, 4);
    const int64_t chunk = ((B + S - 1) / S + 31) / 32 * 32;
    const int S_used = (int)((B + chunk - 1) / chunk);
    PCHK((gemm::run<128, 128, 2, 2, 1>(LdBF16I{P->dz1, kHid, kHid, B}, LdXI{xs},
                                       EpiPartial{part, o.k1, (int64_t)kHid * o.k1}, kHid, o.k1, B, (int)S, st)));
    k_reduce<<<1024, 256, 0, st>>>(part, S_used, (int64_t)kHid * o.k1, grads + o.f1w, 0, (int64_t)kHid * o.k1);
    PCHK(hipGetLastError());
  }
  // dA2 -> dz2c = (dz1 W1[:, :8192]) * [a2 > 0]
  PCHK((gemm::run<128, 128, 2, 2, 1>(LdBF16K{P->dz1, kHid, B, kHid}, LdF32I{params + o.f1w, o.k1, kFeat, kHid},
                                     EpiReluGradBF16{P->dz2c, P->a2, kFeat}, B, kFeat, kHid, 1, st)));
  // conv2 bias
  k_bias_c2<<<kBiasBlocks, 256, 0, st>>>(P->dz2c, B, part);
  PCHK(hipGetLastError());
  k_reduce<<<1, 64, 0, st>>>(part, kBiasBlocks, kC2, grads + o.c2b, 0, kC2);
  PCHK(hipGetLastError());
  // conv2 weight: dW2c[co][tap*16+ci] = sum_{b,p} dz2c[b][co][p] im2col(a1)[b,p][tap*16+ci]
  {
    const int64_t K = (int64_t)B * 256;
    const int64_t S = splits_for(K, 8192, 512);
    const int64_t chunk = ((K + S - 1) / S + 31) / 32 * 32;
    const int S_used = (int)((K + chunk - 1) / chunk);
    PCHK((gemm::run<32, 160, 2, 2, 1>(LdDz2cK{P->dz2c, (int)K}, LdIm2colI{P->a1, (int)K},
                                      EpiPartial{part, 144, (int64_t)kC2 * 144}, kC2, 144, (int)K, (int)S, st)));
    k_reduce<<<18, 256, 0, st>>>(part, S_used, (int64_t)kC2 * 144, grads + o.c2w, 1, (int64_t)kC2 * 144);
    PCHK(hipGetLastError());
  }
  // conv2 input gradient, one sub-pixel phase at a time -> dz1c = da1 * [a1 > 0]
  for (int ry = 0; ry < 2; ++ry)
    for (int rx = 0; rx < 2; ++rx) {
      const Phase ph = make_phase(ry, rx);
      PCHK((gemm::run<128, 16, 4, 1, 1>(LdPhaseA{P->dz2c, B * 256, ph}, LdPhaseB{params + o.c2w, ph},
                                        EpiPhase{P->dz1c, P->a1, ry, rx}, B * 256, kC1, 32 * ph.nty * ph.ntx, 1,
                                        st)));
    }
  // conv1 bias
  k_bias_rows<<<kBiasBlocks, 256, 0, st>>>(P->dz1c, (int64_t)B * kA1 * kA1, kC1, part);
  PCHK(hipGetLastError());
  k_reduce<<<1, 64, 0, st>>>(part, kBiasBlocks, kC1, grads + o.c1b, 0, kC1);
  PCHK(hipGetLastError());
  // conv1 weight: dW1c[co][tap] = sum_{b,y,x} dz1c[b][y][x][co] in(b, 2y+ky-1, 2x+kx-1)
  {
    const int64_t K = (int64_t)B * kA1 * kA1;
    const int64_t S = splits_for(K, 16384, 1024);
    const int64_t chunk = ((K + S - 1) / S + 31) / 32 * 32;
    const int S_used = (int)((K + chunk - 1) / chunk);
    PCHK((gemm::run<16, 16, 1, 1, 4>(LdDz1cI{P->dz1c, (int)K}, LdCropTapK{crop, (int)K},
                                     EpiPartial{part, 16, 256}, kC1, 16, (int)K, (int)S, st)));
    k_reduce<<<1, 256, 0, st>>>(part, S_used, 256, grads + o.c1w, 2, 256);
    PCHK(hipGetLastError());
  }
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

}  // extern "C"
