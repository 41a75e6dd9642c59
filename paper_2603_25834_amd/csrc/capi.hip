// capi.hip -- C-ABI of the gfx950 Active-SLAM library (declared in include/aslam.h).
//
// Host side only: argument validation, device allocation at create time,
// the library's own lookup tables (heading directions, binary entropy), the
// LDS plan of the step kernels, and HIP graph capture of step sequences.
// No call after create allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "aslam.h"
#include "env_internal.h"
#include "slam_internal.h"

using namespace aslam;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(ASL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace aslam {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace aslam

struct aslam_env {
  aslam_env_config cfg{};
  aslam_exec_config ex{};
  int32_t n = 0;
  std::vector<int32_t> sides;
  std::vector<RobotMeta> meta_h;
  int64_t world_words = 0, cells = 0, visits = 0;
  int32_t max_side = 0;
  int32_t lds_max = 0, cu_count = 0;
  bool was_reset = false;
  EnvParams P{};
  LdsPlan L{};
  // device allocations
  void* d_meta = nullptr;
  void* d_order = nullptr;
  void* d_cost = nullptr;
  int64_t fused_steps = 0;   // fused steps launched: the robot order is refreshed on every kOrderEvery-th
  void* d_world = nullptr;
  void* d_belief = nullptr;
  void* d_pose = nullptr;
  void* d_est = nullptr;
  void* d_cov = nullptr;
  void* d_hq_total = nullptr;
  void* d_step = nullptr;
  void* d_last_lc = nullptr;
  void* d_visit_t = nullptr;
  void* d_visit_xy = nullptr;
  void* d_rho = nullptr;
  void* d_hitc = nullptr;
  void* d_flags = nullptr;
  void* d_terms = nullptr;
  void* d_counters = nullptr;
  void* d_raylen = nullptr;
  void* d_dirtab = nullptr;
  void* d_hq_lut = nullptr;
  void* d_visit_last = nullptr;
  void* d_prev_vcell = nullptr;
  void* d_u_prev = nullptr;
  void* d_dcells = nullptr;
  void* d_dmin = nullptr;
  void* d_draws = nullptr;
  void* d_odo_u = nullptr;
  // fixed-lag backend
  FixedLag F{};
  std::vector<void*> fl_bufs;
  // captured step sequence
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;
};

namespace {

void free_env(aslam_env* e) {
  void** ptrs[] = {&e->d_meta, &e->d_order, &e->d_cost, &e->d_world, &e->d_belief, &e->d_pose, &e->d_est, &e->d_cov,
                   &e->d_hq_total, &e->d_step, &e->d_last_lc, &e->d_visit_t, &e->d_visit_xy, &e->d_rho,
                   &e->d_hitc, &e->d_flags, &e->d_terms, &e->d_counters, &e->d_raylen, &e->d_dirtab, &e->d_hq_lut,
                   &e->d_visit_last, &e->d_prev_vcell, &e->d_u_prev, &e->d_dcells, &e->d_dmin, &e->d_draws};
  for (void** p : ptrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  for (void* q : e->fl_bufs)
    if (q) (void)hipFree(q);
  e->fl_bufs.clear();
  if (e->d_odo_u) (void)hipFree(e->d_odo_u);
  e->d_odo_u = nullptr;
  if (e->graph_exec) (void)hipGraphExecDestroy(e->graph_exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
}

int32_t quantise_logodds(float l) { return (int32_t)std::lrint((double)l * 256.0); }

// Direction of heading step k, rounded to Q14, packed (cos low, sin high).
void build_dirtab(std::vector<int32_t>& t) {
  t.resize(kNang);
  for (int k = 0; k < kNang; ++k) {
    const double ang = (2.0 * M_PI * (double)k) / (double)kNang;
    const int32_t c = (int32_t)std::llround(std::cos(ang) * (double)kDirOne);
    const int32_t s = (int32_t)std::llround(std::sin(ang) * (double)kDirOne);
    t[k] = (int32_t)(((uint32_t)c & 0xffffu) | ((uint32_t)s << 16));
  }
}

// Binary entropy (nats) of a cell whose log-odds is L/256, in units of 2^-32 nat.
void build_entropy_lut(int32_t lc, std::vector<uint32_t>& h) {
  h.resize(2 * lc + 1);
  for (int32_t L = -lc; L <= lc; ++L) {
    const double l = (double)L / 256.0;
    const double p = 1.0 / (1.0 + std::exp(-l));
    const double q = 1.0 - p;
    const double ent = -(p * std::log(p) + q * std::log(q));
    h[L + lc] = (uint32_t)std::llround(ent * 4294967296.0);
  }
}

// Ray fan width in heading steps: the configured fov, or the full circle.
int32_t fan_steps(const aslam_env_config* c) {
  return (c->fov_steps > 0 && c->fov_steps < kNang) ? c->fov_steps : kNang;
}

bool uses_visits(const aslam_env_config* c) { return c->loop_closure || c->reward_mode == 1; }

int32_t noise_width(const aslam_env_config* c) { return 5 + (c->range_sigma_m > 0.0f ? c->n_rays : 0); }

int validate_config(const aslam_env_config* c) {
  if (!c) return fail(ASL_EINVAL, "config is NULL");
  if (c->fov_steps < 0 || c->fov_steps > kNang) return fail(ASL_EINVAL, "fov_steps must be in [0, 46080]");
  if (c->n_rays < 1 || c->n_rays > 4096 || fan_steps(c) % c->n_rays != 0)
    return fail(ASL_EINVAL, "n_rays must divide the fan (46080 heading steps for a full circle) and be in [1, 4096]");
  if (!(c->cell_m > 0.0f) || !(c->r_max_m > 0.0f)) return fail(ASL_EINVAL, "cell_m and r_max_m must be > 0");
  if ((double)c->r_max_m / (double)c->cell_m > 4096.0) return fail(ASL_EINVAL, "r_max_m exceeds 4096 cells");
  if (!(c->dt >= 0.0f) || !(c->v_max >= 0.0f) || !(c->w_max >= 0.0f)) return fail(ASL_EINVAL, "bad action box");
  const int32_t lc = quantise_logodds(c->l_clamp);
  if (lc < 1 || lc > 16384) return fail(ASL_EINVAL, "l_clamp out of range");
  if (c->loop_closure && (!(c->lc_cell_m > 0.0f) || c->lc_gap < 0))
    return fail(ASL_EINVAL, "bad loop-closure parameters");
  if (c->reward_mode != 0 && c->reward_mode != 1) return fail(ASL_EINVAL, "reward_mode must be 0 or 1");
  if (!(c->r_min_m >= 0.0f) || !(c->range_sigma_m >= 0.0f) || !(c->range_quant_m >= 0.0f) ||
      !(c->r_min_m <= c->r_max_m))
    return fail(ASL_EINVAL, "sensor model needs 0 <= r_min <= r_max, sigma >= 0, quantum >= 0");
  if (!(c->d_crash_m >= 0.0f) || (double)c->d_crash_m / (double)c->cell_m > 32.0)
    return fail(ASL_EINVAL, "d_crash_m must be in [0, 32 cells]");
  if (c->slam_backend != 0 && c->slam_backend != 1) return fail(ASL_EINVAL, "slam_backend must be 0 or 1");
  if (c->slam_backend == 1) {
    if (c->reward_mode != 1 || c->loop_closure)
      return fail(ASL_EINVAL, "the fixed-lag backend needs reward_mode 1 and loop_closure 0");
    if (c->lag_len < 2 || c->lag_len > slam::kMaxWindow || c->gn_iters < 0 || c->gn_iters > 100)
      return fail(ASL_EINVAL, "the fixed-lag backend needs lag_len in [2, 64] and gn_iters in [0, 100]");
    if (c->csm_W < 0 || c->csm_W > slam::kMaxHalf || c->csm_V < 0 || c->csm_V > slam::kMaxHalf ||
        (int64_t)(2 * c->csm_V + 1) * c->n_rays > slam::kMaxRayHeadings)
      return fail(ASL_EINVAL, "csm_W and csm_V must be in [0, 8] with (2 csm_V + 1) n_rays <= 8192");
    if (c->csm_step_xy_q < 1 || c->csm_step_xy_q > (1 << 20) || c->csm_step_h < 0 || c->csm_step_h > kNang)
      return fail(ASL_EINVAL, "csm steps out of range (step_xy_q in [1, 2^20], step_h in [0, 46080])");
    if (!(c->scan_sigma_xy_m > 0.0f) || !(c->scan_sigma_th > 0.0f) || !(c->int_weight_floor >= 0.0f) ||
        !(c->int_weight_floor <= 1.0f) || !(c->sigma_x > 0.0f) || !(c->sigma_y > 0.0f) || !(c->sigma_th > 0.0f) ||
        !(c->var0_xy > 0.0f) || !(c->var0_th > 0.0f))
      return fail(ASL_EINVAL, "the fixed-lag backend needs positive sigmas and var0, and a floor in [0, 1]");
  }
  if (c->reward_mode == 1) {
    if (!(c->lc_cell_m > 0.0f)) return fail(ASL_EINVAL, "reward_mode 1 needs lc_cell_m > 0 (novelty cells)");
    if (!(c->u_hi > 0.0f) || !(c->kappa > 0.0f) || !(c->d_full_m > c->d_crash_m))
      return fail(ASL_EINVAL, "reward_mode 1 needs u_hi > 0, kappa > 0 and d_full > d_crash");
  }
  return ASL_OK;
}

// LDS plan: lut | rho | perm | seg | shared | union(world rows, code bitmaps of one band).
int plan_lds(aslam_env* e, const aslam_exec_config& ex, LdsPlan& L) {
  const int32_t lc = e->P.lclamp;
  const int32_t rhat_cells = e->P.rhat_cells;
  L.off_lut = 0;
  L.off_rho = (int32_t)align_up((2 * lc + 1) * 4, 16);
  L.off_perm = L.off_rho + (int32_t)align_up(e->cfg.n_rays * 4, 16);
  L.off_seg = L.off_perm + (int32_t)align_up(e->cfg.n_rays * 4, 16);
  L.off_hist = L.off_seg + (int32_t)align_up(e->cfg.n_rays * 4, 16);
  L.off_misc = L.off_hist + 256;
  L.off_union = L.off_misc + 256;
  L.world_halo = rhat_cells + 3;
  int64_t world_max = 0, nw_max = 0, rows_max = 0;
  const int32_t hu = rhat_cells + 3;
  for (int32_t s : e->sides) {
    const int64_t rows = std::min<int64_t>(s, 2 * (int64_t)L.world_halo + 1);
    world_max = std::max<int64_t>(world_max, (rows * (s / 32) + 2 * (int64_t)march_guard_words(s)) * 4);
    const int64_t span = std::min<int64_t>(s, 2 * (int64_t)hu + 1);
    nw_max = std::max<int64_t>(nw_max, std::min<int64_t>(s / 32, (span + 31) / 32 + 1));
    rows_max = std::max<int64_t>(rows_max, span);
  }
  const int64_t budget = ex.lds_bytes > 0 ? std::min<int64_t>(ex.lds_bytes, e->lds_max) : e->lds_max;
  const int64_t free_bytes = budget - L.off_union;
  if (world_max > free_bytes)
    return fail(ASL_ENOTIMPL, "world window of the largest grid does not fit the LDS budget");
  int64_t band = ex.band_rows > 0 ? ex.band_rows : free_bytes / (8 * nw_max);
  band = std::min<int64_t>(band, rows_max);
  // bitmaps: 2 x band x nw words, cleared with 16-byte stores (+16 B slack)
  if (band > 8 && 8 * band * nw_max + 16 > free_bytes) band = (free_bytes - 16) / (8 * nw_max);
  if (band < 8 || 8 * band * nw_max + 16 > free_bytes)
    return fail(ASL_EINVAL, "band_rows does not fit the LDS budget (need >= 8 rows)");
  L.band_rows = (int32_t)band;
  L.union_bytes = (int32_t)std::max<int64_t>(world_max, 8 * band * nw_max + 16);
  L.total = L.off_union + L.union_bytes;
  L.record = ex.record_rays;
  L.mark_seg = ex.mark_seg;
  return ASL_OK;
}

// Device buffers of the fixed-lag backend and its constants (FP64 of the FP32 configuration values).
int setup_fixedlag(aslam_env* e, const std::vector<int32_t>& order) {
  (void)order;
  const aslam_env_config* c = &e->cfg;
  const int64_t n = e->n, L = c->lag_len, R = c->n_rays;
  FixedLag& F = e->F;
  F.L = (int32_t)L;
  F.iters = c->gn_iters;
  F.W = c->csm_W;
  F.V = c->csm_V;
  F.step_xy = c->csm_step_xy_q;
  F.step_h = c->csm_step_h;
  F.max_side = e->max_side;
  F.cell = (double)c->cell_m;
  F.l_max = (double)e->P.lclamp;
  F.floor = (double)c->int_weight_floor;
  const double sx = c->sigma_x, sy = c->sigma_y, st = c->sigma_th;
  F.odo_info[0] = 1.0 / (sx * sx);
  F.odo_info[1] = 1.0 / (sy * sy);
  F.odo_info[2] = 1.0 / (st * st);
  const double ss = c->scan_sigma_xy_m, sh = c->scan_sigma_th;
  F.scan_info[0] = 1.0 / (ss * ss);
  F.scan_info[1] = 1.0 / (ss * ss);
  F.scan_info[2] = 1.0 / (sh * sh);
  F.var0[0] = (double)c->var0_xy;
  F.var0[1] = (double)c->var0_xy;
  F.var0[2] = (double)c->var0_th;
  struct B { void** p; size_t bytes; } bufs[] = {
      {(void**)&F.x, sizeof(double) * n * L * 3},      {(void**)&F.prior, sizeof(double) * n * 6},
      {(void**)&F.odo, sizeof(double) * n * (L - 1) * 6}, {(void**)&F.scan, sizeof(double) * n * L * 6},
      {(void**)&F.sig, sizeof(double) * n * L * 3},    {(void**)&F.count, sizeof(int32_t) * n},
      {(void**)&F.xout, sizeof(double) * n * L * 3},   {(void**)&F.covw, sizeof(double) * n * 9},
      {(void**)&F.pose_q, sizeof(int32_t) * n * 3},    {(void**)&F.rho_q, sizeof(int32_t) * n * R},
      {(void**)&F.match, sizeof(int32_t) * n * 6},     {(void**)&F.pose_al, sizeof(int32_t) * n * 3},
      {(void**)&F.wq, sizeof(int32_t) * n},            {(void**)&F.coded, sizeof(int32_t) * n},
      {(void**)&F.a_off, sizeof(int32_t) * R},         {(void**)&F.cell_off, sizeof(int64_t) * n},
      {(void**)&F.side, sizeof(int32_t) * n},          {&e->d_odo_u, sizeof(float) * n * 2},
  };
  for (auto& b : bufs) {
    hipError_t he = hipMalloc(b.p, b.bytes);
    if (he != hipSuccess) return fail(ASL_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(he));
    if (b.p != &e->d_odo_u) e->fl_bufs.push_back(*b.p);
  }
  std::vector<int32_t> a_off(R), side(n);
  std::vector<int64_t> cell_off(n);
  for (int64_t k = 0; k < R; ++k) a_off[k] = (int32_t)((e->P.ray0 + k * e->P.step_ang) % kNang);
  for (int64_t i = 0; i < n; ++i) {
    side[i] = e->meta_h[i].side;
    cell_off[i] = e->meta_h[i].cell_off;
  }
  hipError_t he = hipMemcpy((void*)F.a_off, a_off.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy((void*)F.side, side.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy((void*)F.cell_off, cell_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemset(F.count, 0, sizeof(int32_t) * n);
  if (he == hipSuccess) he = hipMemset(F.match, 0, sizeof(int32_t) * n * 6);
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) return hip_fail(he, "fixed-lag setup");
  e->P.odo_u = (float*)e->d_odo_u;
  return ASL_OK;
}

}  // namespace

extern "C" {

const char* aslam_last_error(void) { return g_err.c_str(); }

int aslam_device_info(int32_t* lds_per_block, int32_t* cu_count) {
  int dev = 0, v = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (lds_per_block) {
    HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "lds attribute");
    *lds_per_block = v;
  }
  if (cu_count) {
    HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev), "cu attribute");
    *cu_count = v;
  }
  return ASL_OK;
}

int aslam_env_create(const aslam_env_config* cfg, int32_t n_robots, const int32_t* sides_host, aslam_env** out) {
  if (!out) return fail(ASL_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_config(cfg);
  if (rc) return rc;
  if (n_robots < 1 || !sides_host) return fail(ASL_EINVAL, "n_robots must be >= 1 and sides non-NULL");
  for (int32_t i = 0; i < n_robots; ++i) {
    const int32_t s = sides_host[i];
    if (s < 32 || s > 4096 || s % 32 != 0)
      return fail(ASL_EINVAL, "grid side " + std::to_string(s) + " of robot " + std::to_string(i) +
                                  " is not a multiple of 32 in [32, 4096]");
  }
  aslam_env* e = new (std::nothrow) aslam_env();
  if (!e) return fail(ASL_ENOMEM, "host allocation failed");
  e->cfg = *cfg;
  e->n = n_robots;
  e->sides.assign(sides_host, sides_host + n_robots);
  e->meta_h.resize(n_robots);
  for (int32_t i = 0; i < n_robots; ++i) {
    const int32_t s = e->sides[i];
    RobotMeta& m = e->meta_h[i];
    m.side = s;
    m.visit_side = uses_visits(cfg)
                       ? (int32_t)std::ceil((double)s * (double)cfg->cell_m / (double)cfg->lc_cell_m)
                       : 0;
    m.world_off = e->world_words;
    m.cell_off = e->cells;
    m.visit_off = e->visits;
    m.inv_ext = (float)(1.0 / ((double)s * (double)cfg->cell_m));
    m.pad = 0;
    e->world_words += (int64_t)s * s / 32;
    e->cells += (int64_t)s * s;
    e->visits += (int64_t)m.visit_side * m.visit_side;
    e->max_side = std::max(e->max_side, s);
  }
  std::vector<int32_t> order(n_robots);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return e->sides[a] > e->sides[b]; });

  rc = aslam_device_info(&e->lds_max, &e->cu_count);
  if (rc) { delete e; return rc; }

  const int64_t R = cfg->n_rays;
  struct Alloc { void** p; size_t bytes; } allocs[] = {
      {&e->d_meta, sizeof(RobotMeta) * (size_t)n_robots},
      {&e->d_order, sizeof(int32_t) * (size_t)n_robots},
      {&e->d_cost, sizeof(int32_t) * (size_t)n_robots},
      {&e->d_world, sizeof(uint32_t) * (size_t)e->world_words},
      {&e->d_belief, sizeof(int16_t) * (size_t)e->cells},
      {&e->d_pose, sizeof(float) * 3 * (size_t)n_robots},
      {&e->d_est, sizeof(float) * 3 * (size_t)n_robots},
      {&e->d_cov, sizeof(float) * 6 * (size_t)n_robots},
      {&e->d_hq_total, sizeof(int64_t) * (size_t)n_robots},
      {&e->d_step, sizeof(int32_t) * (size_t)n_robots},
      {&e->d_last_lc, sizeof(int32_t) * (size_t)n_robots},
      {&e->d_visit_t, sizeof(int32_t) * (size_t)std::max<int64_t>(e->visits, 1)},
      {&e->d_visit_xy, sizeof(float) * 2 * (size_t)std::max<int64_t>(e->visits, 1)},
      {&e->d_rho, sizeof(int32_t) * (size_t)(R * n_robots)},
      {&e->d_hitc, sizeof(int32_t) * (size_t)(R * n_robots)},
      {&e->d_flags, 2 * (size_t)n_robots},
      {&e->d_terms, sizeof(float) * 2 * (size_t)n_robots},
      {&e->d_counters, sizeof(int64_t) * 3 * (size_t)n_robots},
      {&e->d_raylen, sizeof(int16_t) * (size_t)(R * n_robots)},
      {&e->d_dirtab, sizeof(int32_t) * (size_t)kNang},
      {&e->d_hq_lut, sizeof(uint32_t) * (size_t)(2 * quantise_logodds(cfg->l_clamp) + 1)},
      {&e->d_visit_last, sizeof(int32_t) * (size_t)std::max<int64_t>(e->visits, 1)},
      {&e->d_prev_vcell, sizeof(int32_t) * (size_t)n_robots},
      {&e->d_u_prev, sizeof(double) * (size_t)n_robots},
      {&e->d_dcells, sizeof(double) * (size_t)n_robots},
      {&e->d_dmin, sizeof(int32_t) * (size_t)n_robots},
      {&e->d_draws, sizeof(uint64_t) * (size_t)n_robots},
  };
  for (auto& a : allocs) {
    hipError_t he = hipMalloc(a.p, a.bytes);
    if (he != hipSuccess) {
      free_env(e);
      delete e;
      return fail(ASL_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(he));
    }
  }
  std::vector<int32_t> dirtab;
  build_dirtab(dirtab);
  std::vector<uint32_t> lut;
  const int32_t lc = quantise_logodds(cfg->l_clamp);
  build_entropy_lut(lc, lut);
  hipError_t he = hipSuccess;
  if (he == hipSuccess) he = hipMemcpy(e->d_meta, e->meta_h.data(), sizeof(RobotMeta) * n_robots, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(e->d_order, order.data(), sizeof(int32_t) * n_robots, hipMemcpyHostToDevice);
  // until a robot has stepped, its grid area stands in for its work
  std::vector<int32_t> cost0(n_robots);
  for (int32_t r = 0; r < n_robots; ++r) cost0[r] = (int32_t)std::min<int64_t>((int64_t)e->sides[r] * e->sides[r] / 4, 1 << 30);
  if (he == hipSuccess) he = hipMemcpy(e->d_cost, cost0.data(), sizeof(int32_t) * n_robots, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(e->d_dirtab, dirtab.data(), sizeof(int32_t) * kNang, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(e->d_hq_lut, lut.data(), sizeof(uint32_t) * lut.size(), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemset(e->d_draws, 0, sizeof(uint64_t) * (size_t)n_robots);
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking);
  if (he != hipSuccess) {
    free_env(e);
    delete e;
    return hip_fail(he, "create");
  }

  EnvParams& P = e->P;
  P.n = n_robots;
  P.R = cfg->n_rays;
  P.step_ang = fan_steps(cfg) / cfg->n_rays;
  P.loop_closure = cfg->loop_closure ? 1 : 0;
  P.lc_gap = cfg->lc_gap;
  P.episode_len = cfg->episode_len;
  P.lhit = quantise_logodds(cfg->l_hit);
  P.lmiss = quantise_logodds(cfg->l_miss);
  P.lclamp = lc;
  P.rhat_q = (int32_t)std::llround((double)cfg->r_max_m / (double)cfg->cell_m * 65536.0);
  P.rhat_cells = (P.rhat_q + kQ16 - 1) / kQ16;
  P.v_max = cfg->v_max;
  P.w_max = cfg->w_max;
  P.dt = cfg->dt;
  P.sigma_x = cfg->sigma_x;
  P.sigma_y = cfg->sigma_y;
  P.sigma_th = cfg->sigma_th;
  P.qx = cfg->sigma_x * cfg->sigma_x;
  P.qy = cfg->sigma_y * cfg->sigma_y;
  P.qth = cfg->sigma_th * cfg->sigma_th;
  P.var0_xy = cfg->var0_xy;
  P.var0_th = cfg->var0_th;
  P.inv_c16 = (float)(65536.0 / (double)cfg->cell_m);
  P.c16 = (float)((double)cfg->cell_m / 65536.0);
  P.k_ang = (float)((double)kNang / (2.0 * M_PI));
  P.inv_lc = uses_visits(cfg) ? (float)(1.0 / (double)cfg->lc_cell_m) : 0.0f;
  P.lc_r2 = cfg->lc_radius_m * cfg->lc_radius_m;
  P.lc_sigma = cfg->lc_sigma_m;
  P.lc_var = cfg->lc_sigma_m * cfg->lc_sigma_m;
  P.w_entropy = cfg->w_entropy;
  P.w_dopt = cfg->w_dopt;
  P.lambda_col = cfg->lambda_col;
  P.inv_rmax = (float)(1.0 / (double)cfg->r_max_m);
  P.inv_pi = (float)(1.0 / M_PI);
  P.ray0 = fan_steps(cfg) == kNang ? 0 : kNang - fan_steps(cfg) / 2;
  P.reward_mode = cfg->reward_mode;
  P.uses_visits = uses_visits(cfg) ? 1 : 0;
  P.G = noise_width(cfg);
  P.sensed = (cfg->range_sigma_m > 0.0f || cfg->range_quant_m > 0.0f || cfg->r_min_m > 0.0f) ? 1 : 0;
  P.crash_q = (int32_t)std::llround((double)cfg->d_crash_m / (double)cfg->cell_m * 65536.0);
  P.tep = cfg->episode_len > 0 ? cfg->episode_len : 2048;
  P.r_max = cfg->r_max_m;
  P.r_min = cfg->r_min_m;
  P.range_sigma = cfg->range_sigma_m;
  P.range_quant = cfg->range_quant_m;
  P.inv_quant = cfg->range_quant_m > 0.0f ? (float)(1.0 / (double)cfg->range_quant_m) : 0.0f;
  P.d_crash = cfg->d_crash_m;
  P.d_full = cfg->d_full_m;
  P.lambda_explore = cfg->lambda_explore;
  P.lambda_abs = cfg->lambda_abs;
  P.lambda_delta = cfg->lambda_delta;
  P.u_hi = cfg->u_hi;
  P.kappa = cfg->kappa;
  P.meta = (const RobotMeta*)e->d_meta;
  P.order = (int32_t*)e->d_order;
  P.cost = (int32_t*)e->d_cost;
  P.world = (const uint32_t*)e->d_world;
  P.belief = (int16_t*)e->d_belief;
  P.pose = (float*)e->d_pose;
  P.est = (float*)e->d_est;
  P.cov = (float*)e->d_cov;
  P.hq_total = (int64_t*)e->d_hq_total;
  P.step = (int32_t*)e->d_step;
  P.last_lc = (int32_t*)e->d_last_lc;
  P.visit_t = (int32_t*)e->d_visit_t;
  P.visit_xy = (float*)e->d_visit_xy;
  P.rho = (int32_t*)e->d_rho;
  P.hitc = (int32_t*)e->d_hitc;
  P.flags = (uint8_t*)e->d_flags;
  P.terms = (float*)e->d_terms;
  P.counters = (int64_t*)e->d_counters;
  P.raylen = (int16_t*)e->d_raylen;
  P.dirtab = (const int32_t*)e->d_dirtab;
  P.hq_lut = (const uint32_t*)e->d_hq_lut;
  P.visit_last = (int32_t*)e->d_visit_last;
  P.prev_vcell = (int32_t*)e->d_prev_vcell;
  P.u_prev = (double*)e->d_u_prev;
  P.dcells = (double*)e->d_dcells;
  P.dmin_bits = (int32_t*)e->d_dmin;
  P.seed = cfg->noise_seed;
  P.draws = (uint64_t*)e->d_draws;
  P.odo_u = nullptr;
  if (cfg->slam_backend == 1) {
    rc = setup_fixedlag(e, order);
    if (rc) {
      std::string msg = g_err;
      free_env(e);
      delete e;
      return fail(rc, msg);
    }
  }

  he = set_kernel_lds_limits(e->lds_max);
  if (he != hipSuccess) {
    free_env(e);
    delete e;
    return hip_fail(he, "hipFuncSetAttribute");
  }
  aslam_exec_config ex{};
  ex.form = ASLAM_FORM_FUSED;
  ex.threads = 256;
  ex.band_rows = 0;
  ex.grid = 0;
  ex.record_rays = 0;
  ex.mark_seg = 0;
  ex.lds_bytes = 0;
  rc = aslam_env_set_exec(e, &ex);
  if (rc) {
    std::string msg = g_err;
    free_env(e);
    delete e;
    return fail(rc, msg);
  }
  *out = e;
  return ASL_OK;
}

int aslam_env_destroy(aslam_env* env) {
  if (!env) return fail(ASL_EINVAL, "env is NULL");
  free_env(env);
  delete env;
  return ASL_OK;
}

int64_t aslam_env_world_words(const aslam_env* env) { return env ? env->world_words : -1; }
int64_t aslam_env_cells(const aslam_env* env) { return env ? env->cells : -1; }
int32_t aslam_env_noise_width(const aslam_env* env) { return env ? noise_width(&env->cfg) : -1; }
int64_t aslam_env_visit_cells(const aslam_env* env) { return env ? env->visits : -1; }

int aslam_env_set_exec(aslam_env* env, const aslam_exec_config* ex) {
  if (!env || !ex) return fail(ASL_EINVAL, "env or exec config is NULL");
  if (ex->form != ASLAM_FORM_PLAIN && ex->form != ASLAM_FORM_FUSED) return fail(ASL_EINVAL, "unknown form");
  if (ex->threads != 128 && ex->threads != 192 && ex->threads != 256 && ex->threads != 384 && ex->threads != 512)
    return fail(ASL_EINVAL, "threads must be 128, 192, 256, 384 or 512");
  if (ex->grid < 0 || ex->band_rows < 0 || ex->lds_bytes < 0) return fail(ASL_EINVAL, "negative exec field");
  if (ex->mark_seg != 0 && (ex->mark_seg < 8 || ex->mark_seg > 1024))
    return fail(ASL_EINVAL, "mark_seg must be 0 or in [8, 1024]");
  LdsPlan L{};
  int rc = plan_lds(env, *ex, L);
  if (rc) return rc;
  env->ex = *ex;
  env->L = L;
  return ASL_OK;
}

int aslam_env_get_exec(const aslam_env* env, aslam_exec_config* ex) {
  if (!env || !ex) return fail(ASL_EINVAL, "env or exec config is NULL");
  *ex = env->ex;
  ex->band_rows = env->L.band_rows;
  ex->lds_bytes = env->L.total;
  return ASL_OK;
}

int aslam_env_reset(aslam_env* env, const uint32_t* world_dev, const float* init_pose_dev, const uint8_t* mask_dev,
                    aslam_stream_t stream) {
  if (!env || !world_dev || !init_pose_dev) return fail(ASL_EINVAL, "env, world or init_pose is NULL");
  HIP_TRY(launch_reset(env->P, world_dev, init_pose_dev, mask_dev, env->max_side, (hipStream_t)stream), "reset");
  if (env->cfg.slam_backend == 1)
    HIP_TRY(launch_reset_fixedlag(env->P, env->F, init_pose_dev, mask_dev, (hipStream_t)stream), "reset");
  env->was_reset = true;
  return ASL_OK;
}

static int do_step(aslam_env* env, const StepArgs& A, hipStream_t st) {
  hipError_t he;
  if (env->cfg.slam_backend == 1) {
    he = launch_step_fixedlag(env->P, A, env->L, env->F, env->ex.threads, st);
  } else if (env->ex.form == ASLAM_FORM_PLAIN) {
    he = launch_step_plain(env->P, A, env->L, env->ex.threads, st);
  } else {
    const int grid = env->ex.grid > 0 ? std::min(env->ex.grid, env->n) : env->n;
    he = launch_step_fused(env->P, A, env->L, env->ex.threads, grid, env->fused_steps++ % kOrderEvery == 0, st);
  }
  if (he != hipSuccess) return hip_fail(he, "env_step launch");
  return ASL_OK;
}

int aslam_env_step(aslam_env* env, const float* actions_dev, const float* noise_dev, float* ranges_dev,
                   float* reward_dev, uint8_t* done_dev, aslam_stream_t stream) {
  if (!env || !actions_dev || !ranges_dev || !reward_dev || !done_dev)
    return fail(ASL_EINVAL, "null argument to env_step");
  if (!env->was_reset) return fail(ASL_ESTATE, "env_step called before env_reset");
  StepArgs A{actions_dev, noise_dev, ranges_dev, reward_dev, done_dev};
  return do_step(env, A, (hipStream_t)stream);
}

int aslam_env_observe(aslam_env* env, const float* ranges_dev, int16_t* crop_dev, int32_t crop, float* scan_dev,
                      float* state_dev, aslam_stream_t stream) {
  if (!env || !ranges_dev || !crop_dev || !scan_dev || !state_dev) return fail(ASL_EINVAL, "null argument");
  if (crop < 2 || crop > 1024 || crop % 2) return fail(ASL_EINVAL, "crop must be even in [2, 1024]");
  if (!env->was_reset) return fail(ASL_ESTATE, "observe called before env_reset");
  HIP_TRY(launch_observe(env->P, ranges_dev, crop_dev, crop, scan_dev, state_dev, nullptr, 0.0, (hipStream_t)stream),
          "observe");
  return ASL_OK;
}

int aslam_env_observe_bridge(aslam_env* env, const float* ranges_dev, int16_t* crop_dev, int32_t crop,
                             float* scan_dev, float* state_dev, const float* u_new_dev, int64_t t, int64_t t_bridge,
                             aslam_stream_t stream) {
  if (!env || !ranges_dev || !crop_dev || !scan_dev || !state_dev || !u_new_dev)
    return fail(ASL_EINVAL, "null argument");
  if (crop < 2 || crop > 1024 || crop % 2) return fail(ASL_EINVAL, "crop must be even in [2, 1024]");
  if (env->cfg.reward_mode != 1) return fail(ASL_EINVAL, "the bridge needs reward_mode 1 (U_t in the observation)");
  if (t < 0 || t_bridge < 1) return fail(ASL_EINVAL, "need t >= 0 and t_bridge >= 1");
  if (!env->was_reset) return fail(ASL_ESTATE, "observe called before env_reset");
  const double alpha = std::min(1.0, (double)t / (double)t_bridge);
  HIP_TRY(launch_observe(env->P, ranges_dev, crop_dev, crop, scan_dev, state_dev, u_new_dev, alpha,
                         (hipStream_t)stream),
          "observe");
  return ASL_OK;
}

int aslam_env_read(const aslam_env* env, int32_t field, void* dst_dev, aslam_stream_t stream) {
  if (!env || !dst_dev) return fail(ASL_EINVAL, "env or dst is NULL");
  const void* src = nullptr;
  size_t bytes = 0;
  const size_t n = (size_t)env->n, R = (size_t)env->cfg.n_rays;
  switch (field) {
    case ASLAM_FIELD_BELIEF: src = env->d_belief; bytes = 2 * (size_t)env->cells; break;
    case ASLAM_FIELD_POSE: src = env->d_pose; bytes = 12 * n; break;
    case ASLAM_FIELD_EST: src = env->d_est; bytes = 12 * n; break;
    case ASLAM_FIELD_COV: src = env->d_cov; bytes = 24 * n; break;
    case ASLAM_FIELD_RHO_Q: src = env->d_rho; bytes = 4 * n * R; break;
    case ASLAM_FIELD_HIT_CELL: src = env->d_hitc; bytes = 4 * n * R; break;
    case ASLAM_FIELD_ENTROPY_Q: src = env->d_hq_total; bytes = 8 * n; break;
    case ASLAM_FIELD_STEP: src = env->d_step; bytes = 4 * n; break;
    case ASLAM_FIELD_FLAGS: src = env->d_flags; bytes = 2 * n; break;
    case ASLAM_FIELD_TERMS: src = env->d_terms; bytes = 8 * n; break;
    case ASLAM_FIELD_COUNTERS: src = env->d_counters; bytes = 24 * n; break;
    case ASLAM_FIELD_U_PREV: src = env->d_u_prev; bytes = 8 * n; break;
    case ASLAM_FIELD_VISIT_LAST: src = env->d_visit_last; bytes = 4 * (size_t)env->visits; break;
    case ASLAM_FIELD_DRAWS: src = env->d_draws; bytes = 8 * n; break;
    case ASLAM_FIELD_MATCH:
      if (env->cfg.slam_backend != 1) return fail(ASL_EINVAL, "no scan match without the fixed-lag backend");
      src = env->F.match;
      bytes = 24 * n;
      break;
    default: return fail(ASL_EINVAL, "unknown field");
  }
  HIP_TRY(hipMemcpyAsync(dst_dev, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream), "read");
  return ASL_OK;
}

int aslam_env_graph_build(aslam_env* env, int32_t k_steps, const float* actions_dev, int64_t a_stride,
                          const float* noise_dev, int64_t g_stride, float* ranges_dev, int64_t r_stride,
                          float* reward_dev, int64_t w_stride, uint8_t* done_dev, int64_t d_stride) {
  if (!env || k_steps < 1 || !actions_dev || !ranges_dev || !reward_dev || !done_dev)
    return fail(ASL_EINVAL, "bad graph arguments");
  if (a_stride < 0 || g_stride < 0 || r_stride < 0 || w_stride < 0 || d_stride < 0)
    return fail(ASL_EINVAL, "negative stride");
  if (env->graph_exec) {
    (void)hipGraphExecDestroy(env->graph_exec);
    env->graph_exec = nullptr;
  }
  if (env->graph) {
    (void)hipGraphDestroy(env->graph);
    env->graph = nullptr;
  }
  hipStream_t cs = env->capture_stream;
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  for (int32_t k = 0; k < k_steps; ++k) {
    StepArgs A{actions_dev + k * a_stride, noise_dev ? noise_dev + k * g_stride : nullptr, ranges_dev + k * r_stride,
               reward_dev + k * w_stride, done_dev + k * d_stride};
    int rc = do_step(env, A, cs);
    if (rc) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
  }
  HIP_TRY(hipStreamEndCapture(cs, &env->graph), "end capture");
  HIP_TRY(hipGraphInstantiate(&env->graph_exec, env->graph, nullptr, nullptr, 0), "instantiate");
  return ASL_OK;
}

int aslam_env_graph_launch(aslam_env* env, aslam_stream_t stream) {
  if (!env) return fail(ASL_EINVAL, "env is NULL");
  if (!env->graph_exec) return fail(ASL_ESTATE, "no graph built");
  if (!env->was_reset) return fail(ASL_ESTATE, "graph launched before env_reset");
  HIP_TRY(hipGraphLaunch(env->graph_exec, (hipStream_t)stream), "graph launch");
  return ASL_OK;
}

}  // extern "C"
