/*
 * aslam_oracle.c -- CPU oracle of the batched Active-SLAM environment step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  Plain
 * loops, one robot at a time, rays in index order, cells in traversal order.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math):
 * the pose and covariance state is FP32 as the workload fixes it, so every
 * FP32 expression below is written with explicit parentheses and is evaluated
 * exactly in that order.
 *
 * Method source: arXiv 2603.25834.  Sec. III-B (POMDP step), Sec. III-C
 * (action box, Eq. 4), Sec. III-D (log-odds grid, integration of the scan,
 * pose covariance), Sec. III-E (collision penalty, Eq. 7), Sec. IV-A (LiDAR,
 * collision ends the episode).  The EKF stands in for the fixed-lag backend
 * of Sec. III-D, and the reward is the map-entropy decrease plus a
 * D-optimality term (Table I "D-opt"; map entropy as in the related work of
 * Sec. II).  Where the paper is silent, each function's comment states the
 * reading it takes.
 */
#include "aslam_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define HIT_CODE 2
#define MISS_CODE 1

static const float PI_F = 3.14159265358979f;
static const float TWO_PI_F = 6.28318530717959f;

/* ------------------------------------------------------------------ tables */

/* Heading table: direction of heading step k is (cos, sin)(2 pi k / NANG),
 * rounded to the nearest Q14 integer.  Reading R1 (quantised headings). */
void orc_trig_table(int32_t* cq, int32_t* sq) {
  for (int k = 0; k < ORC_NANG; ++k) {
    double ang = (2.0 * M_PI * (double)k) / (double)ORC_NANG;
    cq[k] = (int32_t)llround(cos(ang) * (double)ORC_DIR_ONE);
    sq[k] = (int32_t)llround(sin(ang) * (double)ORC_DIR_ONE);
  }
}

/* Log-odds in 1/256 nat, nearest integer (ties away from zero do not occur
 * for the configured values). */
int32_t orc_logodds_q(float l) { return (int32_t)lrint((double)l * 256.0); }

/* Binary entropy of a cell with log-odds L/256 (nats), in Q32 units.
 * p = 1/(1+exp(-l)); h = -p ln p - (1-p) ln(1-p). */
void orc_entropy_table(int32_t lc, uint32_t* hq) {
  for (int32_t L = -lc; L <= lc; ++L) {
    double l = (double)L / 256.0;
    double p = 1.0 / (1.0 + exp(-l));
    double q = 1.0 - p;
    double h = -(p * log(p) + q * log(q));
    hq[L + lc] = (uint32_t)llround(h * 4294967296.0);
  }
}

/* ---------------------------------------------------------- random numbers
 * Philox4x64-10 as published (Salmon et al., SC'11): each round multiplies
 * counter words 0 and 2 by the two round multipliers (128-bit products), and
 * the new counter is (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1,
 * lo(M0 x0)); the key grows by the two Weyl constants between rounds. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Irwin-Hall(12) normal: the 256-bit block gives twelve 21-bit uniforms (bits
 * 63..43, 42..22 and 21..1 of each word); their integer sum minus its mean
 * 6 (2^21 - 1) is below 2^24 in magnitude, so the FP32 value is exact.  Mean
 * 0, variance 1 - 2^-42, support [-6, 6]: a reproducible stand-in for the
 * Gaussian draws of the workload. */
float orc_normal(uint64_t seed, uint64_t domain, uint64_t c0, uint64_t c1, uint64_t c2) {
  const uint64_t ctr[4] = {c0, c1, c2, 0}, key[2] = {seed, domain};
  uint64_t w[4];
  orc_philox4x64(ctr, key, w);
  const uint64_t m21 = (1ull << 21) - 1;
  int64_t sum = 0;
  for (int i = 0; i < 4; ++i) sum += (int64_t)((w[i] >> 43) & m21) + (int64_t)((w[i] >> 22) & m21) + (int64_t)((w[i] >> 1) & m21);
  return (float)(sum - 6 * (int64_t)m21) * (1.0f / 2097152.0f);
}

/* Feistel network of 8 rounds over b bits (halves of h = b/2 bits); four rounds left the
 * images of tiny domains visibly non-uniform after cycle walking. */
static uint64_t feistel(uint64_t v, int h, uint64_t seed, uint64_t counter) {
  const uint64_t mask = (1ull << h) - 1;
  uint64_t l = v >> h, r = v & mask;
  for (uint64_t round = 0; round < 8; ++round) {
    const uint64_t ctr[4] = {counter, r, round, 0}, key[2] = {seed, ORC_DOMAIN_PERM};
    uint64_t w[4];
    orc_philox4x64(ctr, key, w);
    uint64_t nl = r, nr = l ^ (w[0] & mask);
    l = nl;
    r = nr;
  }
  return (l << h) | r;
}

void orc_permute(int32_t n, uint64_t seed, uint64_t counter, int32_t* out) {
  int b = 2;
  while ((1ll << b) < (int64_t)n) b += 2;
  for (int32_t j = 0; j < n; ++j) {
    uint64_t y = feistel((uint64_t)j, b / 2, seed, counter);
    while (y >= (uint64_t)n) y = feistel(y, b / 2, seed, counter);  /* cycle walking */
    out[j] = (int32_t)y;
  }
}

/* idx(theta) = rint(theta * NANG/(2 pi)) mod NANG, in FP32. */
int32_t orc_heading_index(float theta) {
  const float k_ang = (float)((double)ORC_NANG / (2.0 * M_PI));
  float t = theta * k_ang;
  if (!(t > -1.0e9f && t < 1.0e9f)) t = 0.0f;
  int32_t i = (int32_t)rintf(t);
  i %= ORC_NANG;
  if (i < 0) i += ORC_NANG;
  return i;
}

static float wrap_pi(float th) {
  if (th >= PI_F) th = th - TWO_PI_F;
  else if (th < -PI_F) th = th + TWO_PI_F;
  return th;
}

/* Position in Q16 cells: rint(v * 65536/c) evaluated in FP32, clamped to
 * +-1e9 (a NaN maps to -1e9, i.e. far off the grid). */
static int64_t to_q16(float v, float inv_c16) {
  float t = v * inv_c16;
  if (!(t >= -1.0e9f)) t = -1.0e9f;
  if (!(t <= 1.0e9f)) t = 1.0e9f;
  return (int64_t)rintf(t);
}

int64_t orc_to_q16(float v, float cell_m) { return to_q16(v, (float)(65536.0 / (double)cell_m)); }

static int64_t floor_div_q16(int64_t v) {
  /* floor(v / 65536) for any sign */
  int64_t q = v / ORC_Q16;
  if (v % ORC_Q16 != 0 && v < 0) q -= 1;
  return q;
}

/* --------------------------------------------------------- exact traversal
 * The ray starts at the Q16 point O and runs along the integer direction
 * (a, b).  The origin cell is visited first (entry distance 0); then the walk
 * moves to the neighbour across whichever cell boundary the ray meets first.
 * Crossing the k-th x boundary happens at x-distance Ex = ex0 + k*65536
 * (Q16), i.e. at ray parameter Ex/|a|; the x crossing comes first iff
 * Ex*|b| <= Ey*|a| (an exact corner steps x first).  A cell entered at axis
 * distance E along an axis of direction component |d| is visited iff
 * E*scale <= lim*|d|.  For a LiDAR ray (a,b) is the Q14 table direction and
 * scale = 2^14, lim = range in Q16 cells; for a motion segment (a,b) is the
 * Q16 displacement and scale = lim = 1. */
typedef struct {
  int32_t s;
  int32_t cx, cy;
  int64_t ex, ey;      /* Q16 axis distance of the next x / y crossing */
  int64_t a, b;
  int64_t scale, lim;
  int started, finished;
  int end_reason;      /* 0 limit, 1 left grid, 2 origin outside */
  int64_t e_last;      /* axis distance at which the current cell was entered */
  int axis_last;       /* -1 origin, 0 x, 1 y */
} walker;

static void walk_init(walker* w, int64_t ox, int64_t oy, int64_t a, int64_t b, int64_t scale,
                      int64_t lim, int32_t s) {
  memset(w, 0, sizeof(*w));
  w->s = s;
  int64_t cx = floor_div_q16(ox), cy = floor_div_q16(oy);
  w->a = a; w->b = b; w->scale = scale; w->lim = lim;
  if (cx < 0 || cx >= s || cy < 0 || cy >= s) {
    w->finished = 1;
    w->end_reason = 2;
    return;
  }
  w->cx = (int32_t)cx;
  w->cy = (int32_t)cy;
  int64_t fx = ox - cx * ORC_Q16, fy = oy - cy * ORC_Q16;
  w->ex = (a > 0) ? (ORC_Q16 - fx) : fx;
  w->ey = (b > 0) ? (ORC_Q16 - fy) : fy;
}

/* Advance to the next visited cell.  Returns 1 and sets (cx,cy) when a cell
 * is visited, 0 when the walk has ended. */
static int walk_next(walker* w) {
  if (w->finished) return 0;
  if (!w->started) {
    w->started = 1;
    w->e_last = 0;
    w->axis_last = -1;
    return 1;
  }
  int64_t aa = llabs(w->a), bb = llabs(w->b);
  int step_x;
  if (aa == 0 && bb == 0) { w->finished = 1; w->end_reason = 0; return 0; }
  if (aa == 0) step_x = 0;
  else if (bb == 0) step_x = 1;
  else step_x = ((__int128)w->ex * bb <= (__int128)w->ey * aa);
  if (step_x) {
    if ((__int128)w->ex * w->scale > (__int128)w->lim * aa) { w->finished = 1; w->end_reason = 0; return 0; }
    int32_t nx = w->cx + (w->a > 0 ? 1 : -1);
    if (nx < 0 || nx >= w->s) { w->finished = 1; w->end_reason = 1; return 0; }
    w->cx = nx;
    w->e_last = w->ex;
    w->axis_last = 0;
    w->ex += ORC_Q16;
  } else {
    if ((__int128)w->ey * w->scale > (__int128)w->lim * bb) { w->finished = 1; w->end_reason = 0; return 0; }
    int32_t ny = w->cy + (w->b > 0 ? 1 : -1);
    if (ny < 0 || ny >= w->s) { w->finished = 1; w->end_reason = 1; return 0; }
    w->cy = ny;
    w->e_last = w->ey;
    w->axis_last = 1;
    w->ey += ORC_Q16;
  }
  return 1;
}

int32_t orc_walk(int64_t ox, int64_t oy, int64_t a, int64_t b, int64_t scale, int64_t lim,
                 int32_t s, int32_t* cells_x, int32_t* cells_y, int64_t* e_out, int32_t* axis_out,
                 int32_t max_out, int32_t* end_reason) {
  walker w;
  walk_init(&w, ox, oy, a, b, scale, lim, s);
  int32_t n = 0;
  while (n < max_out && walk_next(&w)) {
    cells_x[n] = w.cx;
    cells_y[n] = w.cy;
    e_out[n] = w.e_last;
    axis_out[n] = w.axis_last;
    ++n;
  }
  *end_reason = w.end_reason;
  return n;
}

static int world_occ(const uint32_t* wd, int32_t s, int32_t i, int32_t j) {
  int64_t bit = (int64_t)j * s + i;
  return (int)((wd[bit >> 5] >> (bit & 31)) & 1u);
}

/* ------------------------------------------------------------ reset/step */

static int32_t visit_side(const orc_config* cfg, int32_t s) {
  return (int32_t)ceil((double)s * (double)cfg->cell_m / (double)cfg->lc_cell_m);
}

/* The visit grid is kept for loop closure and for the paper's exploration reward. */
static int uses_visits(const orc_config* cfg) { return cfg->loop_closure || cfg->reward_mode == 1; }

/* Ray fan (Sec. IV-A): R rays equally spaced over fov heading steps; a full
 * circle starts along the heading, a partial fan at -fov/2 (reading). */
static int32_t fan_steps(const orc_config* cfg) {
  return (cfg->fov_steps > 0 && cfg->fov_steps < ORC_NANG) ? cfg->fov_steps : ORC_NANG;
}
static int32_t fan_start(const orc_config* cfg) {
  int32_t f = fan_steps(cfg);
  return f == ORC_NANG ? 0 : ORC_NANG - f / 2;
}

int32_t orc_noise_width(const orc_config* cfg) { return 5 + (cfg->range_sigma_m > 0.0f ? cfg->n_rays : 0); }

/* The reported range goes through the sensor model (noise, quantisation,
 * minimum range) when any of its parameters is set. */
static int sensor_model(const orc_config* cfg) {
  return cfg->range_sigma_m > 0.0f || cfg->range_quant_m > 0.0f || cfg->r_min_m > 0.0f;
}

/* det Sigma by cofactors along row 0, FP64 from the FP32 entries. */
static double cov_det(const float* c) {
  return (double)c[0] * ((double)c[3] * c[5] - (double)c[4] * c[4]) -
         (double)c[1] * ((double)c[1] * c[5] - (double)c[4] * c[2]) +
         (double)c[2] * ((double)c[1] * c[4] - (double)c[3] * c[2]);
}

/* SLAM uncertainty scalar U_t (reading: the cube root of det Sigma, the
 * geometric mean of the covariance eigenvalues; 0 if det <= 0). */
static double uncertainty(const float* c) {
  double d = cov_det(c);
  return d > 0.0 ? cbrt(d) : 0.0;
}

double orc_uncertainty(const float* c6) { return uncertainty(c6); }

static double clip01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Eq. (7): -lambda_col on collision, else R*_explore - R_abs + R*_Delta with
 *   R_explore = lambda_explore * dcells * I                         (Eq. 8)
 *   I = c + (1 - c) iota, c = clip((U_hi - U_{t-1}) / U_hi)^2,
 *   iota = clip(max(U_{t-1} - U_t, 0) / kappa)                     (Eqs. 10-12)
 *   R_abs = lambda_abs e^{U_{t-1}} U_{t-1}                           (Eq. 13)
 *   R_Delta = lambda_Delta e^{U_{t-1}} (U_{t-1} - U_t)               (Eq. 14)
 *   alpha = clip((d_min - d_crash) / (d_full - d_crash))             (Eq. 15)
 *   R*_explore = alpha R_explore; R*_Delta = alpha R_Delta if U fell, else R_Delta (Eqs. 16-17). */
double orc_paper_reward(const orc_config* cfg, int collided, double dcells, double u_prev, double u,
                        double d_min) {
  if (collided) return -(double)cfg->lambda_col;
  double cg = clip01(((double)cfg->u_hi - u_prev) / (double)cfg->u_hi);
  cg = cg * cg;
  double iota = clip01(fmax(u_prev - u, 0.0) / (double)cfg->kappa);
  double in = cg + (1.0 - cg) * iota;
  double r_explore = (double)cfg->lambda_explore * dcells * in;
  double eu = exp(u_prev);
  double r_abs = (double)cfg->lambda_abs * eu * u_prev;
  double r_delta = (double)cfg->lambda_delta * eu * (u_prev - u);
  double alpha = clip01((d_min - (double)cfg->d_crash_m) / ((double)cfg->d_full_m - (double)cfg->d_crash_m));
  return r_explore * alpha - r_abs + (u_prev - u > 0.0 ? r_delta * alpha : r_delta);
}

/* Proximity collision (Sec. IV-A): some occupied (or off-grid) cell within
 * d_crash of the Q16 point, by the exact integer point-to-square distance. */
static int near_obstacle(const orc_config* cfg, const uint32_t* W, int32_t s, int64_t px, int64_t py) {
  int64_t rc = llround((double)cfg->d_crash_m / (double)cfg->cell_m * 65536.0);
  int64_t cx = floor_div_q16(px), cy = floor_div_q16(py);
  int64_t m = rc / ORC_Q16 + 1;
  for (int64_t j = cy - m; j <= cy + m; ++j)
    for (int64_t i = cx - m; i <= cx + m; ++i) {
      int occ = (i < 0 || j < 0 || i >= s || j >= s) ? 1 : world_occ(W, s, (int32_t)i, (int32_t)j);
      if (!occ) continue;
      int64_t dx = i * ORC_Q16 - px, dy = j * ORC_Q16 - py;
      int64_t ux = px - (i + 1) * ORC_Q16, uy = py - (j + 1) * ORC_Q16;
      if (ux > dx) dx = ux;
      if (uy > dy) dy = uy;
      if (dx < 0) dx = 0;
      if (dy < 0) dy = 0;
      if (dx * dx + dy * dy < rc * rc) return 1;
    }
  return 0;
}

void orc_reset(const orc_config* cfg, orc_state* st, const float* init_pose, const uint8_t* mask) {
  int32_t lc = orc_logodds_q(cfg->l_clamp);
  uint32_t* hq = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(2 * lc + 1));
  orc_entropy_table(lc, hq);
  for (int32_t r = 0; r < st->n; ++r) {
    if (mask && !mask[r]) continue;
    int32_t s = st->side[r];
    int16_t* L = st->belief + st->cell_off[r];
    memset(L, 0, sizeof(int16_t) * (size_t)s * (size_t)s);
    for (int k = 0; k < 3; ++k) {
      st->pose[3 * r + k] = init_pose[3 * r + k];
      st->est[3 * r + k] = init_pose[3 * r + k];
    }
    float* c = st->cov + 6 * r;
    c[0] = cfg->var0_xy; c[1] = 0.0f; c[2] = 0.0f;
    c[3] = cfg->var0_xy; c[4] = 0.0f; c[5] = cfg->var0_th;
    st->h_q[r] = (int64_t)s * (int64_t)s * (int64_t)hq[lc];
    st->step[r] = 0;
    st->last_lc[r] = -(1 << 30);
    st->prev_vcell[r] = -1;
    st->u_prev[r] = uncertainty(c);
    if (uses_visits(cfg)) {
      int32_t nv = visit_side(cfg, s);
      for (int64_t k = 0; k < (int64_t)nv * nv; ++k) {
        st->visit_t[st->visit_off[r] + k] = -1;
        st->visit_x[st->visit_off[r] + k] = 0.0f;
        st->visit_y[st->visit_off[r] + k] = 0.0f;
        st->visit_last[st->visit_off[r] + k] = -1;
      }
    }
  }
  free(hq);
}

typedef struct {
  int32_t cq[ORC_NANG], sq[ORC_NANG];
  uint32_t* hq;
  int32_t lc, lhit, lmiss;
} orc_tables;

static float cos_tab(const orc_tables* T, int32_t idx) { return (float)T->cq[idx] * (1.0f / 16384.0f); }
static float sin_tab(const orc_tables* T, int32_t idx) { return (float)T->sq[idx] * (1.0f / 16384.0f); }

static void step_robot(const orc_config* cfg, const orc_tables* T, orc_state* st, int32_t r,
                       const float* act, const float* g, orc_out* out, uint8_t* code) {
  const int32_t s = st->side[r];
  const int32_t R = cfg->n_rays;
  const uint32_t* W = st->world + st->world_off[r];
  int16_t* L = st->belief + st->cell_off[r];
  float* p = st->pose + 3 * r;
  float* e = st->est + 3 * r;
  float* c = st->cov + 6 * r;
  const int32_t t = st->step[r];
  const float inv_c16 = (float)(65536.0 / (double)cfg->cell_m);
  int64_t cnt_march = 0, cnt_upd = 0, cnt_d = 0, cnt_dw = 0;

  /* --- action intake (Eq. 4 box; reading: NaN -> 0, clamp) */
  float v = fminf(fmaxf(act[0], 0.0f), cfg->v_max);
  float w = fminf(fmaxf(act[1], -cfg->w_max), cfg->w_max);
  if (v != v) v = 0.0f;
  if (w != w) w = 0.0f;
  float d = v * cfg->dt;
  float phi = w * cfg->dt;

  /* --- true motion with additive world-frame noise, then collision test */
  int32_t it = orc_heading_index(p[2]);
  float nx = (p[0] + d * cos_tab(T, it)) + cfg->sigma_x * g[0];
  float ny = (p[1] + d * sin_tab(T, it)) + cfg->sigma_y * g[1];
  float nth = wrap_pi((p[2] + phi) + cfg->sigma_th * g[2]);
  int64_t ox = to_q16(p[0], inv_c16), oy = to_q16(p[1], inv_c16);
  int64_t qx = to_q16(nx, inv_c16), qy = to_q16(ny, inv_c16);
  int collided = 0;
  {
    walker wk;
    walk_init(&wk, ox, oy, qx - ox, qy - oy, 1, 1, s);
    if (wk.end_reason == 2) collided = 1;
    while (!collided && walk_next(&wk)) {
      if (world_occ(W, s, wk.cx, wk.cy)) collided = 1;
    }
    if (!collided && wk.end_reason == 1) collided = 1;
  }
  if (collided) {
    d = 0.0f;
    phi = 0.0f;
  } else {
    p[0] = nx; p[1] = ny; p[2] = nth;
  }
  /* the paper's collision: closer than d_crash to an obstacle (the move stands) */
  if (cfg->d_crash_m > 0.0f && !collided &&
      near_obstacle(cfg, W, s, to_q16(p[0], inv_c16), to_q16(p[1], inv_c16)))
    collided = 1;

  /* --- EKF predict with the commanded motion (F from the heading before the step) */
  {
    int32_t ie = orc_heading_index(e[2]);
    float ch = cos_tab(T, ie), sh = sin_tab(T, ie);
    float a = -(d * sh);
    float b = d * ch;
    float qxv = cfg->sigma_x * cfg->sigma_x;
    float qyv = cfg->sigma_y * cfg->sigma_y;
    float qtv = cfg->sigma_th * cfg->sigma_th;
    float c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
    float n0 = ((c0 + (2.0f * a) * c2) + (a * a) * c5) + qxv;
    float n1 = ((c1 + a * c4) + b * c2) + (a * b) * c5;
    float n2 = c2 + a * c5;
    float n3 = ((c3 + (2.0f * b) * c4) + (b * b) * c5) + qyv;
    float n4 = c4 + b * c5;
    float n5 = c5 + qtv;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3; c[4] = n4; c[5] = n5;
    e[0] = e[0] + d * ch;
    e[1] = e[1] + d * sh;
    e[2] = wrap_pi(e[2] + phi);
  }

  /* --- visit cell of the GT position (loop closure, exploration reward) */
  int64_t vk = -1;
  int32_t vcell = -1;
  if (uses_visits(cfg)) {
    int32_t nv = visit_side(cfg, s);
    float inv_lc = (float)(1.0 / (double)cfg->lc_cell_m);
    int32_t vxi = (int32_t)floorf(p[0] * inv_lc);
    int32_t vyi = (int32_t)floorf(p[1] * inv_lc);
    if (vxi < 0) vxi = 0;
    if (vxi > nv - 1) vxi = nv - 1;
    if (vyi < 0) vyi = 0;
    if (vyi > nv - 1) vyi = nv - 1;
    vcell = vyi * nv + vxi;
    vk = st->visit_off[r] + vcell;
  }
  /* --- exploration novelty (Eq. 9): 1 on entering a never-visited cell, half the
   * fraction of an episode since the last visit on re-entering one, 0 while the
   * robot stays in the cell it was in at the previous step */
  double dcells = 0.0;
  if (cfg->reward_mode == 1) {
    if (vcell != st->prev_vcell[r]) {
      int32_t last = st->visit_last[vk];
      double tep = (double)(cfg->episode_len > 0 ? cfg->episode_len : 2048);
      dcells = last < 0 ? 1.0 : fmin(1.0, 0.5 * (double)(t - last) / tep);
    }
    st->visit_last[vk] = t;
    st->prev_vcell[r] = vcell;
  }

  /* --- loop closure: GT position back within the radius of its first visit */
  int closed = 0;
  if (cfg->loop_closure) {
    if (st->visit_t[vk] < 0) {
      st->visit_t[vk] = t;
      st->visit_x[vk] = p[0];
      st->visit_y[vk] = p[1];
    } else {
      float dx = p[0] - st->visit_x[vk];
      float dy = p[1] - st->visit_y[vk];
      float rr = cfg->lc_radius_m * cfg->lc_radius_m;
      if (t - st->visit_t[vk] >= cfg->lc_gap && t - st->last_lc[r] >= cfg->lc_gap &&
          (dx * dx + dy * dy) <= rr) {
        /* position fix z = GT + noise, H = [I2 0], R = sigma_lc^2 I2 */
        float zx = p[0] + cfg->lc_sigma_m * g[3];
        float zy = p[1] + cfg->lc_sigma_m * g[4];
        float rv = cfg->lc_sigma_m * cfg->lc_sigma_m;
        float c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
        float s00 = c0 + rv, s01 = c1, s11 = c3 + rv;
        float det = s00 * s11 - s01 * s01;
        float i00 = s11 / det, i01 = (-s01) / det, i11 = s00 / det;
        /* K = Sigma[:, xy] S^-1 */
        float kx0 = c0 * i00 + c1 * i01, kx1 = c0 * i01 + c1 * i11;
        float ky0 = c1 * i00 + c3 * i01, ky1 = c1 * i01 + c3 * i11;
        float kt0 = c2 * i00 + c4 * i01, kt1 = c2 * i01 + c4 * i11;
        float v0 = zx - e[0], v1 = zy - e[1];
        e[0] = e[0] + (kx0 * v0 + kx1 * v1);
        e[1] = e[1] + (ky0 * v0 + ky1 * v1);
        e[2] = wrap_pi(e[2] + (kt0 * v0 + kt1 * v1));
        /* Sigma - K Sigma[xy, :], upper triangle */
        c[0] = c0 - (kx0 * c0 + kx1 * c1);
        c[1] = c1 - (kx0 * c1 + kx1 * c3);
        c[2] = c2 - (kx0 * c2 + kx1 * c4);
        c[3] = c3 - (ky0 * c1 + ky1 * c3);
        c[4] = c4 - (ky0 * c2 + ky1 * c4);
        c[5] = c5 - (kt0 * c2 + kt1 * c4);
        st->last_lc[r] = t;
        closed = 1;
      }
    }
  }

  /* --- LiDAR march from the true pose through the world */
  const int64_t rmax_q = llround((double)cfg->r_max_m / (double)cfg->cell_m * 65536.0);
  const int32_t step_ang = fan_steps(cfg) / R;
  const int32_t ray0 = fan_start(cfg);
  const int32_t G = orc_noise_width(cfg);
  const int sensed = sensor_model(cfg);
  const float inv_quant = cfg->range_quant_m > 0.0f ? (float)(1.0 / (double)cfg->range_quant_m) : 0.0f;
  double d_min = 1.0e30;
  const float c16 = (float)((double)cfg->cell_m / 65536.0);
  float* ranges = out->ranges + (int64_t)r * R;
  int32_t* rho = out->rho_q + (int64_t)r * R;
  int32_t* hitc = out->hit_cell + (int64_t)r * R;
  memset(code, 0, (size_t)s * (size_t)s);
  {
    int32_t ib = orc_heading_index(p[2]);
    int64_t tx = to_q16(p[0], inv_c16), ty = to_q16(p[1], inv_c16);
    for (int32_t k = 0; k < R; ++k) {
      int32_t id = (ib + ray0 + k * step_ang) % ORC_NANG;
      int64_t a = T->cq[id], b = T->sq[id];
      walker wk;
      walk_init(&wk, tx, ty, a, b, ORC_DIR_ONE, rmax_q, s);
      int64_t rq = rmax_q;
      int32_t hc = -1;
      while (walk_next(&wk)) {
        ++cnt_march;
        int64_t cell = (int64_t)wk.cy * s + wk.cx;
        if (!(code[cell] & 4)) { code[cell] |= 4; ++cnt_dw; }
        if (world_occ(W, s, wk.cx, wk.cy)) {
          hc = (int32_t)cell;
          if (wk.axis_last < 0) rq = 0;
          else {
            /* range = entry distance of the hit cell, rounded up to the next
             * Q16 step so that the update walk reaches the hit cell */
            int64_t den = (wk.axis_last == 0) ? llabs(a) : llabs(b);
            rq = (wk.e_last * ORC_DIR_ONE + den - 1) / den;
          }
          break;
        }
      }
      /* reported range (Sec. IV-A sensor): true range + sigma * normal, rounded
       * to the quantum, clamped to [r_min, r_max]; the map update walks to it */
      float rep = (float)rq * c16;
      int64_t rho_u = rq;
      if (sensed) {
        if (cfg->range_sigma_m > 0.0f) rep = rep + cfg->range_sigma_m * g[5 + k];
        if (cfg->range_quant_m > 0.0f) rep = rintf(rep * inv_quant) * cfg->range_quant_m;
        rep = fminf(fmaxf(rep, cfg->r_min_m), cfg->r_max_m);
        rho_u = to_q16(rep, inv_c16);
      }
      rho[k] = (int32_t)rho_u;
      hitc[k] = hc;
      ranges[k] = rep;
      if ((double)rep < d_min) d_min = (double)rep;
    }
  }
  memset(code, 0, (size_t)s * (size_t)s);

  if (out->odo) {
    out->odo[2 * (int64_t)r] = d;
    out->odo[2 * (int64_t)r + 1] = phi;
  }
  if (out->d_min) out->d_min[r] = d_min;
  if (out->dcells) out->dcells[r] = dcells;
  if (cfg->slam_backend == 1) {
    /* the fixed-lag backbone finishes the step (scan matching, the window, the weighted map
     * integration and the reward); here: motion, the predicted estimate, the visits and the scan */
    out->collided[r] = (uint8_t)collided;
    out->closed[r] = 0;
    out->done[r] = (uint8_t)(collided || (cfg->episode_len > 0 && t + 1 >= cfg->episode_len));
    st->step[r] = t + 1;
    if (out->counters) {
      int64_t* q = out->counters + 4 * (int64_t)r;
      q[0] = cnt_march; q[1] = 0; q[2] = 0; q[3] = cnt_dw;
    }
    return;
  }

  /* --- map update from the estimated pose: one code per cell and scan
   * (HIT beats MISS), then one saturating add per coded cell. */
  int64_t dH = 0;
  {
    int64_t ex = to_q16(e[0], inv_c16), ey = to_q16(e[1], inv_c16);
    int64_t ecx = floor_div_q16(ex), ecy = floor_div_q16(ey);
    if (ecx >= 0 && ecx < s && ecy >= 0 && ecy < s) {
      int32_t ib = orc_heading_index(e[2]);
      for (int32_t k = 0; k < R; ++k) {
        int32_t id = (ib + ray0 + k * step_ang) % ORC_NANG;
        walker wk;
        walk_init(&wk, ex, ey, T->cq[id], T->sq[id], ORC_DIR_ONE, rho[k], s);
        int64_t last = -1;
        while (walk_next(&wk)) {
          ++cnt_upd;
          last = (int64_t)wk.cy * s + wk.cx;
          if (code[last] < MISS_CODE) code[last] = MISS_CODE;
        }
        if (hitc[k] >= 0 && wk.end_reason == 0 && last >= 0) code[last] = HIT_CODE;
      }
      for (int64_t cell = 0; cell < (int64_t)s * s; ++cell) {
        if (!code[cell]) continue;
        ++cnt_d;
        int32_t l0 = L[cell];
        int32_t l1 = l0 + (code[cell] == HIT_CODE ? T->lhit : T->lmiss);
        if (l1 > T->lc) l1 = T->lc;
        if (l1 < -T->lc) l1 = -T->lc;
        L[cell] = (int16_t)l1;
        dH += (int64_t)T->hq[l1 + T->lc] - (int64_t)T->hq[l0 + T->lc];
      }
    }
  }
  st->h_q[r] += dH;

  /* --- reward: entropy decrease + D-opt (-ln det Sigma) - collision penalty, or
   * the paper's Eq. (7) */
  double rH = (double)(-dH) / 4294967296.0;
  double det = cov_det(c);
  double ld = det > 0.0 ? log(det) : log(1.17549435e-38);
  out->r_entropy[r] = rH;
  out->logdet[r] = ld;
  if (cfg->reward_mode == 1) {
    double u = uncertainty(c);
    out->reward[r] = orc_paper_reward(cfg, collided, dcells, st->u_prev[r], u, d_min);
    st->u_prev[r] = u;
  } else {
    out->reward[r] = (double)cfg->w_entropy * rH - (double)cfg->w_dopt * ld -
                     (double)cfg->lambda_col * (double)collided;
  }
  out->collided[r] = (uint8_t)collided;
  out->closed[r] = (uint8_t)closed;
  out->done[r] = (uint8_t)(collided || (cfg->episode_len > 0 && t + 1 >= cfg->episode_len));
  st->step[r] = t + 1;
  if (out->counters) {
    int64_t* q = out->counters + 4 * (int64_t)r;
    q[0] = cnt_march; q[1] = cnt_upd; q[2] = cnt_d; q[3] = cnt_dw;
  }
}

void orc_step(const orc_config* cfg, orc_state* st, const float* actions, const float* noise,
              orc_out* out, int32_t n_threads) {
  orc_tables* T = (orc_tables*)malloc(sizeof(orc_tables));
  orc_trig_table(T->cq, T->sq);
  T->lc = orc_logodds_q(cfg->l_clamp);
  T->lhit = orc_logodds_q(cfg->l_hit);
  T->lmiss = orc_logodds_q(cfg->l_miss);
  T->hq = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(2 * T->lc + 1));
  orc_entropy_table(T->lc, T->hq);
  int32_t smax = 0;
  for (int32_t r = 0; r < st->n; ++r) if (st->side[r] > smax) smax = st->side[r];
  const int32_t G = orc_noise_width(cfg);
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
  {
    uint8_t* code = (uint8_t*)malloc((size_t)smax * (size_t)smax);
    float* own = (float*)malloc(sizeof(float) * (size_t)G);
#pragma omp for schedule(dynamic, 1)
    for (int32_t r = 0; r < st->n; ++r) {
      const float* g = noise ? noise + (int64_t)G * r : own;
      if (!noise) {
        /* the step's own draws: normal k of robot r at its step count draws[r] */
        for (int32_t k = 0; k < G; ++k)
          own[k] = orc_normal(cfg->noise_seed, ORC_DOMAIN_ENV, st->draws[r], (uint64_t)r, (uint64_t)k);
      }
      step_robot(cfg, T, st, r, actions + 2 * (int64_t)r, g, out, code);
      st->draws[r] += 1;
    }
    free(own);
    free(code);
  }
  free(T->hq);
  free(T);
}

/* Observation: scan / r_max, normalised estimate, covariance, and an
 * axis-aligned crop of the belief centred on the estimated cell (zero off
 * the map).  Reading: the configured observation replaces Eq. (3). */
void orc_observe(const orc_config* cfg, const orc_state* st, const float* ranges, int16_t* crop,
                 int32_t cs, float* scan, float* state12, const float* u_new, double alpha) {
  const int32_t R = cfg->n_rays;
  const float inv_c16 = (float)(65536.0 / (double)cfg->cell_m);
  const float inv_r = (float)(1.0 / (double)cfg->r_max_m);
  const float inv_pi = (float)(1.0 / M_PI);
  for (int32_t r = 0; r < st->n; ++r) {
    const int32_t s = st->side[r];
    const float* e = st->est + 3 * r;
    const float* c = st->cov + 6 * r;
    for (int32_t k = 0; k < R; ++k) scan[(int64_t)r * R + k] = ranges[(int64_t)r * R + k] * inv_r;
    const float inv_ext = (float)(1.0 / ((double)s * (double)cfg->cell_m));
    float* o = state12 + 12 * (int64_t)r;
    if (cfg->reward_mode == 1) {
      /* Eq. (3): [LiDAR, yaw, U_t]; yaw from the IMU (true heading), U_t of the filter */
      for (int k = 0; k < 12; ++k) o[k] = 0.0f;
      o[0] = st->pose[3 * r + 2] * inv_pi;
      double u = uncertainty(c);
      /* uncertainty bridge (Sec. III-G): blend in the external estimator's U */
      if (u_new) u = alpha * (double)u_new[r] + (1.0 - alpha) * u;
      o[1] = (float)u;
    } else {
      o[0] = e[0] * inv_ext; o[1] = e[1] * inv_ext; o[2] = e[2] * inv_pi;
      o[3] = c[0]; o[4] = c[1]; o[5] = c[2];
      o[6] = c[1]; o[7] = c[3]; o[8] = c[4];
      o[9] = c[2]; o[10] = c[4]; o[11] = c[5];
    }
    int64_t ecx = floor_div_q16(to_q16(e[0], inv_c16));
    int64_t ecy = floor_div_q16(to_q16(e[1], inv_c16));
    const int16_t* L = st->belief + st->cell_off[r];
    int16_t* cr = crop + (int64_t)r * cs * cs;
    for (int32_t jj = 0; jj < cs; ++jj)
      for (int32_t ii = 0; ii < cs; ++ii) {
        int64_t i = ecx - cs / 2 + ii, j = ecy - cs / 2 + jj;
        cr[jj * cs + ii] = (i >= 0 && i < s && j >= 0 && j < s) ? L[j * s + i] : 0;
      }
  }
}
