/*
 * aslam_oracle.h -- CPU oracle of the batched Active-SLAM environment step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * statement of what the environment step computes, written from the paper
 * (Massive Parallel Deep Reinforcement Learning for Active SLAM, arXiv
 * 2603.25834).  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header, table or constant
 * generator with the GPU library; each side builds its own tables.
 *
 * Passages followed (section / equation of the paper):
 *   - POMDP step contract: Sec. III-B, Eqs. (1)-(2).
 *   - action space (v, w): Sec. III-C, Eq. (4).
 *   - LiDAR ray fan and max range: Sec. IV-A (sensor description).
 *   - 2-D log-odds occupancy grid, integration of the aligned scan: Sec. III-D.
 *   - pose covariance as the uncertainty source, D-optimality: Sec. III-D,
 *     Eq. (6); Sec. II (Table I, "D-opt").
 *   - collision penalty and episode end: Sec. III-E, Eq. (7); Sec. IV-A.
 *   - the paper's reward (reward_mode 1): Sec. III-E, Eqs. (7)-(17) -- exploration
 *     reward with the cell-novelty factor and the intrinsic scaling, absolute and
 *     differential uncertainty terms, anti-wall-hugging factor; sensor model of
 *     Sec. IV-A (front field of view, minimum range, range noise, quantisation,
 *     proximity collision); observation [LiDAR, yaw, U_t] of Sec. III-C, Eq. (3).
 * Where the paper is silent, the comment of each function states the reading it takes.
 *
 * Parity status: every function here is pinned by a CPU test (closed forms,
 * brute force, invariants) -- see tests/test_oracle_*.py.
 */
#ifndef ASLAM_ORACLE_H
#define ASLAM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NANG 46080          /* heading steps per turn */
#define ORC_Q16 65536           /* position fraction: 1/65536 cell */
#define ORC_DIR_ONE 16384       /* unit direction in the table: Q14 */

typedef struct {
  int32_t n_rays;        /* R; must divide ORC_NANG */
  int32_t loop_closure;  /* 0 / 1 */
  int32_t lc_gap;        /* minimum steps between first visit / last closure and a closure */
  int32_t episode_len;   /* steps per episode; 0 = unbounded */
  float cell_m;          /* cell side (m) */
  float r_max_m;         /* LiDAR max range (m) */
  float dt;              /* control period (s) */
  float v_max, w_max;    /* action box [0,v_max] x [-w_max,w_max] */
  float sigma_x, sigma_y, sigma_th;  /* odometry noise std per step */
  float var0_xy, var0_th;            /* initial covariance diagonal */
  float lc_cell_m, lc_radius_m, lc_sigma_m; /* loop-closure visit cell, radius, fix std */
  float l_hit, l_miss, l_clamp;      /* log-odds increments and clamp (nats) */
  float w_entropy, w_dopt, lambda_col; /* reward weights */
  /* sensor model and the paper's reward (zeros keep the workload's step) */
  int32_t fov_steps;     /* heading steps spanned by the ray fan; 0 or ORC_NANG = full circle */
  int32_t reward_mode;   /* 0 workload reward, 1 the paper's Eq. (7) */
  float r_min_m;         /* reported ranges below this are raised to it */
  float range_sigma_m;   /* range noise std; then the noise input has R more normals per robot */
  float range_quant_m;   /* reported ranges rounded to multiples of this */
  float d_crash_m;       /* proximity collision distance (0 = off) */
  float d_full_m;        /* clearance at which the wall-hugging factor reaches 1 */
  float lambda_explore, lambda_abs, lambda_delta, u_hi, kappa;
  uint64_t noise_seed;   /* key of the step's own normal draws (used when the caller passes none) */
  int32_t slam_backend;  /* 0: the EKF of the step; 1: the fixed-lag graph of Sec. III-D (orc_step then
                            stops after the LiDAR march; oracle/fixedlag_env.py finishes the step) */
} orc_config;

/* Per-robot state, caller-owned arrays (robots are independent). */
typedef struct {
  int32_t n;                 /* robots in this batch */
  const int32_t* side;       /* [n] grid side (cells), multiple of 32 */
  const int64_t* world_off;  /* [n] offset of robot i's world in 32-bit words */
  const int64_t* cell_off;   /* [n] offset of robot i's belief in cells */
  const int64_t* visit_off;  /* [n] offset of robot i's visit grid in entries */
  const uint32_t* world;     /* occupancy bits: cell (i,j) -> bit (j*s+i) */
  int16_t* belief;           /* log-odds, Q8 (1/256 nat), row-major j*s+i */
  float* pose;               /* [n,3] true (x,y,theta) */
  float* est;                /* [n,3] estimate */
  float* cov;                /* [n,6] xx,xy,xt,yy,yt,tt */
  int64_t* h_q;              /* [n] map entropy, Q32 nats */
  int32_t* step;             /* [n] steps since reset */
  int32_t* last_lc;          /* [n] step of the last loop closure */
  int32_t* visit_t;          /* ragged first-visit step (-1 none) */
  float* visit_x;            /* ragged first-visit position */
  float* visit_y;
  int32_t* visit_last;       /* ragged last-visit step (-1 none; reward_mode 1) */
  int32_t* prev_vcell;       /* [n] visit cell of the previous step (-1 none; reward_mode 1) */
  double* u_prev;            /* [n] U_{t-1} = cbrt(det Sigma) of the previous step (reward_mode 1) */
  uint64_t* draws;           /* [n] steps taken since the state was created (counter of the draws) */
} orc_state;

typedef struct {
  float* ranges;       /* [n,R] */
  int32_t* rho_q;      /* [n,R] Q16 cells */
  int32_t* hit_cell;   /* [n,R] j*s+i or -1 */
  double* reward;      /* [n] */
  uint8_t* done;       /* [n] */
  uint8_t* collided;   /* [n] */
  uint8_t* closed;     /* [n] loop closure fired this step */
  double* r_entropy;   /* [n] entropy decrease (nats) */
  double* logdet;      /* [n] ln det Sigma */
  int64_t* counters;   /* [n,4]: march visits, update visits, distinct updated cells, distinct world cells read */
  float* odo;          /* [n,2] commanded motion (d, phi) of the step, 0 when blocked (may be NULL) */
  double* d_min;       /* [n] smallest reported range (may be NULL) */
  double* dcells;      /* [n] novelty of the step's visit cell, Eq. (9) (may be NULL) */
} orc_out;

/* Tables built by the oracle's own code. */
void orc_trig_table(int32_t* cq, int32_t* sq);           /* [ORC_NANG] each, Q14 */
int32_t orc_logodds_q(float l);                          /* RNE(l*256) */
void orc_entropy_table(int32_t l_clamp_q, uint32_t* hq); /* [2*l_clamp_q+1], Q32 nats */
int32_t orc_heading_index(float theta);

/* Exact integer traversal (one ray or segment); writes visited cells in order.
 * Returns the number of cells written (<= max_out); *end_reason: 0 limit,
 * 1 left grid, 2 origin outside the grid. e_out receives the axis distance
 * (Q16) at which each cell was entered (0 for the origin cell), axis_out 0=x,
 * 1=y, -1 origin. */
int32_t orc_walk(int64_t ox, int64_t oy, int64_t a, int64_t b, int64_t scale, int64_t lim,
                 int32_t s, int32_t* cells_x, int32_t* cells_y, int64_t* e_out, int32_t* axis_out,
                 int32_t max_out, int32_t* end_reason);

/* Counter-based random numbers (test twin of the library's generator).
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): out = 10 rounds over the 4-word counter under the
 * 2-word key. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* One standard-normal draw: the Irwin-Hall sum of the twelve 21-bit fields of
 * the block at counter (c0, c1, c2, 0) under key (seed, domain), centred and
 * scaled exactly: (sum - 6 (2^21 - 1)) / 2^21. */
float orc_normal(uint64_t seed, uint64_t domain, uint64_t c0, uint64_t c1, uint64_t c2);
/* Keyed permutation of [0, n): an 8-round Feistel network on the smallest even
 * number of bits b >= 2 with 2^b >= n, round function = low b/2 bits of word 0
 * of Philox at counter (counter, half, round, 0) under key (seed, 3), with
 * cycle walking back into [0, n).  out[j] = image of j. */
void orc_permute(int32_t n, uint64_t seed, uint64_t counter, int32_t* out);
#define ORC_DOMAIN_ENV 1        /* env step draws: counter (robot's step count, robot, draw index) */
#define ORC_DOMAIN_ACTION 2     /* action sampling: counter (caller's counter, row, action dimension) */
#define ORC_DOMAIN_PERM 3       /* minibatch permutations */

void orc_reset(const orc_config* cfg, orc_state* st, const float* init_pose, const uint8_t* mask);
/* Normal draws per robot and step in the noise input: 5, plus R with range noise. */
int32_t orc_noise_width(const orc_config* cfg);
/* The paper's reward, Eq. (7) with Eqs. (8)-(17), from its inputs (all FP64). */
double orc_paper_reward(const orc_config* cfg, int collided, double delta_cells, double u_prev, double u,
                        double d_min);
/* Q16 cells of a coordinate: rint(v * (float)(65536 / c)) in FP32, clamped to +-1e9 (as the step). */
int64_t orc_to_q16(float v, float cell_m);
/* U_t = cbrt(det Sigma) of the 6 unique FP32 entries (0 if det <= 0), as the reward uses it. */
double orc_uncertainty(const float* c6);
/* One step of every robot.  noise: caller's normals [n, orc_noise_width], or
 * NULL to draw them: normal k of robot r is orc_normal(noise_seed, ORC_DOMAIN_ENV,
 * draws[r], r, k).  Either way draws[r] grows by one. */
void orc_step(const orc_config* cfg, orc_state* st, const float* actions, const float* noise,
              orc_out* out, int32_t n_threads);
/* Observation.  With reward_mode 1 and u_new != NULL the uncertainty entry is
 * the bridged U of the fine-tuning wrapper (Sec. III-G, Eqs. 21-22): alpha * U_new + (1 - alpha) * U_t,
 * alpha = min(1, t / T_bridge) given by the caller. */
void orc_observe(const orc_config* cfg, const orc_state* st, const float* ranges, int16_t* crop,
                 int32_t crop_side, float* scan, float* state12, const float* u_new, double alpha);

#ifdef __cplusplus
}
#endif
#endif
