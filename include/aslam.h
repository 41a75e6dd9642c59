/*
 * aslam.h -- C-ABI of the MI355X (gfx950) batched Active-SLAM hot path.
 *
 * Method: "Massive Parallel Deep Reinforcement Learning for Active SLAM"
 * (arXiv 2603.25834).  The environment step follows the POMDP statement of
 * Sec. III-B (Eqs. 1-2): at each step the agent applies a_t = (v, w) from the
 * continuous action space of Sec. III-C (Eq. 4), the simulator moves every
 * robot, the SLAM backbone of Sec. III-D integrates the LiDAR scan into a
 * 2-D log-odds occupancy grid and propagates the pose covariance, and the
 * reward of Sec. III-E (collision penalty of Eq. 7) combined with an
 * uncertainty term is returned with the next observation.  The policy calls
 * implement the PPO actor-critic of Sec. III-F (Eqs. 18-20).
 *
 * Conventions for every call:
 *   - Return value: ASL_OK (0) or a negative ASL_E* code; aslam_last_error()
 *     returns a thread-local message describing the last failure.  On error
 *     the handle's state is unchanged.
 *   - "dev" pointers are device (HBM) pointers owned by the caller; "host"
 *     pointers are read during the call only.  The library owns the state
 *     behind each handle and frees it in the matching destroy call.
 *   - Every device-side call is asynchronous on the given HIP stream (NULL =
 *     the legacy default stream), allocates nothing and never synchronises
 *     the host, so it can be captured into a HIP graph.
 *   - Units: metres, radians, seconds.  A robot's world frame has its origin
 *     at the lower-left corner of its grid; cell (i, j) covers
 *     [i c, (i+1) c) x [j c, (j+1) c); grids are square, side s_i cells,
 *     s_i a multiple of 32 in [32, 4096].  Row-major cell index j*s + i.
 *   - Ragged per-robot buffers are concatenated in robot order without gaps.
 */
#ifndef ASLAM_H
#define ASLAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASL_OK 0
#define ASL_EINVAL (-1)   /* invalid argument (null pointer, bad size or config) */
#define ASL_ENOMEM (-2)   /* device or host allocation failed (create calls only) */
#define ASL_EHIP (-3)     /* a HIP runtime call failed; the HIP error text is in the message */
#define ASL_ESTATE (-4)   /* call not valid in the current state (e.g. step before reset) */
#define ASL_ENOTIMPL (-5) /* feature not built */

typedef struct hipStream_t_opaque* aslam_stream_t; /* a hipStream_t */

/* ------------------------------------------------------------------ env */

typedef struct aslam_env aslam_env;

/* Environment parameters.  Sec. IV-A fixes the sensor as a LiDAR ray fan with
 * a maximum range; Sec. III-C fixes the action box; the remaining fields are
 * the workload's choices (odometry noise, initial covariance, loop-closure
 * and log-odds constants, reward weights). */
typedef struct {
  int32_t n_rays;       /* R rays over 360 deg, ray 0 along the heading, counter-clockwise; R divides 46080 */
  int32_t loop_closure; /* 1: EKF position fix when a robot returns to its first visit of a coarse cell */
  int32_t lc_gap;       /* steps required since that first visit and since the last fix */
  int32_t episode_len;  /* steps per episode for `done`; 0 = unbounded */
  float cell_m;         /* cell side c (m), > 0 */
  float r_max_m;        /* LiDAR max range (m), > 0, <= 4096 cells */
  float dt;             /* control period (s) */
  float v_max, w_max;   /* action box [0, v_max] x [-w_max, w_max] (Eq. 4) */
  float sigma_x, sigma_y, sigma_th; /* odometry noise std per step (world frame) */
  float var0_xy, var0_th;           /* initial covariance diagonal */
  float lc_cell_m, lc_radius_m, lc_sigma_m; /* visit cell (m; also the novelty cell of Eq. 9), fix radius (m), fix std (m) */
  float l_hit, l_miss, l_clamp;     /* log-odds increments and clamp (nats); stored in 1/256 nat */
  float w_entropy, w_dopt, lambda_col; /* reward = w_entropy*dH - w_dopt*ln det(Sigma) - lambda_col*collided */
  /* Sensor, collision and reward of the paper (Sec. IV-A, Eq. 7).  All zero
   * keeps the full-circle noiseless scan and the entropy / D-opt reward. */
  int32_t fov_steps;    /* fan width in heading steps (46080 = 360 deg); 0 or 46080 = full circle from the
                           heading; else rays start at heading - fov/2; n_rays must divide the fan */
  int32_t reward_mode;  /* 0: entropy / D-opt reward above; 1: Eq. (7) with the observation of Eq. (3) */
  float r_min_m;        /* reported ranges are clamped to [r_min, r_max] (with the sensor model) */
  float range_sigma_m;  /* range noise std (m); > 0 adds n_rays normal draws per robot to the noise row */
  float range_quant_m;  /* reported ranges rounded to this quantum (m); 0 = no rounding */
  float d_crash_m;      /* > 0: collided when an occupied or off-grid cell is closer than this (<= 32 cells) */
  float d_full_m;       /* Eq. 15: the positive reward terms reach full weight at this clearance (> d_crash) */
  float lambda_explore, lambda_abs, lambda_delta; /* Eqs. 8, 13, 14 */
  float u_hi, kappa;    /* Eq. 11 uncertainty gate, Eq. 12 saturation drop (both > 0 in mode 1) */
  uint64_t noise_seed;  /* key of the step's own normal draws (env_step with noise_dev NULL) */
  /* SLAM backend (Sec. III-D).  0: the EKF above.  1: the fixed-lag graph in the loop (needs
   * reward_mode 1 and loop_closure 0), per robot and step:
   *   - the predicted pose (the previous estimate moved by the commanded motion, as the EKF mean) is
   *     the centre of a correlative search (aslam_csm_match's rules) of the scan -- the reported
   *     ranges of the rays whose true march hit, Q16 -- over the robot's log-odds grid;
   *   - alignment: with match weight w = q m > 0 (aslam_csm_factor's rule, l_max = l_clamp in 1/256)
   *     the aligned pose is the best candidate, else the prediction; the estimate becomes the aligned
   *     pose, x = ax c / 65536, y likewise, theta = wrap(2 pi h / 46080) in FP64, stored in FP32;
   *   - the window of the last lag_len poses (FP64): a prior on the oldest, odometry factors (the
   *     commanded (d, 0, phi) in the earlier pose's frame, 0 when blocked, information 1/sigma^2 of the
   *     odometry noise), a scan factor on each added pose (the aligned pose, information
   *     w (1/s_xy^2, 1/s_xy^2, 1/s_th^2)); a full window drops its oldest pose and the next one takes
   *     as prior its estimate with the inverse covariance diagonal it had as the newest; after a reset
   *     the window is the initial pose with the prior (pose, 1/var0);
   *   - gn_iters Gauss-Newton steps (aslam_fixedlag_solve's rules) from the last estimates and the
   *     aligned pose; the newest pose's covariance becomes the state's Sigma (FP32), U_t = cbrt(det);
   *   - the scan is integrated from the aligned pose (aslam_csm_integrate's rules) with weight
   *     w_q = rint(256 (f + (1 - f) w)), f = int_weight_floor;
   *   - reward Eq. (7) with U_{t-1}, U_t; the map entropy is not tracked.
   * The step is a sequence of launches in every exec form (threads per robot from the exec config). */
  int32_t slam_backend;
  int32_t lag_len;        /* poses in the window, 2..64 */
  int32_t gn_iters;       /* Gauss-Newton steps per env step, 0..100 */
  int32_t csm_W, csm_V;   /* lattice half-widths (translation, heading), 0..8, (2 csm_V + 1) n_rays <= 8192 */
  int32_t csm_step_xy_q;  /* lattice translation step, Q16 cells, 1..2^20 */
  int32_t csm_step_h;     /* lattice heading step, table steps, 0..46080 */
  float scan_sigma_xy_m, scan_sigma_th; /* scan-factor standard deviations (> 0) */
  float int_weight_floor; /* integration weight floor f in [0, 1] */
} aslam_env_config;

/* Standard-normal draws per robot in the step's noise row: 5 (odometry x,
 * y, theta, loop-closure x, y), plus n_rays range draws when range_sigma_m
 * > 0.  Returns -1 for a NULL handle.
 *
 * The library's own draws (env_step with noise_dev NULL): draw k of robot r
 * at a step is the Irwin-Hall(12) normal of one Philox4x64-10 block (Salmon
 * et al., SC'11) at counter (c_r, r, k, 0) under key (noise_seed, 1), where c_r
 * counts the robot's env_step calls since create (resets keep it): the sum of
 * the block's twelve 21-bit fields (bits 63..43, 42..22, 21..1 of each word)
 * minus 6 (2^21 - 1), times 2^-21 (exact in FP32; mean 0, variance 1 - 2^-42).
 * A stand-in for the Gaussian odometry and range noise (Sec. IV-A) that any
 * implementation reproduces bit for bit. */
int32_t aslam_env_noise_width(const aslam_env* env);

/* Execution form of env_step.  PLAIN issues one launch per stage (motion and
 * EKF, LiDAR march, map update and reward); FUSED issues one persistent launch
 * that pulls robots in largest-grid-first order and keeps the per-ray results
 * in LDS. */
#define ASLAM_FORM_PLAIN 0
#define ASLAM_FORM_FUSED 1

typedef struct {
  int32_t form;          /* ASLAM_FORM_* */
  int32_t threads;       /* threads per workgroup: 128, 192, 256, 384 or 512 */
  int32_t band_rows;     /* rows of the LDS code window per pass (>= 8); 0 = as many as fit */
  int32_t grid;          /* FUSED: workgroups launched; 0 = one per robot */
  int32_t record_rays;   /* FUSED: also write per-ray rho_q / hit_cell to the state (PLAIN always does) */
  int32_t lds_bytes;     /* LDS budget per workgroup; 0 = device maximum */
  int32_t mark_seg;      /* map update's walk: 0 = one lane per ray; k in [8, 1024] = the rays cut into
                            segments of k steps shared out over the lanes (results are identical) */
} aslam_exec_config;

/* Create n_robots environments.  sides_host[n_robots]: grid side of each
 * robot.  Allocates all device state (worlds, beliefs, poses, covariances,
 * visit grids, per-ray buffers) on the current device.  Errors: ASL_EINVAL,
 * ASL_ENOMEM, ASL_EHIP. */
int aslam_env_create(const aslam_env_config* cfg, int32_t n_robots, const int32_t* sides_host,
                     aslam_env** out);
int aslam_env_destroy(aslam_env* env);

/* Device-state sizes, for callers that export or import state. */
int64_t aslam_env_world_words(const aslam_env* env); /* sum s_i^2 / 32 */
int64_t aslam_env_cells(const aslam_env* env);       /* sum s_i^2 */
int64_t aslam_env_visit_cells(const aslam_env* env); /* sum v_i^2 (visit grids), 0 when none is kept */

int aslam_env_set_exec(aslam_env* env, const aslam_exec_config* ex);
int aslam_env_get_exec(const aslam_env* env, aslam_exec_config* ex);

/* Start (or restart) episodes.  world_dev: uint32 occupancy bits, cell (i,j)
 * of robot r at bit (j*s+i) of its slice (little-endian words), all robots
 * concatenated.  init_pose_dev: float [n,3] (x, y, theta), inside a free
 * cell.  mask_dev: uint8 [n], non-zero = reset this robot; NULL = all.
 * Reset robots get a blank belief (log-odds 0), the estimate equal to the
 * initial pose, covariance diag(var0_xy, var0_xy, var0_th), step 0 and an
 * empty visit grid. */
int aslam_env_reset(aslam_env* env, const uint32_t* world_dev, const float* init_pose_dev,
                    const uint8_t* mask_dev, aslam_stream_t stream);

/* One environment step for every robot (Sec. III-B, one POMDP transition).
 *   actions_dev float [n,2] (v, w), clamped to the box; NaN -> 0.
 *   noise_dev   float [n,G] standard-normal draws, G = aslam_env_noise_width:
 *               odometry x, y, theta, the loop-closure measurement x, y, then
 *               (with range noise) one draw per ray; NULL = the library's own
 *               draws (above).  Either way each robot's draw counter moves on.
 *   ranges_dev  float [n,R] out: range (m) to the entry face of the first
 *               occupied cell, r_max when none within range; with the sensor
 *               model, plus noise, rounded to the quantum and clamped to
 *               [r_min, r_max].  The map update walks the reported range.
 *   reward_dev  float [n]   out.
 *   done_dev    uint8 [n]   out: collided this step (swept into an occupied
 *               cell, or within d_crash of one), or episode length reached.
 * Errors: ASL_EINVAL (null pointer), ASL_ESTATE (before the first reset). */
int aslam_env_step(aslam_env* env, const float* actions_dev, const float* noise_dev, float* ranges_dev,
                   float* reward_dev, uint8_t* done_dev, aslam_stream_t stream);

/* Observation for the policy from the current state and the last ranges:
 *   crop_dev  int16 [n,crop,crop]: belief log-odds (1/256 nat) in an
 *             axis-aligned window centred on the estimated cell, 0 off-map.
 *   scan_dev  float [n,R]: ranges / r_max.
 *   state_dev float [n,12]: x/(s c), y/(s c), theta/pi, Sigma (9, row-major);
 *             reward_mode 1 (Eq. 3): true yaw/pi, U_t = cbrt(det Sigma), 0 x 10. */
int aslam_env_observe(aslam_env* env, const float* ranges_dev, int16_t* crop_dev, int32_t crop,
                      float* scan_dev, float* state_dev, aslam_stream_t stream);

/* Observation with the uncertainty bridge of the fine-tuning wrapper
 * (Sec. III-G, Eqs. 21-22): as aslam_env_observe in reward_mode 1, with the
 * uncertainty entry alpha * U_new + (1 - alpha) * U_t, alpha = min(1, t / t_bridge),
 * formed in FP64.  u_new_dev float [n]: the external estimator's uncertainty
 * per robot; t >= 0 fine-tuning steps so far, t_bridge >= 1.  ASL_EINVAL for
 * reward_mode 0 (its observation carries no U_t) or bad t / t_bridge. */
int aslam_env_observe_bridge(aslam_env* env, const float* ranges_dev, int16_t* crop_dev, int32_t crop,
                             float* scan_dev, float* state_dev, const float* u_new_dev, int64_t t,
                             int64_t t_bridge, aslam_stream_t stream);

/* Copy a state field into caller memory (device), for checks and export. */
#define ASLAM_FIELD_BELIEF 0     /* int16 [sum s^2] */
#define ASLAM_FIELD_POSE 1       /* float [n,3] true pose */
#define ASLAM_FIELD_EST 2        /* float [n,3] estimate */
#define ASLAM_FIELD_COV 3        /* float [n,6] xx, xy, xt, yy, yt, tt */
#define ASLAM_FIELD_RHO_Q 4      /* int32 [n,R] range in 1/65536 cell */
#define ASLAM_FIELD_HIT_CELL 5   /* int32 [n,R] j*s+i of the hit cell, -1 none */
#define ASLAM_FIELD_ENTROPY_Q 6  /* int64 [n] map entropy in 2^-32 nat */
#define ASLAM_FIELD_STEP 7       /* int32 [n] steps since reset */
#define ASLAM_FIELD_FLAGS 8      /* uint8 [n,2] collided, loop closure fired (last step) */
#define ASLAM_FIELD_TERMS 9      /* float [n,2] entropy decrease (nats), ln det Sigma (last step) */
#define ASLAM_FIELD_COUNTERS 10  /* int64 [n,3] since reset: coded (updated) cells, LiDAR-march cell
                                    visits, map-update cell visits -- the work measures of the step */
#define ASLAM_FIELD_U_PREV 11    /* double [n] U of the last step (reward_mode 1), cbrt(det Sigma) */
#define ASLAM_FIELD_VISIT_LAST 12 /* int32 [sum v_i^2] last step each visit cell held the robot, -1 never
                                     (v_i = ceil(s_i c / lc_cell_m); loop closure or reward_mode 1) */
#define ASLAM_FIELD_DRAWS 13     /* uint64 [n] env_step calls since create (the draw counter) */
#define ASLAM_FIELD_MATCH 14     /* int32 [n,6] the last step's scan match (slam_backend 1), as aslam_csm_match */
int aslam_env_read(const aslam_env* env, int32_t field, void* dst_dev, aslam_stream_t stream);

/* HIP graph of K consecutive env_step calls.  Step k reads
 * actions_dev + k*a_stride, noise_dev + k*g_stride and writes
 * ranges_dev + k*r_stride, reward_dev + k*w_stride, done_dev + k*d_stride
 * (strides in elements; 0 = same buffer every step).  noise_dev NULL: every
 * step takes the library's own draws, whose counters live on the device, so
 * each replay draws new numbers.  The graph is instantiated once and replayed
 * with aslam_env_graph_launch. */
int aslam_env_graph_build(aslam_env* env, int32_t k_steps, const float* actions_dev, int64_t a_stride,
                          const float* noise_dev, int64_t g_stride, float* ranges_dev, int64_t r_stride,
                          float* reward_dev, int64_t w_stride, uint8_t* done_dev, int64_t d_stride);
int aslam_env_graph_launch(aslam_env* env, aslam_stream_t stream);

/* --------------------------------------------------------------- policy */

/* PPO actor-critic (Sec. III-F; Eqs. 18-20) with the workload's network:
 * conv 1->16 and 16->32 (3x3, stride 2, padding 1, ReLU) on the 64x64 belief
 * crop (input L/256), the 8192 features (channel-major, as c*256 + y*16 + x)
 * concatenated with scan[R] and state[12], FC 256 + ReLU, FC 256 + ReLU, mean
 * head (2), value head (1), state-independent log std (2).
 *
 * Parameters and gradients are FP32 flat vectors, in this order (row-major
 * tensors): conv1.w [16,1,3,3], conv1.b [16], conv2.w [32,16,3,3], conv2.b
 * [32], fc1.w [256, 8192+R+12], fc1.b [256], fc2.w [256,256], fc2.b [256],
 * mu.w [2,256], mu.b [2], v.w [1,256], v.b [1], log_std [2].
 * GEMM operands are rounded to BF16 and accumulated in FP32 (MFMA);
 * activations between layers are BF16; heads, loss and reductions are FP32. */
typedef struct aslam_policy aslam_policy;

typedef struct {
  int32_t n_scan;     /* R, scan length */
  int32_t max_batch;  /* largest batch passed to forward / backward (sizes the workspaces) */
  float clip_eps;     /* PPO clip epsilon (Eq. 19) */
  float c_value;      /* value-loss weight */
  float c_entropy;    /* entropy-bonus weight */
  int32_t recurrent;  /* 1: the GRU of Sec. III-F ("Recurrent Layer", 256 units) in place of FC2, layout
                         below; such a handle takes aslam_policy_act_rnn / _backward_seq only */
  int32_t precision;  /* 0: BF16 operands with FP32 accumulation throughout.  1 (feed-forward only):
                         split forward -- every operand v of the four forward products (crop, weights,
                         activations, scan and state) is the pair hi = bf16(v), lo = bf16(v - hi), and
                         each product is hi*hi + hi*lo + lo*hi on MFMA with FP32 accumulation, so the
                         ReLU pre-activations are FP32-accurate (the forward and its recomputation in
                         the backward cost about three times the MFMA work); the backward's products
                         stay BF16.  This is the mode whose gradients agree with the exact FP64
                         network to 1e-2 per tensor on random minibatches. */
} aslam_policy_config;

/* Number of parameters for scan length n_scan (2,264,005 for R = 360), feed-forward layout. */
int64_t aslam_policy_num_params(int32_t n_scan);
/* Number of parameters of either layout (-1 for a bad config).  The recurrent
 * layout replaces fc2.w, fc2.b by gru.w_ih [768,256], gru.w_hh [768,256],
 * gru.b_ih [768], gru.b_hh [768] (gate rows reset, update, new). */
int64_t aslam_policy_param_count(const aslam_policy_config* cfg);
/* Allocates the minibatch workspaces (about 100 KB per sample of max_batch). */
int aslam_policy_create(const aslam_policy_config* cfg, aslam_policy** out);
int aslam_policy_destroy(aslam_policy* pol);

/* Forward pass: crop_dev int16 [B,64,64], scan_dev float [B,R], state_dev
 * float [B,12] -> mu_dev float [B,2], value_dev float [B].  The log std is
 * params[last 2].  1 <= B <= max_batch. */
int aslam_policy_forward(aslam_policy* pol, const float* params_dev, const int16_t* crop_dev, const float* scan_dev,
                         const float* state_dev, int32_t batch, float* mu_dev, float* value_dev,
                         aslam_stream_t stream);

/* Forward pass that allocates nothing, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc).  Same kernels and results as
 * aslam_policy_forward (bit for bit) without a handle: params_dev is the feed-forward layout for
 * n_scan, inputs and outputs as aslam_policy_forward.  What the forward stages between its kernels
 * (weight copies, FC1 input rows, split-K partial sums) lives in one static device array of the
 * library, sized for n_scan <= 720 and batch <= 256 (about 18 MB per GPU, held until the process ends;
 * the first call on a device looks up its address, no allocation).  Every call on a GPU shares that
 * array: calls that overlap on one GPU (other streams, other host threads) race and must be ordered by
 * the caller.  ASL_EINVAL on NULL pointers, n_scan outside [1, 720] or batch outside [1, 256]. */
int aslam_policy_forward_noalloc(const float* params_dev, int32_t n_scan, const int16_t* crop_dev,
                                 const float* scan_dev, const float* state_dev, int32_t batch, float* mu_dev,
                                 float* value_dev, aslam_stream_t stream);
/* The limits of aslam_policy_forward_noalloc (largest n_scan and batch, written if not NULL); returns
 * the size of its static device array in bytes. */
int64_t aslam_policy_noalloc_limits(int32_t* max_scan, int32_t* max_batch);

/* BF16 copies of the weights that the forward reads (FC1 and FC2), formed
 * from params_dev into the handle.  aslam_policy_forward, _act (prepared = 0)
 * and _backward form them themselves; a caller whose parameters do not change
 * between calls (a rollout) prepares once and passes prepared = 1 to
 * aslam_policy_act. */
int aslam_policy_prepare(aslam_policy* pol, const float* params_dev, aslam_stream_t stream);

/* Rollout step of the actor (Sec. III-F): the forward pass and the Gaussian
 * action sample in one call.  Inputs as aslam_policy_forward; eps_dev [B,2]
 * standard normals drawn by the caller, or NULL for the library's own: the
 * normal of row b, dimension d is the Irwin-Hall(12) value of the Philox4x64-10
 * block at counter (counter, b, d, 0) under key (seed, 2) (the generator
 * described at aslam_env_noise_width).  Writes value_dev [B], act_dev [B,2],
 * logp_dev [B] and, if mu_dev is not NULL, mu_dev [B,2]; the results equal
 * aslam_policy_forward followed by aslam_policy_sample bit for bit.
 * prepared = 1 uses the weight copies of the last prepare, forward, act or
 * backward call on this handle: the caller guarantees that params_dev has not
 * changed since (ASL_ESTATE if no such call was made); prepared = 0 forms
 * them first. */
int aslam_policy_act(aslam_policy* pol, const float* params_dev, int32_t prepared, const int16_t* crop_dev,
                     const float* scan_dev, const float* state_dev, int32_t batch, const float* eps_dev,
                     uint64_t seed, uint64_t counter, float* mu_dev, float* value_dev, float* act_dev,
                     float* logp_dev, aslam_stream_t stream);

/* PPO loss and its gradient over one minibatch, recomputing the forward
 * activations (only the inputs are stored across the rollout).
 *   loss = L_clip + c_value * mean((V - ret)^2) - c_entropy * H[pi],
 *   L_clip = -mean(min(r A, clip(r, 1-eps, 1+eps) A)), r = exp(logp - old_logp).
 * act_dev [B,2], old_logp_dev/adv_dev/ret_dev [B].  grads_dev [P] is ADDED
 * to (accumulate over minibatches; zero it first).  loss_dev float [4] out:
 * total, L_clip, mean((V-ret)^2), entropy. */
int aslam_policy_backward(aslam_policy* pol, const float* params_dev, const int16_t* crop_dev,
                          const float* scan_dev, const float* state_dev, int32_t batch, const float* act_dev,
                          const float* old_logp_dev, const float* adv_dev, const float* ret_dev, float* grads_dev,
                          float* loss_dev, aslam_stream_t stream);

/* The same over the rows rows_dev[0 .. batch-1] (int32, device) of rollout-sized
 * arrays: sample b of the minibatch is row rows_dev[b] of crop_dev, scan_dev,
 * state_dev, act_dev, old_logp_dev, adv_dev and ret_dev, so a shuffled
 * minibatch needs no gathered copy.  Rows are not checked against the arrays'
 * size: the caller guarantees 0 <= rows_dev[b] < their row count. */
int aslam_policy_backward_rows(aslam_policy* pol, const float* params_dev, const int16_t* crop_dev,
                               const float* scan_dev, const float* state_dev, const int32_t* rows_dev, int32_t batch,
                               const float* act_dev, const float* old_logp_dev, const float* adv_dev,
                               const float* ret_dev, float* grads_dev, float* loss_dev, aslam_stream_t stream);

/* Recurrent rollout step (Sec. III-F, a single-layer GRU of 256 units):
 *   r = sigmoid(W_ir x + b_ir + W_hr h + b_hr), z = sigmoid(W_iz x + b_iz + W_hz h + b_hz),
 *   n = tanh(W_in x + b_in + r (W_hn h + b_hn)), h' = (1 - z) n + z h,
 * x = the FC1 output, h = h_in_dev [B,256] FP32 row b, or 0 where first_dev[b]
 * (uint8 [B], may be NULL) marks the first step of an episode.  Writes the new
 * state h_out_dev [B,256] (may alias h_in_dev) and, from the heads on h', as
 * aslam_policy_act: value_dev, act_dev, logp_dev and mu_dev if not NULL
 * (eps_dev, seed, counter as there).  prepared as in aslam_policy_act.  BF16 products with FP32 accumulation;
 * gate math and state in FP32. */
int aslam_policy_act_rnn(aslam_policy* pol, const float* params_dev, int32_t prepared, const int16_t* crop_dev,
                         const float* scan_dev, const float* state_dev, int32_t batch, const float* h_in_dev,
                         const uint8_t* first_dev, const float* eps_dev, uint64_t seed, uint64_t counter,
                         float* mu_dev, float* value_dev, float* act_dev, float* logp_dev, float* h_out_dev,
                         aslam_stream_t stream);

/* PPO loss and its gradient for the recurrent policy over whole sequences,
 * with backpropagation through time.  The rollout arrays are time-major:
 * crop_dev [T,N,64,64], scan_dev [T,N,R], state_dev [T,N,12], act_dev [T,N,2],
 * old_logp_dev / adv_dev / ret_dev [T,N], first_dev uint8 [T,N] (step t of
 * robot n starts an episode: its state is zeroed before the step), h0_dev
 * [N,256] the state entering step 0.  The minibatch is the nb robots
 * robots_dev[0 .. nb-1] (int32, device) over all T steps: T * nb samples,
 * at most max_batch; the loss is the mean over them.  grads_dev is ADDED to;
 * loss_dev [4] as aslam_policy_backward. */
int aslam_policy_backward_seq(aslam_policy* pol, const float* params_dev, const int16_t* crop_dev,
                              const float* scan_dev, const float* state_dev, int32_t T, int32_t N,
                              const int32_t* robots_dev, int32_t nb, const float* h0_dev, const uint8_t* first_dev,
                              const float* act_dev, const float* old_logp_dev, const float* adv_dev,
                              const float* ret_dev, float* grads_dev, float* loss_dev, aslam_stream_t stream);

/* Generalized Advantage Estimation (Sec. III-F) over a [T,N] rollout (time-major):
 *   delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t,  A_t = delta_t + gamma lam (1 - d_t) A_{t+1},
 * V_T = last_value_dev [N].  Writes adv_dev and ret_dev = adv + values, [T,N] float. */
int aslam_gae(const float* rewards_dev, const float* values_dev, const uint8_t* dones_dev,
              const float* last_value_dev, int32_t T, int32_t N, float gamma, float lam, float* adv_dev,
              float* ret_dev, aslam_stream_t stream);

/* One Adam step (bias-corrected, step >= 1) on n FP32 parameters, in place. */
int aslam_adam(float* params_dev, const float* grads_dev, float* m_dev, float* v_dev, int64_t n, int32_t step,
               float lr, float beta1, float beta2, float eps, aslam_stream_t stream);

/* Action sampling of the Gaussian policy (Sec. III-F): act = mu + exp(log_std) * eps and
 * logp = sum_d [-eps_d^2 / 2 - log_std_d - ln(2 pi) / 2], the log-density of act.  mu_dev and eps_dev
 * are [batch,2] float (eps: standard normals drawn by the caller, or NULL for the library's own at
 * (seed, counter) as in aslam_policy_act), log_std is read from params_dev; act_dev [batch,2] and
 * logp_dev [batch] are written.  The env step clamps actions to its box. */
int aslam_policy_sample(aslam_policy* pol, const float* params_dev, const float* mu_dev, const float* eps_dev,
                        uint64_t seed, uint64_t counter, int32_t batch, float* act_dev, float* logp_dev,
                        aslam_stream_t stream);

/* Keyed permutation of [0, n) for PPO's shuffled minibatches (Sec. III-F): out_dev int32 [n],
 * out[j] = the image of j under an 8-round balanced Feistel network on the smallest even bit width
 * b >= 2 with 2^b >= n (halves of b/2 bits; round i maps (l, r) to (r, l ^ f), f = the low b/2 bits of
 * word 0 of the Philox4x64-10 block at counter (counter, r, i, 0) under key (seed, 3)), applied again
 * while the image is >= n (cycle walking).  A bijection for every key.  ASL_EINVAL on n < 0 or a NULL
 * out_dev with n > 0. */
int aslam_permutation(int32_t n, uint64_t seed, uint64_t counter, int32_t* out_dev, void* work_dev,
                      int64_t work_bytes, aslam_stream_t stream);

/* Bytes of the optional device workspace of aslam_permutation: 4 * 2^b (at most 16 n for n >= 1), 0
 * for n <= 0.  With a workspace (4-byte aligned, at least this size, caller-owned, overwritten) the
 * call tabulates the Feistel image of the whole 2^b domain in one pass and walks the cycles through
 * that table -- the same permutation, without each lane evaluating its whole walk; with
 * work_dev = NULL each element walks its cycle by itself.  ASL_EINVAL on a short or misaligned
 * workspace. */
int64_t aslam_permutation_work_bytes(int32_t n);

/* Row gather for minibatch assembly: dst row i = src row idx_dev[i], i < n, rows of row_bytes bytes
 * (a multiple of 4; src and dst 4-byte aligned).  Indices are not checked against the source size:
 * the caller guarantees 0 <= idx < rows of src.  ASL_EINVAL on NULL pointers or bad sizes. */
int aslam_gather_rows(const void* src_dev, int64_t row_bytes, const int32_t* idx_dev, int32_t n, void* dst_dev,
                      aslam_stream_t stream);

/* ------------------------------------------------------------------ fixed-lag SLAM backbone
 *
 * The pose estimator of Sec. III-D as batched calls: correlative scan matching of each robot's scan
 * against its log-odds grid, the scan factor of the match, the confidence-weighted integration of the
 * aligned scan into the grid, and the Gauss-Newton solve of a sliding window of poses with the newest
 * pose's covariance.  The paper gives the method but not its
 * constants or exact rules; the rules below are this library's reading of it. */

/* The backbone's handle: the 46080-entry direction table (cos and sin of 2 pi k / 46080 rounded to
 * Q14) on the device current at create (180 KB).  Created and destroyed outside any stream capture;
 * the scan-matching and integration calls only read it, so they allocate nothing and never
 * synchronise (they can be captured into a HIP graph).  Errors: ASL_EINVAL (NULL out), ASL_ENOMEM,
 * ASL_EHIP.  A call with a handle of another device returns ASL_ESTATE. */
typedef struct aslam_slam aslam_slam;
int aslam_slam_create(aslam_slam** out);
int aslam_slam_destroy(aslam_slam* slam);

typedef struct {
  int32_t W;          /* translation half-width of the candidate lattice, in steps, 0..8 */
  int32_t V;          /* heading half-width, in steps, 0..8 */
  int32_t step_xy_q;  /* translation step, Q16 cells (65536 = one cell), 1..2^20 */
  int32_t step_h;     /* heading step, in steps of the 46080-per-turn heading table, 0..46080 */
} aslam_csm_config;

/* Correlative scan matching (Sec. III-D: candidate poses on a discrete lattice around the prediction,
 * each scored on the log-odds grid) for n robots, one workgroup each, exact integer arithmetic.
 *   belief_dev   int16 log-odds; robot r's s x s grid starts at element cell_off_dev[r] (int64 [n]),
 *                cell (cx, cy) at cy * s + cx, s = side_dev[r] (int32 [n]);
 *   pose_q_dev   int32 [n,3]: predicted pose, x and y in Q16 cells, heading index in [0, 46080);
 *   rho_q_dev    int32 [n,R]: ray ranges in Q16 cells, < 0 = no return;
 *   a_off_dev    int32 [R]: ray heading offsets (table steps) relative to the robot heading.
 * The endpoint of ray q under pose (x, y, h) is x + ((rho * cos_q) >> 14), y + ((rho * sin_q) >> 14)
 * with (cos_q, sin_q) the Q14 table direction of (h + a_off) mod 46080 (cos, sin of 2 pi k / 46080
 * rounded to the nearest 1/16384); its cell is (ex >> 16, ey >> 16).  Candidate (i, j, k), |i|,|j| <= W,
 * |k| <= V, is (x + i step_xy_q, y + j step_xy_q, h + k step_h); its score is the int32 sum of the
 * log-odds of its rays' endpoint cells inside the grid.  out_dev int32 [n,6]: best i, j, k (highest
 * score, lowest index ((k+V)(2W+1) + j+W)(2W+1) + i+W on ties), best score, second score (highest at
 * lattice Chebyshev distance >= 2 from the best; INT32_MIN if none), rays with a return.
 * max_side: the largest side (a host value): lattices of at most 1024 candidates stage in LDS the part
 * of each grid that the candidates' endpoints can reach, with room sized for a whole grid of this side
 * when that fits beside the ray offsets; a larger part is staged in bands of rows, and a robot whose
 * part has rows wider than that room, or whose centre or ray offsets lie beyond 2^28 / 2^29 (Q16),
 * reads global memory (results do not depend on it).
 * Device arrays are not checked: the caller guarantees grids inside belief_dev, 0 <= rho_q < 2^31.
 * ASL_EINVAL on NULL pointers, n < 0 or a config outside the ranges above, or (2V + 1) R > 8192. */
int aslam_csm_match(const aslam_slam* slam, const int16_t* belief_dev, const int64_t* cell_off_dev,
                    const int32_t* side_dev, int32_t max_side, int32_t n, const int32_t* pose_q_dev, const int32_t* rho_q_dev, int32_t R,
                    const int32_t* a_off_dev, const aslam_csm_config* cfg, int32_t* out_dev, aslam_stream_t stream);

/* The scan factor of a match (Sec. III-D: an absolute pose measurement whose information is scaled
 * by the normalised score and the ambiguity margin).  match_dev int32 [n,6] (aslam_csm_match's output),
 * pose_q_dev the poses it was matched around.  meas_dev double [n,3]: the best candidate in metres /
 * radians (theta wrapped to [-pi, pi]); info_dev double [n,3]: the information diagonal
 * w (1 / sigma_xy^2, 1 / sigma_xy^2, 1 / sigma_th^2), w = q m, q = clamp(best / (rays * l_max), 0, 1),
 * m = clamp((best - second) / max(best, 1), 0, 1).  ASL_EINVAL on NULL pointers or non-positive scales. */
int aslam_csm_factor(const int32_t* match_dev, const int32_t* pose_q_dev, int32_t n, const aslam_csm_config* cfg,
                     double cell_m, double l_max, double sigma_xy, double sigma_th, double* meas_dev,
                     double* info_dev, aslam_stream_t stream);

/* Confidence-weighted map integration (Sec. III-D: the aligned scan enters the grid with a weight that
 * grows with the match score) for n robots, one workgroup each, in place on belief_dev (layout as for
 * aslam_csm_match).  The aligned pose is pose_q_dev[r] moved by match_dev[r]'s lattice offsets
 * (i step_xy_q, j step_xy_q, k step_h); the weight w = q m as in aslam_csm_factor, quantised to
 * w_q = rint(256 w).  With match_dev NULL the pose is pose_q_dev[r] itself and w_q = 256 (cfg and l_max
 * are then unused).  Each ray walks from the aligned position along the Q14 table direction of
 * (heading + a_off_dev[q]) mod 46080 with the exact traversal of the env step: a cell is visited when
 * its entry distance is within the range (rho_q_dev, Q16 cells; rays with rho < 0 have no return and
 * walk rmax_q), an x crossing before a y crossing at equal distance, stopping at the grid's edge.
 * Visited cells are MISS; the last cell of a ray with a return that stopped at its range is HIT (HIT
 * beats MISS).  Each coded cell gets one add, L <- clamp(L + floor((w_q l + 128) / 256), -l_clamp,
 * l_clamp), l = l_hit or l_miss (log-odds units of the grid).  An aligned position outside the grid
 * leaves it unchanged.  coded_dev int32 [n] (may be NULL): coded cells per robot (-1: side above 32768,
 * grid left unchanged).  max_side: the largest side (a host value) sizes the LDS bitmaps so that such a
 * grid is one band of rows (at most 64 KB; larger grids take several bands; results do not depend on
 * it).  The result does not depend on ray order.  Device arrays are not checked (the caller guarantees
 * grids inside belief_dev).  ASL_EINVAL on NULL pointers, n < 0, max_side < 0, R outside [1, 65536],
 * rmax_q < 0, l_clamp outside [1, 32767], increments outside [-32767, 32767], or, with a
 * match, a NULL cfg, steps outside aslam_csm_config's ranges or l_max <= 0. */
int aslam_csm_integrate(const aslam_slam* slam, int16_t* belief_dev, const int64_t* cell_off_dev,
                        const int32_t* side_dev, int32_t n,
                        const int32_t* pose_q_dev, const int32_t* rho_q_dev, int32_t R, const int32_t* a_off_dev,
                        int32_t max_side, int32_t rmax_q, const int32_t* match_dev, const aslam_csm_config* cfg,
                        double l_max, int32_t l_hit, int32_t l_miss, int32_t l_clamp, int32_t* coded_dev,
                        aslam_stream_t stream);

/* Fixed-lag pose graph (Sec. III-D; the minimisation of the weighted residuals and the covariance
 * of the newest pose as the last block of the inverse Gauss-Newton Hessian), n windows of L poses in
 * FP64, one wavefront each (the poses are linearised in parallel, one lane each; one lane runs the
 * elimination sweep; the window lives in LDS).  Factors: a prior on pose 0, prior_dev [n,6] (mean x, y, theta; information
 * diagonal); odometry between poses i and i+1, odo_dev [n,L-1,6] (the motion in the frame of pose i,
 * residual (R(th_i)^T (t_{i+1} - t_i) - u_t, wrap(th_{i+1} - th_i - u_th)); information diagonal; may
 * be NULL when L = 1); scan factors scan_dev [n,L,6] (measurement; information diagonal, all zero = no
 * factor).  From x0_dev [n,L,3] it takes `iters` Gauss-Newton steps (analytic Jacobians, block
 * elimination of the block-tridiagonal normal equations) into x_dev [n,L,3], then writes the newest
 * pose's covariance, formed at the result, to cov_dev [n,3,3].
 * ASL_EINVAL on NULL pointers, n < 0, L outside [1, 64] or
 * iters outside [0, 100].  A singular window (no prior information) gives non-finite results. */
int aslam_fixedlag_solve(int32_t n, int32_t L, const double* x0_dev, const double* prior_dev, const double* odo_dev,
                         const double* scan_dev, int32_t iters, double* x_dev, double* cov_dev,
                         aslam_stream_t stream);

/* ------------------------------------------------------------------ misc */

const char* aslam_last_error(void);
/* Device limits used by the autotuner: LDS bytes per workgroup, compute units. */
int aslam_device_info(int32_t* lds_per_block, int32_t* cu_count);

#ifdef __cplusplus
}
#endif
#endif
