// env_internal.h -- library-internal types of the gfx950 environment step.
//
// Not part of the public ABI (include/aslam.h).  Device layout of the batch:
//   world   : uint32 bits, robot-major, row-major inside a robot (bit j*s+i)
//   belief  : int16 log-odds in 1/256 nat, robot-major, row-major
//   visit   : per robot a (ceil(s c / lc_cell))^2 grid of first and last visits
// Robots are independent; one workgroup owns one robot at a time.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aslam {

constexpr int kNang = 46080;     // heading steps per turn
constexpr int kQ16 = 65536;      // position unit: 1/65536 cell
constexpr int kDirOne = 16384;   // direction unit in the heading table (Q14)
constexpr int kMarchLook = 8;    // DDA steps per LDS round trip in the LiDAR march

// Guard words before and after the staged world rows of a grid of side s: a
// lane reads up to kMarchLook steps past the end of its walk (never counted
// as hits), i.e. at most kMarchLook rows and one word beyond the window, so
// with this much addressable LDS on both sides no read needs a clamp.
__host__ __device__ inline int32_t march_guard_words(int32_t s) { return (kMarchLook * (s >> 5) + 1 + 3) & ~3; }

struct RobotMeta {
  int32_t side;        // s
  int32_t visit_side;  // loop-closure grid side
  int64_t world_off;   // first word of the robot's world bits
  int64_t cell_off;    // first cell of the robot's belief
  int64_t visit_off;   // first entry of the robot's visit grid
  float inv_ext;       // 1 / (s c), observation normalisation
  int32_t pad;
};

// Everything a step kernel needs besides the per-call buffers.
struct EnvParams {
  int32_t n, R, step_ang;
  int32_t loop_closure, lc_gap, episode_len;
  int32_t lhit, lmiss, lclamp;
  int32_t rhat_q;        // max range in 1/65536 cell
  int32_t rhat_cells;    // ceil of the max range in cells
  float v_max, w_max, dt;
  float sigma_x, sigma_y, sigma_th;
  float qx, qy, qth;     // sigma^2 (FP32 products)
  float var0_xy, var0_th;
  float inv_c16;         // 65536 / c
  float c16;             // c / 65536
  float k_ang;           // kNang / (2 pi)
  float inv_lc;          // 1 / lc_cell
  float lc_r2;           // lc_radius^2
  float lc_sigma, lc_var;
  float w_entropy, w_dopt, lambda_col;
  float inv_rmax, inv_pi;
  // sensor, proximity collision and reward of the paper (Sec. IV-A, Eq. 7)
  int32_t ray0;          // heading steps from the heading to ray 0 (0 for a full circle)
  int32_t reward_mode;   // 0: entropy / D-opt, 1: Eq. (7)
  int32_t uses_visits;   // visit grid kept (loop closure or reward_mode 1)
  int32_t G;             // noise row width: 5, + R with range noise
  int32_t sensed;        // reported range goes through the sensor model
  int32_t crash_q;       // d_crash in 1/65536 cell; 0 = no proximity test
  int32_t tep;           // episode length used by the novelty factor
  float r_max, r_min, range_sigma, range_quant, inv_quant;
  float d_crash, d_full, lambda_explore, lambda_abs, lambda_delta, u_hi, kappa;
  const RobotMeta* meta;
  int32_t* order;        // [n] the fused step's robot of each workgroup: the most work first
  int32_t* cost;         // [n] DDA cell visits of the robot's last step (its next step's work, nearly)
  const uint32_t* world;
  int16_t* belief;
  float* pose;
  float* est;
  float* cov;
  int64_t* hq_total;
  int32_t* step;
  int32_t* last_lc;
  int32_t* visit_t;
  float* visit_xy;
  int32_t* rho;          // [n,R]
  int32_t* hitc;         // [n,R]
  uint8_t* flags;        // [n,2] collided, closed
  float* terms;          // [n,2] entropy decrease, ln det
  int64_t* counters;     // [n,3] cumulative: coded cells, march visits, update visits
  int16_t* raylen;       // [n,R] steps of each ray's last LiDAR walk (lane-order key)
  const int32_t* dirtab; // [kNang] (cos & 0xffff) | (sin << 16), Q14
  const uint32_t* hq_lut;// [2*lclamp+1] binary entropy, 2^-32 nat
  int32_t* visit_last;   // [sum v^2] last step the robot was in each visit cell, -1 never
  int32_t* prev_vcell;   // [n] visit cell of the previous step, -1 after reset
  double* u_prev;        // [n] U_{t-1} = cbrt(det Sigma) of the previous step
  double* dcells;        // [n] novelty of this step's visit cell (motion -> reward)
  int32_t* dmin_bits;    // [n] FP32 bits of the smallest reported range (march -> reward)
  uint64_t seed;         // key of the step's own normal draws
  uint64_t* draws;       // [n] steps taken since create: counter of the robot's draws
  float* odo_u;          // [n,2] commanded motion (d, phi) of the step, 0 when blocked (fixed-lag backend)
};

// The fixed-lag SLAM backend (Sec. III-D in the loop): per-robot windows of up to L poses (FP64,
// [n][L][3] poses, [n][6] prior, [n][L-1][6] odometry factors, [n][L][6] scan factors, [n][L][3] the
// covariance diagonal each pose had when it was the newest) and the step's scan-matching buffers.
struct FixedLag {
  int32_t L, iters, W, V, step_xy, step_h, max_side;
  double cell, l_max, floor;
  double odo_info[3], scan_info[3], var0[3];
  double* x;
  double* prior;
  double* odo;
  double* scan;
  double* sig;
  int32_t* count;
  double* xout;
  double* covw;          // [n][3][3] newest pose's covariance
  int32_t* pose_q;       // [n,3] predicted pose: Q16 x, y, heading index
  int32_t* rho_q;        // [n,R] reported ranges of the rays that hit (Q16), -1 otherwise
  int32_t* match;        // [n,6]
  int32_t* pose_al;      // [n,3] aligned pose (Q16, heading index)
  int32_t* wq;           // [n] integration weight, 1/256
  int32_t* coded;        // [n] coded cells of the integration
  const int32_t* a_off;  // [R] ray heading offsets
  const int64_t* cell_off;
  const int32_t* side;
};

struct StepArgs {
  const float* actions;  // [n,2]
  const float* noise;    // [n,G], or NULL: the step draws its own normals
  float* ranges;         // [n,R]
  float* reward;         // [n]
  uint8_t* done;         // [n]
};

// LDS plan of the per-robot kernels (byte offsets into dynamic LDS).
struct LdsPlan {
  int32_t off_lut, off_rho, off_perm, off_seg, off_hist, off_misc, off_union;
  int32_t total;
  int32_t union_bytes;
  int32_t band_rows;      // code-window rows per pass
  int32_t world_halo;     // rows staged around the robot: rhat_cells + 3
  int32_t record;         // fused: write rho / hitc to the state
  int32_t mark_seg;       // map update's walk: 0 one lane per ray, else segments of this many steps
};

struct ExecState;

// Launchers (env_kernels.hip); all asynchronous on `stream`.
hipError_t launch_reset(const EnvParams& P, const uint32_t* world_src, const float* init_pose,
                        const uint8_t* mask, int32_t max_side, hipStream_t stream);
hipError_t launch_step_plain(const EnvParams& P, const StepArgs& A, const LdsPlan& L, int threads,
                             hipStream_t stream);
// The fused step's robot order (most work first) is refreshed by a sort of the robots' last-step work
// before every kOrderEvery-th fused step: the work a robot does changes slowly from step to step, and
// the order never changes a result.
constexpr int kOrderEvery = 4;
hipError_t launch_step_fused(const EnvParams& P, const StepArgs& A, const LdsPlan& L, int threads,
                             int grid, bool order, hipStream_t stream);
hipError_t launch_step_fixedlag(const EnvParams& P, const StepArgs& A, const LdsPlan& L, const FixedLag& F,
                                int threads, hipStream_t stream);
hipError_t launch_reset_fixedlag(const EnvParams& P, const FixedLag& F, const float* init_pose, const uint8_t* mask,
                                 hipStream_t stream);
hipError_t launch_observe(const EnvParams& P, const float* ranges, int16_t* crop, int32_t cs,
                          float* scan, float* state, const float* u_new, double alpha, hipStream_t stream);
hipError_t set_kernel_lds_limits(int bytes);

}  // namespace aslam
