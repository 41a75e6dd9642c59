// env_kernels.hip -- gfx950 kernels of the batched Active-SLAM environment step.
//
// Method: arXiv 2603.25834.  One POMDP transition per robot (Sec. III-B):
// the robot moves under the continuous action of Sec. III-C (Eq. 4), the
// LiDAR of Sec. IV-A samples the world, the scan is integrated into the 2-D
// log-odds grid of Sec. III-D, the pose covariance is propagated (an EKF
// stands in for the fixed-lag backend of Sec. III-D), and the reward combines
// the collision penalty of Eq. (7) with the map-entropy decrease and the
// D-optimality term -ln det(Sigma) (Table I, "D-opt").
//
// Execution model (CDNA4): one workgroup owns one robot at a time.  Rays are
// spread over the workgroup's lanes; each lane walks its ray through the grid
// with an exact integer DDA (32-bit decision variable, no division in the
// loop).  The LiDAR march reads the robot's world bits from LDS.  The map
// update marks a per-scan code window in LDS (two bitmaps: MISS and HIT;
// OR-ing bits makes the result independent of ray and lane order), then a
// coalesced pass applies one saturating int16 add to each coded cell and
// accumulates the exact entropy change in int64.
#include <algorithm>

#include "env_internal.h"
#include "rng.h"
#include "slam_internal.h"

namespace aslam {

namespace {

__device__ __forceinline__ int32_t heading_index(float th, float k_ang) {
  float t = th * k_ang;
  if (!(t > -1.0e9f && t < 1.0e9f)) t = 0.0f;
  int32_t i = (int32_t)rintf(t);
  i %= kNang;
  if (i < 0) i += kNang;
  return i;
}

__device__ __forceinline__ float wrap_pi(float th) {
  const float pi = 3.14159265358979f;
  const float two_pi = 6.28318530717959f;
  if (th >= pi) th = th - two_pi;
  else if (th < -pi) th = th + two_pi;
  return th;
}

// Position in 1/65536 cell: rint(v * 65536/c) in FP32, clamped to +-1e9 (NaN -> -1e9).
__device__ __forceinline__ int32_t to_q16(float v, float inv_c16) {
  float t = v * inv_c16;
  if (!(t >= -1.0e9f)) t = -1.0e9f;
  if (!(t <= 1.0e9f)) t = 1.0e9f;
  return (int32_t)rintf(t);
}

__device__ __forceinline__ float dir_cos(int32_t d) { return (float)(int16_t)(d & 0xffff) * (1.0f / 16384.0f); }
__device__ __forceinline__ float dir_sin(int32_t d) { return (float)(d >> 16) * (1.0f / 16384.0f); }

__device__ __forceinline__ bool world_bit(const uint32_t* w, int32_t s, int32_t i, int32_t j) {
  int32_t bit = j * s + i;
  return (w[bit >> 5] >> (bit & 31)) & 1u;
}

// Motion segment from Q16 (ox,oy) to (nx,ny): blocked if any cell it enters
// (entry parameter <= 1, exact corner steps x first) is occupied or off-grid.
__device__ bool segment_blocked(const uint32_t* w, int32_t s, int32_t ox, int32_t oy, int32_t nx, int32_t ny) {
  int32_t cx = ox >> 16, cy = oy >> 16;
  if (cx < 0 || cx >= s || cy < 0 || cy >= s) return true;
  if (world_bit(w, s, cx, cy)) return true;
  int64_t a = (int64_t)nx - ox, b = (int64_t)ny - oy;
  if (a == 0 && b == 0) return false;
  int64_t aa = a < 0 ? -a : a, bb = b < 0 ? -b : b;
  int64_t fx = ox & 0xffff, fy = oy & 0xffff;
  int64_t ex = a > 0 ? kQ16 - fx : fx;
  int64_t ey = b > 0 ? kQ16 - fy : fy;
  for (int32_t it = 0; it < 2 * s + 4; ++it) {
    bool stepx = (aa == 0) ? false : ((bb == 0) ? true : (ex * bb <= ey * aa));
    if (stepx) {
      if (ex > aa) return false;
      cx += a > 0 ? 1 : -1;
      if (cx < 0 || cx >= s) return true;
      ex += kQ16;
    } else {
      if (ey > bb) return false;
      cy += b > 0 ? 1 : -1;
      if (cy < 0 || cy >= s) return true;
      ey += kQ16;
    }
    if (world_bit(w, s, cx, cy)) return true;
  }
  return true;
}

// Proximity collision (Sec. IV-A): an occupied or off-grid cell lies closer
// than rc (1/65536 cell) to the Q16 point, by the exact integer distance from
// the point to the cell's square.  The (2m+1)^2 cells around the point's cell
// (m = rc / 65536 + 1) are shared out: this lane tests cells k0, k0 + stride, ...
__device__ bool near_obstacle_part(const uint32_t* w, int32_t s, int32_t px, int32_t py, int32_t rc, int32_t k0,
                                   int32_t stride) {
  const int32_t cx = px >> 16, cy = py >> 16;
  const int32_t m = rc / kQ16 + 1, side = 2 * m + 1;
  const int64_t rc2 = (int64_t)rc * rc;
  bool near = false;
  for (int32_t k = k0; k < side * side; k += stride) {
    const int32_t j = cy - m + k / side, i = cx - m + k % side;
    const bool occ = (i < 0 || j < 0 || i >= s || j >= s) || world_bit(w, s, i, j);
    if (occ) {
      const int64_t dx = max(max((int64_t)i * kQ16 - px, (int64_t)px - (int64_t)(i + 1) * kQ16), (int64_t)0);
      const int64_t dy = max(max((int64_t)j * kQ16 - py, (int64_t)py - (int64_t)(j + 1) * kQ16), (int64_t)0);
      near = near || dx * dx + dy * dy < rc2;
    }
  }
  return near;
}

// The test by a whole workgroup, one cell per thread; sets *flag (LDS) when some cell is near.
template <int NT>
__device__ void near_obstacle_wg(const uint32_t* w, int32_t s, int32_t px, int32_t py, int32_t rc, int32_t* flag) {
  const bool near = near_obstacle_part(w, s, px, py, rc, (int32_t)threadIdx.x, NT);
  if (__builtin_amdgcn_ballot_w64(near) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Heading index of ray 0 of the fan whose heading index is ib.
__device__ __forceinline__ int32_t fan_base(const EnvParams& P, int32_t ib) {
  const int32_t id = ib + P.ray0;
  return id >= kNang ? id - kNang : id;
}

__device__ __forceinline__ double cov_det(const float* c) {
  return (double)c[0] * ((double)c[3] * c[5] - (double)c[4] * c[4]) -
         (double)c[1] * ((double)c[1] * c[5] - (double)c[4] * c[2]) +
         (double)c[2] * ((double)c[1] * c[4] - (double)c[3] * c[2]);
}

// SLAM uncertainty scalar U = cbrt(det Sigma) (0 when det <= 0).
__device__ __forceinline__ double uncertainty(const float* c) {
  const double d = cov_det(c);
  return d > 0.0 ? cbrt(d) : 0.0;
}

__device__ __forceinline__ double clip01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

// Reward of Eq. (7): the collision penalty alone on a collision, else the
// exploration reward (Eq. 8, novelty of Eq. 9 times the intrinsic factor of
// Eqs. 10-12) minus the absolute uncertainty penalty (Eq. 13) plus the
// differential term (Eq. 14); the clearance factor of Eq. 15 scales the
// exploration term and a falling-uncertainty differential term (Eqs. 16-17).
__device__ double paper_reward(const EnvParams& P, int32_t collided, double dcells, double up, double u,
                               double d_min) {
  if (collided) return -(double)P.lambda_col;
  double cg = clip01(((double)P.u_hi - up) / (double)P.u_hi);
  cg = cg * cg;
  const double iota = clip01(fmax(up - u, 0.0) / (double)P.kappa);
  const double in = cg + (1.0 - cg) * iota;
  const double r_explore = (double)P.lambda_explore * dcells * in;
  const double eu = exp(up);
  const double r_abs = (double)P.lambda_abs * eu * up;
  const double r_delta = (double)P.lambda_delta * eu * (up - u);
  const double alpha = clip01((d_min - (double)P.d_crash) / ((double)P.d_full - (double)P.d_crash));
  return r_explore * alpha - r_abs + (up - u > 0.0 ? r_delta * alpha : r_delta);
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The step's standard-normal draws of robot r: column k of the caller's noise row, or the
// library's own draw k at the robot's draw counter (the counter moves on at the end of the step).
struct StepNoise {
  const float* row;
  uint64_t seed, ctr;
  int32_t r;
  __device__ __forceinline__ float operator()(int32_t k) const {
    return row ? row[k] : rng::normal(seed, rng::kDomainEnv, ctr, (uint64_t)r, (uint64_t)k);
  }
};

__device__ __forceinline__ StepNoise step_noise(const EnvParams& P, const StepArgs& A, int32_t r) {
  StepNoise g{nullptr, P.seed, 0ull, r};
  if (A.noise)
    g.row = A.noise + (int64_t)P.G * r;
  else
    g.ctr = P.draws[r];
  return g;
}

struct MotionOut {
  int32_t tox, toy, ib_t;   // true origin (Q16) and heading index of ray 0
  int32_t eox, eoy, ib_e;   // estimated origin and heading index of ray 0
  int32_t collided, closed;
};

// The step's five motion normals of robot r (odometry x, y, theta; loop-closure x, y), drawn by five
// lanes of a wave at once and gathered in every lane of the group of eight that holds `lane0`
// (a library draw is a long dependent chain; one lane drawing all five would wait for five).
struct MotionDraws {
  float g[5];
  __device__ __forceinline__ float operator()(int k) const { return g[k]; }
};

__device__ __forceinline__ MotionDraws motion_draws(const EnvParams& P, const StepArgs& A, int32_t r, bool valid,
                                                    int lane0) {
  const int sub = (int)(threadIdx.x & 63) - lane0;
  float gk = 0.0f;
  if (valid && sub >= 0 && sub < 5) gk = step_noise(P, A, r)(sub);
  MotionDraws d;
#pragma unroll
  for (int k = 0; k < 5; ++k) d.g[k] = __shfl(gk, lane0 + k, 64);
  return d;
}

// Motion, collision, EKF predict and loop closure of robot r (one thread, with the robot's draws).  The
// proximity part of the collision test (which leaves the move standing) is left to the caller's lanes:
// the fused step runs it on the whole workgroup, k_motion on the robot's sixteen lanes.
__device__ MotionOut robot_motion(const EnvParams& P, const StepArgs& A, int32_t r, const MotionDraws& g) {
  const RobotMeta m = P.meta[r];
  const int32_t s = m.side;
  const float a0 = A.actions[2 * r], a1 = A.actions[2 * r + 1];
  float v = fminf(fmaxf(a0, 0.0f), P.v_max);
  float w = fminf(fmaxf(a1, -P.w_max), P.w_max);
  if (v != v) v = 0.0f;
  if (w != w) w = 0.0f;
  float d = v * P.dt;
  float phi = w * P.dt;

  float* p = P.pose + 3 * (int64_t)r;
  float px = p[0], py = p[1], pth = p[2];
  const int32_t dt_ = P.dirtab[heading_index(pth, P.k_ang)];
  const float nx = (px + d * dir_cos(dt_)) + P.sigma_x * g(0);
  const float ny = (py + d * dir_sin(dt_)) + P.sigma_y * g(1);
  const float nth = wrap_pi((pth + phi) + P.sigma_th * g(2));
  const uint32_t* W = P.world + m.world_off;
  const bool col = segment_blocked(W, s, to_q16(px, P.inv_c16), to_q16(py, P.inv_c16),
                                   to_q16(nx, P.inv_c16), to_q16(ny, P.inv_c16));
  if (col) {
    d = 0.0f;
    phi = 0.0f;
  } else {
    px = nx; py = ny; pth = nth;
    p[0] = px; p[1] = py; p[2] = pth;
  }
  if (P.odo_u) {
    P.odo_u[2 * (int64_t)r] = d;
    P.odo_u[2 * (int64_t)r + 1] = phi;
  }
  const int32_t collided = col;

  // EKF predict; F uses the estimated heading before the step.
  float* e = P.est + 3 * (int64_t)r;
  float* c = P.cov + 6 * (int64_t)r;
  float ex = e[0], ey = e[1], eth = e[2];
  float c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
  {
    const int32_t de = P.dirtab[heading_index(eth, P.k_ang)];
    const float ch = dir_cos(de), sh = dir_sin(de);
    const float fa = -(d * sh);
    const float fb = d * ch;
    const float n0 = ((c0 + (2.0f * fa) * c2) + (fa * fa) * c5) + P.qx;
    const float n1 = ((c1 + fa * c4) + fb * c2) + (fa * fb) * c5;
    const float n2 = c2 + fa * c5;
    const float n3 = ((c3 + (2.0f * fb) * c4) + (fb * fb) * c5) + P.qy;
    const float n4 = c4 + fb * c5;
    const float n5 = c5 + P.qth;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3; c4 = n4; c5 = n5;
    ex = ex + d * ch;
    ey = ey + d * sh;
    eth = wrap_pi(eth + phi);
  }

  const int32_t t = P.step[r];
  // visit cell of the true position (loop closure, exploration novelty)
  int32_t vcell = -1;
  int64_t vk = 0;
  if (P.uses_visits) {
    const int32_t nv = m.visit_side;
    int32_t vx = (int32_t)floorf(px * P.inv_lc);
    int32_t vy = (int32_t)floorf(py * P.inv_lc);
    vx = min(max(vx, 0), nv - 1);
    vy = min(max(vy, 0), nv - 1);
    vcell = vy * nv + vx;
    vk = m.visit_off + vcell;
  }
  // novelty (Eq. 9): 1 on entering a never-visited cell, half the episode
  // fraction since the last visit on re-entering one, 0 while staying
  if (P.reward_mode == 1) {
    double dcells = 0.0;
    if (vcell != P.prev_vcell[r]) {
      const int32_t last = P.visit_last[vk];
      dcells = last < 0 ? 1.0 : fmin(1.0, 0.5 * (double)(t - last) / (double)P.tep);
    }
    P.visit_last[vk] = t;
    P.prev_vcell[r] = vcell;
    P.dcells[r] = dcells;
  }
  int32_t closed = 0;
  if (P.loop_closure) {
    const int32_t t0 = P.visit_t[vk];
    if (t0 < 0) {
      P.visit_t[vk] = t;
      P.visit_xy[2 * vk] = px;
      P.visit_xy[2 * vk + 1] = py;
    } else {
      const float dx = px - P.visit_xy[2 * vk];
      const float dy = py - P.visit_xy[2 * vk + 1];
      if (t - t0 >= P.lc_gap && t - P.last_lc[r] >= P.lc_gap && (dx * dx + dy * dy) <= P.lc_r2) {
        const float zx = px + P.lc_sigma * g(3);
        const float zy = py + P.lc_sigma * g(4);
        const float s00 = c0 + P.lc_var, s01 = c1, s11 = c3 + P.lc_var;
        const float det = s00 * s11 - s01 * s01;
        const float i00 = s11 / det, i01 = (-s01) / det, i11 = s00 / det;
        const float kx0 = c0 * i00 + c1 * i01, kx1 = c0 * i01 + c1 * i11;
        const float ky0 = c1 * i00 + c3 * i01, ky1 = c1 * i01 + c3 * i11;
        const float kt0 = c2 * i00 + c4 * i01, kt1 = c2 * i01 + c4 * i11;
        const float v0 = zx - ex, v1 = zy - ey;
        ex = ex + (kx0 * v0 + kx1 * v1);
        ey = ey + (ky0 * v0 + ky1 * v1);
        eth = wrap_pi(eth + (kt0 * v0 + kt1 * v1));
        const float m0 = c0 - (kx0 * c0 + kx1 * c1);
        const float m1 = c1 - (kx0 * c1 + kx1 * c3);
        const float m2 = c2 - (kx0 * c2 + kx1 * c4);
        const float m3 = c3 - (ky0 * c1 + ky1 * c3);
        const float m4 = c4 - (ky0 * c2 + ky1 * c4);
        const float m5 = c5 - (kt0 * c2 + kt1 * c4);
        c0 = m0; c1 = m1; c2 = m2; c3 = m3; c4 = m4; c5 = m5;
        P.last_lc[r] = t;
        closed = 1;
      }
    }
  }
  e[0] = ex; e[1] = ey; e[2] = eth;
  c[0] = c0; c[1] = c1; c[2] = c2; c[3] = c3; c[4] = c4; c[5] = c5;
  P.step[r] = t + 1;
  P.flags[2 * (int64_t)r] = (uint8_t)collided;
  P.flags[2 * (int64_t)r + 1] = (uint8_t)closed;

  MotionOut o;
  o.tox = to_q16(px, P.inv_c16);
  o.toy = to_q16(py, P.inv_c16);
  o.ib_t = fan_base(P, heading_index(pth, P.k_ang));
  o.eox = to_q16(ex, P.inv_c16);
  o.eoy = to_q16(ey, P.inv_c16);
  o.ib_e = fan_base(P, heading_index(eth, P.k_ang));
  o.collided = collided;
  o.closed = closed;
  return o;
}

// Per-robot values shared by the workgroup (LDS).
struct RobotShared {
  int32_t r;
  int32_t tox, toy, ib_t;
  int32_t eox, eoy, ib_e;
  int32_t collided;
  int32_t cnt_march, cnt_upd;
  int32_t bx0, bx1, by0, by1;   // cell bounding box of the ray end points (estimated pose)
  int32_t dmin_bits;            // FP32 bits of the smallest reported range (non-negative)
  int32_t near;                 // proximity collision found by the workgroup
  long long part[16];
  int32_t dpart[16];
};

// Pointers into the dynamic LDS of a per-robot kernel.
struct LdsView {
  uint32_t* lut;     // binary entropy table
  int32_t* rho;      // [R] range (Q16) | bit 31 = hit
  int32_t* perm;     // [R] ray of each lane slot, longest walk first (march); steps of each ray (mark)
  int32_t* seg;      // [R] first walk segment of each ray (mark)
  int32_t* hist;     // [64] sort buckets
  RobotShared* sh;
  uint32_t* uni;     // world rows, then the code bitmaps
};

__device__ __forceinline__ LdsView lds_view(unsigned char* smem, const LdsPlan& L) {
  LdsView v;
  v.lut = reinterpret_cast<uint32_t*>(smem + L.off_lut);
  v.rho = reinterpret_cast<int32_t*>(smem + L.off_rho);
  v.perm = reinterpret_cast<int32_t*>(smem + L.off_perm);
  v.seg = reinterpret_cast<int32_t*>(smem + L.off_seg);
  v.hist = reinterpret_cast<int32_t*>(smem + L.off_hist);
  v.sh = reinterpret_cast<RobotShared*>(smem + L.off_misc);
  v.uni = reinterpret_cast<uint32_t*>(smem + L.off_union);
  return v;
}

// ---------------------------------------------------------------- DDA setup
// Ray from Q16 origin o with table direction (a,b) (Q14), limit lim (Q16 cells).
// x crossings happen at axis distances ex0 + k*65536; the k-th is within the
// limit iff (ex0 + k*65536) * 2^14 <= lim * |a|.
// The walk stops at the first crossing that is not allowed (beyond the limit
// or off the grid); crossings are taken in parameter order, an x crossing
// before a y crossing at the same parameter.  `n` is the exact number of
// steps before that crossing, so the loops run a known trip count.
struct RaySetup {
  int32_t D, DX, DY;
  int32_t nx, ny;          // x / y steps allowed (limit and grid)
  int32_t gx, gy;          // 1: running out of x / y steps means leaving the grid
  int32_t ex0, ey0, aa, bb;
  int32_t n;               // steps taken by the walk (cells visited = n + 1)
  int32_t kx, ky;          // x / y steps among them
  int32_t gend;            // 1: the walk ends by leaving the grid (else by the limit)
};

__device__ __forceinline__ RaySetup ray_setup(int32_t ox, int32_t oy, int32_t a, int32_t b, int32_t lim,
                                              int32_t s) {
  RaySetup q;
  const int32_t cx = ox >> 16, cy = oy >> 16;
  const int32_t aa = abs(a), bb = abs(b);
  const int32_t fx = ox & 0xffff, fy = oy & 0xffff;
  const int32_t ex0 = a > 0 ? kQ16 - fx : fx;
  const int32_t ey0 = b > 0 ? kQ16 - fy : fy;
  const int64_t emx = ((int64_t)lim * aa) >> 14;
  const int64_t emy = ((int64_t)lim * bb) >> 14;
  const int32_t nxl = (aa == 0 || emx < ex0) ? 0 : (int32_t)((emx - ex0) >> 16) + 1;
  const int32_t nyl = (bb == 0 || emy < ey0) ? 0 : (int32_t)((emy - ey0) >> 16) + 1;
  const int32_t nxg = a > 0 ? s - 1 - cx : cx;
  const int32_t nyg = b > 0 ? s - 1 - cy : cy;
  q.nx = min(nxl, nxg);
  q.ny = min(nyl, nyg);
  q.gx = nxg < nxl;
  q.gy = nyg < nyl;
  if (aa == 0) { q.D = 1; q.DX = 0; q.DY = 0; }
  else if (bb == 0) { q.D = -1; q.DX = 0; q.DY = 0; }
  else { q.D = ex0 * bb - ey0 * aa; q.DX = bb << 16; q.DY = aa << 16; }
  q.ex0 = ex0; q.ey0 = ey0; q.aa = aa; q.bb = bb;
  // Which forbidden crossing comes first: x crossing #nx at parameter
  // Tx/(aa bb), y crossing #ny at Ty/(aa bb) (x first on a tie).
  if (aa == 0) {
    q.kx = 0; q.ky = q.ny; q.gend = q.gy;
  } else if (bb == 0) {
    q.kx = q.nx; q.ky = 0; q.gend = q.gx;
  } else {
    const int64_t Tx = (int64_t)(ex0 + (int64_t)q.nx * kQ16) * bb;
    const int64_t Ty = (int64_t)(ey0 + (int64_t)q.ny * kQ16) * aa;
    if (Tx <= Ty) {
      // y crossings j strictly before it: (ey0 + j*65536)*aa < Tx
      const int64_t X = Tx - (int64_t)ey0 * aa;
      const int64_t den = (int64_t)aa << 16;
      const int32_t cnt = X <= 0 ? 0 : (int32_t)((X + den - 1) / den);
      q.kx = q.nx; q.ky = min(cnt, q.ny); q.gend = q.gx;
    } else {
      // x crossings k at or before it: (ex0 + k*65536)*bb <= Ty
      const int64_t Y = Ty - (int64_t)ex0 * bb;
      const int64_t den = (int64_t)bb << 16;
      const int32_t cnt = Y < 0 ? 0 : (int32_t)(Y / den) + 1;
      q.kx = min(cnt, q.nx); q.ky = q.ny; q.gend = q.gy;
    }
  }
  q.n = q.kx + q.ky;
  return q;
}

// Entry axis of the cell reached after at least one step: with D in
// (-DY, DX], an x step leaves D in (DX-DY, DX] and a y step in (-DY, DX-DY].
__device__ __forceinline__ bool last_step_x(const RaySetup& q, int32_t D) {
  if (q.aa == 0) return false;
  if (q.bb == 0) return true;
  return D > q.DX - q.DY;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int32_t ray_dir(const EnvParams& P, int32_t ib, int32_t k) {
  int32_t id = ib + k * P.step_ang;
  id -= (id >= kNang) ? kNang : 0;
  return P.dirtab[id];
}

// Counting sort of the R rays by a bucket key in [0, 63] (larger = longer
// walk), longest first: perm[j] is the ray walked by lane slot j.  Lanes of a
// wave then walk rays of similar length, so a wave's trip count (its longest
// walk) stays close to its lanes' own.  Results do not depend on the order.
template <int NT, typename KeyFn>
__device__ void sort_rays(int32_t R, int32_t* perm, int32_t* hist, KeyFn key_of) {
  constexpr int kMaxPer = 8;
  const int32_t tid = threadIdx.x;
  if (R > kMaxPer * NT) {
    for (int32_t k = tid; k < R; k += NT) perm[k] = k;
    __syncthreads();
    return;
  }
  for (int32_t b = tid; b < 64; b += NT) hist[b] = 0;
  __syncthreads();
  int32_t key[kMaxPer], pos[kMaxPer];
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) {
    const int32_t k = tid + i * NT;
    if (k < R) {
      key[i] = 63 - min(max(key_of(k), 0), 63);
      pos[i] = atomicAdd(&hist[key[i]], 1);
    }
  }
  __syncthreads();
  if (tid < 64) {
    const int32_t v = hist[tid];
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(x, o, 64);
      if (tid >= o) x += y;
    }
    hist[tid] = x - v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxPer; ++i) {
    const int32_t k = tid + i * NT;
    if (k < R) perm[hist[key[i]] + pos[i]] = k;
  }
  __syncthreads();
}

// Cell bounding box of the end points of all rays walked from the Q16 origin
// (eox, eoy) with the ranges in rho (Q16).  Every cell a walk visits lies
// within one cell of its segment, so the box grown by 2 cells holds them all.
template <int NT>
__device__ void endpoint_bbox(const EnvParams& P, const int32_t* rho, int32_t eox, int32_t eoy, int32_t ib,
                              RobotShared* sh) {
  int32_t mnx = eox >> 16, mxx = mnx, mny = eoy >> 16, mxy = mny;
  for (int32_t k = threadIdx.x; k < P.R; k += NT) {
    const int32_t lim = rho[k] & 0x7fffffff;
    const int32_t dv = ray_dir(P, ib, k);
    const int32_t a = (int16_t)(dv & 0xffff), b = dv >> 16;
    const int32_t qx = (int32_t)(((int64_t)eox + (((int64_t)lim * a) >> 14)) >> 16);
    const int32_t qy = (int32_t)(((int64_t)eoy + (((int64_t)lim * b) >> 14)) >> 16);
    mnx = min(mnx, qx); mxx = max(mxx, qx);
    mny = min(mny, qy); mxy = max(mxy, qy);
  }
  mnx = wave_min_i32(mnx); mxx = wave_max_i32(mxx);
  mny = wave_min_i32(mny); mxy = wave_max_i32(mxy);
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&sh->bx0, mnx); atomicMax(&sh->bx1, mxx);
    atomicMin(&sh->by0, mny); atomicMax(&sh->by1, mxy);
  }
}

// ---------------------------------------------------------------- stages
template <int NT>
__device__ void stage_world(const EnvParams& P, const RobotMeta& m, int32_t cy, int32_t halo, uint32_t* sw,
                            int32_t& wy0) {
  const int32_t s = m.side;
  const int32_t y0 = max(0, min(s - 1, cy - halo));
  const int32_t y1 = max(0, min(s - 1, cy + halo));
  const int32_t wpr = s >> 5;
  const int32_t nwords = (y1 - y0 + 1) * wpr;
  const uint32_t* src = P.world + m.world_off + (int64_t)y0 * wpr;
  // rows start on 16-byte boundaries when s is a multiple of 128 (8 when of 64)
  if ((wpr & 3) == 0) {
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(sw);
#pragma unroll 4
    for (int32_t k = threadIdx.x; k < (nwords >> 2); k += NT) d4[k] = s4[k];
  } else if ((wpr & 1) == 0) {
    const uint2* s2 = reinterpret_cast<const uint2*>(src);
    uint2* d2 = reinterpret_cast<uint2*>(sw);
#pragma unroll 4
    for (int32_t k = threadIdx.x; k < (nwords >> 1); k += NT) d2[k] = s2[k];
  } else {
#pragma unroll 4
    for (int32_t k = threadIdx.x; k < nwords; k += NT) sw[k] = src[k];
  }
  wy0 = y0;
}

constexpr int kLook = kMarchLook;

// LiDAR march of every ray of the robot from the true pose (lanes = rays),
// then the reported range of each ray (sensor model of Sec. IV-A: true range
// plus noise, rounded to the quantum, clamped to [r_min, r_max]).  The map
// update walks the reported range; ray k takes draw 5 + k of gr.
template <int NT>
__device__ void march_rays(const EnvParams& P, const RobotMeta& m, const LdsView& V, const uint32_t* sw,
                           int32_t wy0, float* ranges_out, const StepNoise& gr, bool record, int32_t r) {
  RobotShared* sh = V.sh;
  int32_t* rho_lds = V.rho;
  const int32_t s = m.side;
  const int32_t tox = sh->tox, toy = sh->toy, ib = sh->ib_t;
  const int32_t cx0 = tox >> 16, cy0 = toy >> 16;
  const bool inside = cx0 >= 0 && cx0 < s && cy0 >= 0 && cy0 < s;
  int16_t* raylen = P.raylen + (int64_t)r * P.R;
  // lane slots ordered by the previous step's walk length of each ray
  sort_rays<NT>(P.R, V.perm, V.hist, [&](int32_t k) { return (int32_t)raylen[k] >> 2; });
  int32_t visits = 0;
  float dmin = __int_as_float(0x7f800000);
  for (int32_t k0 = 0; k0 < P.R; k0 += NT) {
    const int32_t j = k0 + (int32_t)threadIdx.x;
    const int32_t k = j < P.R ? V.perm[j] : P.R;
    const bool active = inside && k < P.R;
    int32_t rq = P.rhat_q;
    int32_t cell = -1;
    RaySetup q{};
    int32_t li = 0, D = 0, i = 0, sx = 0, sy = 0;
    bool hit = false, done = true;
    if (active) {
      const int32_t dv = ray_dir(P, ib, k);
      const int32_t a = (int16_t)(dv & 0xffff), b = dv >> 16;
      q = ray_setup(tox, toy, a, b, P.rhat_q, s);
      li = (cy0 - wy0) * s + cx0;
      sx = a > 0 ? 1 : -1;
      sy = b > 0 ? s : -s;
      D = q.D;
      hit = (sw[li >> 5] >> (li & 31)) & 1u;
      done = hit || q.n == 0;
    }
    // kLook cells per iteration: the next kLook DDA steps are taken first and
    // their world words read together, so one LDS round trip covers kLook
    // cells.  Steps past the walk's own count n are read (from the guard
    // words around the staged rows) but never count as hits.
    while (__builtin_amdgcn_ballot_w64(!done) != 0) {
      if (!done) {
        int32_t l[kLook], d[kLook];
        int32_t lc = li, dc = D;
#pragma unroll
        for (int u = 0; u < kLook; ++u) {
          const bool stepx = dc <= 0;
          lc += stepx ? sx : sy;
          dc += stepx ? q.DX : -q.DY;
          l[u] = lc;
          d[u] = dc;
        }
        uint32_t wd[kLook];
#pragma unroll
        for (int u = 0; u < kLook; ++u) wd[u] = sw[l[u] >> 5];   // inside the guard words
        uint32_t bits = 0u;   // v_bfe_u32 takes the bit offset mod 32 itself
#pragma unroll
        for (int u = 0; u < kLook; ++u) bits |= __builtin_amdgcn_ubfe(wd[u], (uint32_t)l[u], 1u) << u;
        const int32_t rem = q.n - i;   // >= 1 while the lane walks
        bits &= rem >= kLook ? (1u << kLook) - 1u : ((1u << rem) - 1u);
        if (bits) {
          const int32_t u = __builtin_ctz(bits);
#pragma unroll
          for (int j = 0; j < kLook; ++j) {
            if (u == j) {
              li = l[j];
              D = d[j];
            }
          }
          i += u + 1;
          hit = true;
          done = true;
        } else {
          li = l[kLook - 1];
          D = d[kLook - 1];
          i = min(i + kLook, q.n);
          done = i >= q.n;
        }
      }
    }
    if (active) {
      visits += i + 1;
      raylen[k] = (int16_t)min(i, 32767);
      if (hit) {
        cell = li + wy0 * s;
        if (i > 0) {
          const int32_t row = li / s;
          if (last_step_x(q, D)) {
            const int32_t kx = abs(li - row * s - cx0);
            const int64_t E = (int64_t)q.ex0 + (int64_t)(kx - 1) * kQ16;
            rq = (int32_t)((E * kDirOne + q.aa - 1) / q.aa);
          } else {
            const int32_t ky = abs(row + wy0 - cy0);
            const int64_t E = (int64_t)q.ey0 + (int64_t)(ky - 1) * kQ16;
            rq = (int32_t)((E * kDirOne + q.bb - 1) / q.bb);
          }
        } else {
          rq = 0;
        }
      }
    }
    if (k < P.R) {
      float rep = (float)rq * P.c16;
      int32_t rho_u = rq;
      if (P.sensed) {
        if (P.range_sigma > 0.0f) rep = rep + P.range_sigma * gr(5 + k);
        if (P.range_quant > 0.0f) rep = rintf(rep * P.inv_quant) * P.range_quant;
        rep = fminf(fmaxf(rep, P.r_min), P.r_max);
        rho_u = to_q16(rep, P.inv_c16);
      }
      dmin = fminf(dmin, rep);
      rho_lds[k] = rho_u | (cell >= 0 ? (int32_t)0x80000000 : 0);
      ranges_out[(int64_t)r * P.R + k] = rep;
      if (record) {
        P.rho[(int64_t)r * P.R + k] = rho_u;
        P.hitc[(int64_t)r * P.R + k] = cell;
      }
    }
  }
  visits = wave_sum_i32(visits);
  if ((threadIdx.x & 63) == 0 && visits) atomicAdd(&sh->cnt_march, visits);
  if (P.reward_mode == 1) {
    // reported ranges are >= 0, so their FP32 bits order as integers
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmin = fminf(dmin, __shfl_xor(dmin, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMin(&sh->dmin_bits, __float_as_int(dmin));
  }
  __syncthreads();
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One saturating add per coded cell of a band of the code window.  The band
// is split into octets (8 cells, one 16-byte access, 16-byte aligned because
// the window starts on a 32-cell boundary); each thread keeps U octets in
// flight, so a band costs few HBM round trips.  An octet is owned by one
// thread, so the read-modify-write is race-free; uncoded cells of a touched
// octet are written back unchanged, untouched octets are neither read nor
// written.
template <int NT, int U>
__device__ __forceinline__ void apply_band(const EnvParams& P, const uint32_t* miss, const uint32_t* hitm,
                                           int32_t rows, int32_t nw, int16_t* band_base, int32_t s,
                                           const uint32_t* lut, long long& dh, int32_t& ncoded) {
  const int32_t lpr = nw * 4;  // octets per row
  const int32_t total = rows * lpr;
  int32_t row = (int32_t)threadIdx.x / lpr;
  int32_t col = (int32_t)threadIdx.x - row * lpr;
  const int32_t qa = NT / lpr, ra = NT - qa * lpr;
  const int32_t lc = P.lclamp;
  for (int32_t o = threadIdx.x; o < total; o += U * NT) {
    uint32_t code[U];   // miss bits | hit bits << 8
    int32_t off[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t wm = 0u, wh = 0u;
      if (o + u * NT < total) {
        wm = miss[row * nw + (col >> 2)];
        wh = hitm[row * nw + (col >> 2)];
      }
      const int32_t sh = (col & 3) * 8;
      code[u] = ((wm >> sh) & 0xffu) | (((wh >> sh) & 0xffu) << 8);
      off[u] = row * s + col * 8;
      col += ra;
      row += qa;
      if (col >= lpr) { col -= lpr; ++row; }
    }
    int4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (code[u]) v[u] = *reinterpret_cast<const int4*>(band_base + off[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t ch = code[u] >> 8;
      const uint32_t any = (code[u] | ch) & 0xffu;
      if (!any) continue;
      ncoded += __builtin_popcount(any);
      int32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int32_t l0 = (int16_t)(w[j] & 0xffff), l1 = w[j] >> 16;
        int32_t n0 = l0, n1 = l1;
        if ((any >> (2 * j)) & 1u) {
          n0 = min(max(l0 + (((ch >> (2 * j)) & 1u) ? P.lhit : P.lmiss), -lc), lc);
          dh += (long long)lut[n0 + lc] - (long long)lut[l0 + lc];
        }
        if ((any >> (2 * j + 1)) & 1u) {
          n1 = min(max(l1 + (((ch >> (2 * j + 1)) & 1u) ? P.lhit : P.lmiss), -lc), lc);
          dh += (long long)lut[n1 + lc] - (long long)lut[l1 + lc];
        }
        w[j] = (n0 & 0xffff) | (n1 << 16);
      }
      *reinterpret_cast<int4*>(band_base + off[u]) = make_int4(w[0], w[1], w[2], w[3]);
    }
  }
}

constexpr int kApplyInFlight = 4;

// The map update's mark pass over one band: the MISS bit of every cell the walks of all rays visit
// inside the band and the HIT bit of each hit's last cell, for rays from the Q16 origin (eox, eoy)
// with heading index ib of ray 0 and the ranges of rho_lds; bit index (cy - by0) * rowbits + (cx - x0w).
// Two forms with identical results.  One lane per ray (mark_rays): lane slots ordered by the walk
// length, so a wave's trip count stays close to its lanes' own; the pass lasts as long as the longest
// walk.  Segments (mark_segments): a ray of n steps is cut into ceil(n / seg) segments and the lanes
// take the segments of all rays in turn, so the pass lasts about (total steps / lanes) steps plus a
// setup per segment; a segment starts from the DDA state after i0 steps in closed form: with the
// decision variable after i >= 1 steps in (-DY, DX] and equal to D0 + kx DX - (i - kx) DY, kx (the
// x steps among them) is floor((i DY - D0 + DX) / (DX + DY)).  Which is faster depends on how many
// robots share a CU (measured by the autotuner).
// Lane slots ordered by the walk length estimated from the range (once for all bands of mark_rays).
template <int NT>
__device__ void sort_mark_rays(const EnvParams& P, const int32_t* rho_lds, int32_t* perm, int32_t* hist, int32_t ib) {
  sort_rays<NT>(P.R, perm, hist, [&](int32_t k) {
    const int32_t dv = ray_dir(P, ib, k);
    const int32_t ab = abs((int32_t)(int16_t)(dv & 0xffff)) + abs(dv >> 16);
    return (int32_t)((((int64_t)(rho_lds[k] & 0x7fffffff) >> 16) * ab) >> 16);
  });
}

// perm: the lane slots of sort_mark_rays.
template <int NT>
__device__ void mark_rays(const EnvParams& P, const int32_t* rho_lds, const int32_t* perm, int32_t s, int32_t eox,
                          int32_t eoy, int32_t ib, int32_t by0, int32_t x0w, int32_t rowbits, uint32_t band_bits,
                          bool one_band, bool count_visits, uint32_t* miss, uint32_t* hitm, int32_t& uvisits) {
  const int32_t ecx = eox >> 16, ecy = eoy >> 16;
  for (int32_t k0 = 0; k0 < P.R; k0 += NT) {
    const int32_t j = k0 + (int32_t)threadIdx.x;
    const bool valid = j < P.R;
    const int32_t k = valid ? perm[j] : 0;
    RaySetup q{};
    int32_t wi = 0, sx = 0, sy = 0, D = 0, n = -1;
    bool hit = false;
    if (valid) {
      const int32_t pk = rho_lds[k];
      hit = pk < 0;
      const int32_t dv = ray_dir(P, ib, k);
      const int32_t a = (int16_t)(dv & 0xffff), b = dv >> 16;
      q = ray_setup(eox, eoy, a, b, pk & 0x7fffffff, s);
      wi = (ecy - by0) * rowbits + (ecx - x0w);
      sx = a > 0 ? 1 : -1;
      sy = b > 0 ? rowbits : -rowbits;
      D = q.D;
      n = q.n;
      if ((uint32_t)wi < band_bits) atomicOr(&miss[wi >> 5], 1u << (wi & 31));
    }
    const int32_t w0 = wi;
    // Uniform trip counts over the wave.  While every lane is within its
    // own count and the band holds the whole window, every step lands in
    // the bitmap (the window holds every visited cell), so the first
    // loop marks without tests; the word index is clamped only to keep
    // the store inside the bitmap.  The second loop finishes the longer
    // walks, testing each step.
    const int32_t nmax = wave_max_i32(n);
    const int32_t nmin = one_band ? wave_min_i32(valid ? n : 0) : 0;
    const uint32_t last_word = (band_bits >> 5) - 1u;
    int32_t i = 0;
    for (; i < nmin; ++i) {
      const bool stepx = D <= 0;
      wi += stepx ? sx : sy;
      D += stepx ? q.DX : -q.DY;
      atomicOr(&miss[min((uint32_t)wi >> 5, last_word)], 1u << (wi & 31));
    }
    for (; i < nmax; ++i) {
      const bool stepx = D <= 0;
      wi += stepx ? sx : sy;
      D += stepx ? q.DX : -q.DY;
      if (i < n && (uint32_t)wi < band_bits) atomicOr(&miss[wi >> 5], 1u << (wi & 31));
    }
    if (valid) {
      if (count_visits) uvisits += n + 1;
      const int32_t we = w0 + q.kx * sx + q.ky * sy;   // last visited cell
      if (hit && !q.gend && (uint32_t)we < band_bits) atomicOr(&hitm[we >> 5], 1u << (we & 31));
    }
  }
}

// nray and segoff: [R] LDS scratch.
template <int NT>
__device__ void mark_segments(const EnvParams& P, const int32_t* rho_lds, int32_t* nray, int32_t* segoff,
                              int32_t* hist, int32_t s, int32_t eox, int32_t eoy, int32_t ib, int32_t by0, int32_t x0w,
                              int32_t rowbits, uint32_t band_bits, bool one_band, bool count_visits, int32_t seg,
                              uint32_t* miss, uint32_t* hitm, int32_t& uvisits) {
  constexpr int NWAVE = NT / 64;
  const int32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t R = P.R;
  const int32_t w0 = ((eoy >> 16) - by0) * rowbits + ((eox >> 16) - x0w);   // the origin cell
  // per ray: its step count, the HIT bit of its last cell, its visits
  for (int32_t k = tid; k < R; k += NT) {
    const int32_t pk = rho_lds[k];
    const int32_t dv = ray_dir(P, ib, k);
    const int32_t a = (int16_t)(dv & 0xffff), b = dv >> 16;
    const RaySetup q = ray_setup(eox, eoy, a, b, pk & 0x7fffffff, s);
    nray[k] = q.n;
    const int32_t we = w0 + q.kx * (a > 0 ? 1 : -1) + q.ky * (b > 0 ? rowbits : -rowbits);   // last visited cell
    if (pk < 0 && !q.gend && (uint32_t)we < band_bits) atomicOr(&hitm[we >> 5], 1u << (we & 31));
    if (count_visits) uvisits += q.n + 1;
  }
  if (tid == 0 && (uint32_t)w0 < band_bits) atomicOr(&miss[w0 >> 5], 1u << (w0 & 31));   // every walk's first cell
  __syncthreads();
  // segment offsets: exclusive prefix sum of ceil(n / seg) over the rays (each thread a run of rays)
  const int32_t per = (R + NT - 1) / NT;
  const int32_t k0 = min(R, tid * per), k1 = min(R, k0 + per);
  int32_t loc = 0;
  for (int32_t k = k0; k < k1; ++k) loc += (nray[k] + seg - 1) / seg;
  int32_t inc = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) hist[wave] = inc;
  __syncthreads();
  int32_t run = inc - loc, nseg = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) {
    const int32_t t = hist[w];
    run += w < wave ? t : 0;
    nseg += t;
  }
  for (int32_t k = k0; k < k1; ++k) {
    segoff[k] = run;
    run += (nray[k] + seg - 1) / seg;
  }
  __syncthreads();
  const uint32_t last_word = (band_bits >> 5) - 1u;
  for (int32_t j0 = 0; j0 < nseg; j0 += NT) {
    const int32_t j = j0 + tid;
    const bool valid = j < nseg;
    int32_t wi = 0, D = 0, DX = 0, DY = 0, sx = 0, sy = 0, len = 0;
    if (valid) {
      // the ray of segment j: the last ray whose first segment is <= j
      int32_t lo = 0, hi = R - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (segoff[mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      const int32_t k = lo;
      const int32_t i0 = (j - segoff[k]) * seg;
      len = min(seg, nray[k] - i0);
      const int32_t dv = ray_dir(P, ib, k);
      const int32_t a = (int16_t)(dv & 0xffff), b = dv >> 16;
      const int32_t aa = abs(a), bb = abs(b);
      int32_t D0;
      if (aa == 0) { D0 = 1; }
      else if (bb == 0) { D0 = -1; }
      else {
        const int32_t fx = eox & 0xffff, fy = eoy & 0xffff;
        const int32_t ex0 = a > 0 ? kQ16 - fx : fx, ey0 = b > 0 ? kQ16 - fy : fy;
        D0 = ex0 * bb - ey0 * aa;
        DX = bb << 16;
        DY = aa << 16;
      }
      sx = a > 0 ? 1 : -1;
      sy = b > 0 ? rowbits : -rowbits;
      int32_t kx = 0;
      if (i0 > 0) {
        if (DX + DY == 0) {
          kx = D0 <= 0 ? i0 : 0;   // axis rays: x steps only (D = -1) or y steps only (D = 1)
        } else {
          // floor((i0 DY - D0 + DX) / (DX + DY)) in 32 bits: with D0 = 65536 q + rr (0 <= rr < 65536) and
          // M = i0 aa + bb - q >= 0 it is floor(M / (aa + bb)) when rr = 0, else floor((M - 1) / (aa + bb))
          const int32_t aa = DY >> 16, bb = DX >> 16;
          const int32_t q = D0 >> 16, rr = D0 & 0xffff;
          const int32_t M = i0 * aa + bb - q - (rr != 0 ? 1 : 0);
          kx = (int32_t)((uint32_t)M / (uint32_t)(aa + bb));
        }
      }
      const int32_t ky = i0 - kx;
      wi = w0 + kx * sx + ky * sy;
      D = D0 + (int32_t)((uint32_t)(kx * (DX >> 16) - ky * (DY >> 16)) << 16);
    }
    // Uniform trip counts over the wave.  While every lane is within its own segment and the band
    // holds the whole window, every step lands in the bitmap (the window holds every visited cell),
    // so the first loop marks without tests; the word index is clamped only to keep the store inside
    // the bitmap.  The second loop finishes the longer segments, testing each step.
    const int32_t nmax = wave_max_i32(len);
    const int32_t nmin = one_band ? wave_min_i32(len) : 0;
    int32_t i = 0;
    for (; i < nmin; ++i) {
      const bool stepx = D <= 0;
      wi += stepx ? sx : sy;
      D += stepx ? DX : -DY;
      atomicOr(&miss[min((uint32_t)wi >> 5, last_word)], 1u << (wi & 31));
    }
    for (; i < nmax; ++i) {
      const bool stepx = D <= 0;
      wi += stepx ? sx : sy;
      D += stepx ? DX : -DY;
      if (i < len && (uint32_t)wi < band_bits) atomicOr(&miss[wi >> 5], 1u << (wi & 31));
    }
  }
}

// Map update from the estimated pose with the measured ranges, then the
// reward.  rho_lds[k]: range (Q16) with bit 31 set when ray k hit.
template <int NT, bool SEG>
__device__ void update_and_reward(const EnvParams& P, const StepArgs& A, const RobotMeta& m, const LdsView& V,
                                  const LdsPlan& L, int32_t r) {
  constexpr int NWAVE = NT / 64;
  RobotShared* sh = V.sh;
  const int32_t* rho_lds = V.rho;
  uint32_t* uni = V.uni;
  const int32_t s = m.side;
  const int32_t eox = sh->eox, eoy = sh->eoy, ib = sh->ib_e;
  const int32_t ecx = eox >> 16, ecy = eoy >> 16;
  const bool inside = ecx >= 0 && ecx < s && ecy >= 0 && ecy < s;
  long long dh = 0;
  int32_t ncoded = 0, uvisits = 0;
  if (inside) {
    // code window: end-point box grown by 2 cells, clipped to the grid
    const int32_t x0 = max(0, sh->bx0 - 2), x1 = min(s - 1, sh->bx1 + 2);
    const int32_t y0 = max(0, sh->by0 - 2), y1 = min(s - 1, sh->by1 + 2);
    const int32_t x0w = x0 & ~31;
    const int32_t nw = (x1 >> 5) - (x0 >> 5) + 1;
    const int32_t rowbits = nw << 5;
    const int32_t band = L.band_rows;
    uint32_t* miss = uni;
    uint32_t* hitm = uni + band * nw;
    const int64_t base = m.cell_off;
    if (!SEG) sort_mark_rays<NT>(P, rho_lds, V.perm, V.hist, ib);
    for (int32_t by0 = y0; by0 <= y1; by0 += band) {
      const int32_t rows = min(band, y1 - by0 + 1);
      const uint32_t band_bits = (uint32_t)(rows * rowbits);
      const bool one_band = y1 - y0 + 1 <= band;
      {
        uint4* u4 = reinterpret_cast<uint4*>(uni);
        const int32_t nclr = (2 * band * nw + 3) >> 2;
        for (int32_t k = threadIdx.x; k < nclr; k += NT) u4[k] = make_uint4(0u, 0u, 0u, 0u);
      }
      __syncthreads();
      if (SEG)
        mark_segments<NT>(P, rho_lds, V.perm, V.seg, V.hist, s, eox, eoy, ib, by0, x0w, rowbits, band_bits, one_band,
                          by0 == y0, L.mark_seg, miss, hitm, uvisits);
      else
        mark_rays<NT>(P, rho_lds, V.perm, s, eox, eoy, ib, by0, x0w, rowbits, band_bits, one_band, by0 == y0, miss,
                      hitm, uvisits);
      __syncthreads();
      // apply: each coded cell once (8 cells = one 16-byte access per octet)
      apply_band<NT, kApplyInFlight>(P, miss, hitm, rows, nw, P.belief + base + (int64_t)by0 * s + x0w, s, V.lut, dh,
                                     ncoded);
      __syncthreads();
    }
  }
  dh = wave_sum_i64(dh);
  ncoded = wave_sum_i32(ncoded);
  uvisits = wave_sum_i32(uvisits);
  if ((threadIdx.x & 63) == 0) {
    sh->part[threadIdx.x >> 6] = dh;
    sh->dpart[threadIdx.x >> 6] = ncoded;
    if (uvisits) atomicAdd(&sh->cnt_upd, uvisits);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    int64_t dsum = 0;
    for (int w = 0; w < NWAVE; ++w) {
      tot += sh->part[w];
      dsum += sh->dpart[w];
    }
    int64_t* cnt = P.counters + 3 * (int64_t)r;
    cnt[0] += dsum;
    cnt[1] += sh->cnt_march;
    cnt[2] += sh->cnt_upd;
    P.cost[r] = sh->cnt_march + sh->cnt_upd;
    P.hq_total[r] += tot;
    const double rH = (double)(-tot) * (1.0 / 4294967296.0);
    const float* c = P.cov + 6 * (int64_t)r;
    const double det = cov_det(c);
    const double ld = det > 0.0 ? log(det) : log(1.17549435e-38);
    const int32_t col = sh->collided;
    double rew;
    if (P.reward_mode == 1) {
      const double u = det > 0.0 ? cbrt(det) : 0.0;
      rew = paper_reward(P, col, P.dcells[r], P.u_prev[r], u, (double)__int_as_float(sh->dmin_bits));
      P.u_prev[r] = u;
    } else {
      rew = (double)P.w_entropy * rH - (double)P.w_dopt * ld - (double)P.lambda_col * (double)col;
    }
    A.reward[r] = (float)rew;
    const int32_t t = P.step[r];
    A.done[r] = (uint8_t)(col || (P.episode_len > 0 && t >= P.episode_len));
    P.terms[2 * (int64_t)r] = (float)rH;
    P.terms[2 * (int64_t)r + 1] = (float)ld;
    P.draws[r] += 1;   // every step, with or without the caller's draws
  }
}

// ---------------------------------------------------------------- kernels

// Sixteen lanes per robot: five draw its normals, the first one moves it, all sixteen test the paper's
// proximity collision around the new position (the move stands).
constexpr int kMotionLanes = 16;

__global__ void k_motion(EnvParams P, StepArgs A) {
  const int32_t r = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / kMotionLanes);
  const int lane0 = (int)(threadIdx.x & 63) & ~(kMotionLanes - 1);
  const int sub = (int)(threadIdx.x & 63) - lane0;
  const bool valid = r < P.n;
  const MotionDraws g = motion_draws(P, A, r, valid, lane0);
  MotionOut o{};
  if (valid && sub == 0) o = robot_motion(P, A, r, g);
  const int32_t tox = __shfl(o.tox, lane0, 64), toy = __shfl(o.toy, lane0, 64);
  const int32_t col = __shfl(o.collided, lane0, 64);
  bool near = false;
  if (valid && P.crash_q > 0 && !col) {
    const RobotMeta m = P.meta[r];
    near = near_obstacle_part(P.world + m.world_off, m.side, tox, toy, P.crash_q, sub, kMotionLanes);
  }
  const uint64_t b = __builtin_amdgcn_ballot_w64(near);
  if (valid && sub == 0 && ((b >> lane0) & ((1ull << kMotionLanes) - 1ull)) != 0) P.flags[2 * (int64_t)r] = 1;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_march(EnvParams P, StepArgs A, LdsPlan L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsView V = lds_view(smem, L);
  RobotShared* sh = V.sh;
  const int32_t r = blockIdx.x;
  const RobotMeta m = P.meta[r];
  if (threadIdx.x == 0) {
    const float* p = P.pose + 3 * (int64_t)r;
    sh->tox = to_q16(p[0], P.inv_c16);
    sh->toy = to_q16(p[1], P.inv_c16);
    sh->ib_t = fan_base(P, heading_index(p[2], P.k_ang));
    sh->cnt_march = 0;
    sh->dmin_bits = 0x7f800000;
  }
  __syncthreads();
  int32_t wy0;
  uint32_t* sw = V.uni + march_guard_words(m.side);
  stage_world<NT>(P, m, sh->toy >> 16, L.world_halo, sw, wy0);
  __syncthreads();
  march_rays<NT>(P, m, V, sw, wy0, A.ranges, step_noise(P, A, r), true, r);
  if (threadIdx.x == 0) {
    P.counters[3 * (int64_t)r + 1] += sh->cnt_march;
    P.dmin_bits[r] = sh->dmin_bits;
  }
}

__device__ __forceinline__ void init_bbox(RobotShared* sh) {
  sh->bx0 = 0x7fffffff; sh->bx1 = -0x7fffffff;
  sh->by0 = 0x7fffffff; sh->by1 = -0x7fffffff;
}

// SEG: the map update's walk in segments (its own instance: the two forms differ in register use).
template <int NT, bool SEG>
__global__ __launch_bounds__(NT) void k_update(EnvParams P, StepArgs A, LdsPlan L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsView V = lds_view(smem, L);
  RobotShared* sh = V.sh;
  const int32_t r = blockIdx.x;
  const RobotMeta m = P.meta[r];
  for (int32_t i = threadIdx.x; i < 2 * P.lclamp + 1; i += NT) V.lut[i] = P.hq_lut[i];
  if (threadIdx.x == 0) {
    const float* e = P.est + 3 * (int64_t)r;
    sh->eox = to_q16(e[0], P.inv_c16);
    sh->eoy = to_q16(e[1], P.inv_c16);
    sh->ib_e = fan_base(P, heading_index(e[2], P.k_ang));
    sh->collided = P.flags[2 * (int64_t)r];
    sh->cnt_march = 0;
    sh->cnt_upd = 0;
    sh->dmin_bits = P.dmin_bits[r];
    init_bbox(sh);
  }
  for (int32_t k = threadIdx.x; k < P.R; k += NT) {
    const int32_t rq = P.rho[(int64_t)r * P.R + k];
    const int32_t hc = P.hitc[(int64_t)r * P.R + k];
    V.rho[k] = rq | (hc >= 0 ? (int32_t)0x80000000 : 0);
  }
  __syncthreads();
  endpoint_bbox<NT>(P, V.rho, sh->eox, sh->eoy, sh->ib_e, sh);
  __syncthreads();
  update_and_reward<NT, SEG>(P, A, m, V, L, r);
}

// One robot of the fused step (motion, march, update, reward) by the whole workgroup.
template <int NT, bool SEG>
__device__ __forceinline__ void fused_robot(const EnvParams& P, const StepArgs& A, const LdsPlan& L,
                                            const LdsView& V, int32_t r) {
  RobotShared* sh = V.sh;
  const RobotMeta m = P.meta[r];
  if (threadIdx.x < 64) {   // wave 0: lanes 0..4 draw the normals, lane 0 moves the robot
    const MotionDraws g = motion_draws(P, A, r, true, 0);
    if (threadIdx.x == 0) {
      const MotionOut o = robot_motion(P, A, r, g);
      sh->tox = o.tox; sh->toy = o.toy; sh->ib_t = o.ib_t;
      sh->eox = o.eox; sh->eoy = o.eoy; sh->ib_e = o.ib_e;
      sh->collided = o.collided;
      sh->cnt_march = 0;
      sh->cnt_upd = 0;
      sh->dmin_bits = 0x7f800000;
      sh->near = 0;
      init_bbox(sh);
    }
  }
  __syncthreads();
  // the paper's proximity collision (the move stands), one cell per thread
  const bool prox = P.crash_q > 0 && !sh->collided;
  if (prox) near_obstacle_wg<NT>(P.world + m.world_off, m.side, sh->tox, sh->toy, P.crash_q, &sh->near);
  int32_t wy0;
  uint32_t* sw = V.uni + march_guard_words(m.side);
  stage_world<NT>(P, m, sh->toy >> 16, L.world_halo, sw, wy0);
  __syncthreads();
  if (prox && threadIdx.x == 0 && sh->near) {
    sh->collided = 1;
    P.flags[2 * (int64_t)r] = 1;
  }
  march_rays<NT>(P, m, V, sw, wy0, A.ranges, step_noise(P, A, r), L.record != 0, r);
  endpoint_bbox<NT>(P, V.rho, sh->eox, sh->eoy, sh->ib_e, sh);
  __syncthreads();
  update_and_reward<NT, SEG>(P, A, m, V, L, r);
}

// The fused step's order of robots, the most work first (largest-processing-time order): a counting
// sort of the robots' last-step DDA visits into 1024 buckets, one workgroup.  A CU takes its workgroups
// in launch order and its SIMDs issue the oldest waves first, so the robot a CU got last runs on what
// the others leave; with the heaviest robots first and the lightest last, the CUs' robots end together
// instead of the last-placed heavy ones setting the launch's length.  Robots are independent: the order
// changes no result.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 1024;

__global__ __launch_bounds__(kOrderThreads) void k_order(int32_t n, const int32_t* __restrict__ cost,
                                                         int32_t* __restrict__ order) {
  __shared__ int32_t s_hist[kOrderBuckets];
  __shared__ int32_t s_max[kOrderThreads / 64];
  const int32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int32_t mx = 0;
  for (int32_t r = tid; r < n; r += kOrderThreads) mx = max(mx, cost[r]);
  mx = wave_max_i32(mx);
  if (lane == 0) s_max[wave] = mx;
  for (int32_t b = tid; b < kOrderBuckets; b += kOrderThreads) s_hist[b] = 0;
  __syncthreads();
  mx = 0;
  for (int w = 0; w < kOrderThreads / 64; ++w) mx = max(mx, s_max[w]);
  const int32_t q = mx / kOrderBuckets + 1;
  for (int32_t r = tid; r < n; r += kOrderThreads) atomicAdd(&s_hist[kOrderBuckets - 1 - min(cost[r] / q, kOrderBuckets - 1)], 1);
  __syncthreads();
  // exclusive prefix sum of the buckets (the heaviest bucket first), one bucket per thread
  const int32_t v = tid < kOrderBuckets ? s_hist[tid] : 0;
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) s_max[wave] = x;
  __syncthreads();
  int32_t base = 0;
  for (int w = 0; w < wave; ++w) base += s_max[w];
  if (tid < kOrderBuckets) s_hist[tid] = base + x - v;
  __syncthreads();
  for (int32_t r = tid; r < n; r += kOrderThreads)
    order[atomicAdd(&s_hist[kOrderBuckets - 1 - min(cost[r] / q, kOrderBuckets - 1)], 1)] = r;
}

// Fused step, one workgroup per robot: workgroup b takes the b-th robot of the most-work-first order.  The segmented instance
// is held to 80 VGPRs (six waves per SIMD: three 512-thread workgroups per CU, every robot of a
// 750-robot batch resident at once); unbounded it takes 89 and fits two, which costs more than the
// few spilled values do.
template <int NT, bool SEG>
__global__ __launch_bounds__(NT, SEG ? 6 : 1) void k_fused(EnvParams P, StepArgs A, LdsPlan L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsView V = lds_view(smem, L);
  for (int32_t i = threadIdx.x; i < 2 * P.lclamp + 1; i += NT) V.lut[i] = P.hq_lut[i];
  fused_robot<NT, SEG>(P, A, L, V, P.order[blockIdx.x]);
}

// Fused persistent step on a smaller grid: workgroups pull robots in largest-grid-first
// order.  The register budget is capped at four waves per SIMD (128 VGPRs); the
// loop-carried state would otherwise double it.
template <int NT, bool SEG>
__global__ __launch_bounds__(NT, 4) void k_fused_persist(EnvParams P, StepArgs A, LdsPlan L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LdsView V = lds_view(smem, L);
  for (int32_t i = threadIdx.x; i < 2 * P.lclamp + 1; i += NT) V.lut[i] = P.hq_lut[i];
  for (int32_t w = blockIdx.x; w < P.n; w += gridDim.x) {
    fused_robot<NT, SEG>(P, A, L, V, P.order[w]);
    __syncthreads();
  }
}

// Robot r = blockIdx.x; its maps are cleared by gridDim.y workgroups, each taking a contiguous
// share; workgroup y = 0 also resets the per-robot state.
template <bool kVecSrc>   // world_src on a 16-byte boundary: the world copy in 16-byte vectors
__global__ void k_reset(EnvParams P, const uint32_t* world_src, const float* init_pose, const uint8_t* mask) {
  const int32_t r = blockIdx.x;
  if (mask && !mask[r]) return;
  const RobotMeta m = P.meta[r];
  const int32_t s = m.side;
  const int64_t ny = gridDim.y, y = blockIdx.y;
  auto share = [&](int64_t total, int64_t& b, int64_t& e) {
    const int64_t per = (total + ny - 1) / ny;
    b = min(total, y * per);
    e = min(total, b + per);
  };
  int64_t b0, e0;
  // sides are multiples of 32, so a robot's map (s^2 int16) and world (s^2 / 32 words) are whole 16-byte
  // vectors starting on 16-byte boundaries
  uint4* bel = reinterpret_cast<uint4*>(P.belief + m.cell_off);
  share((int64_t)s * s / 8, b0, e0);
  for (int64_t k = b0 + threadIdx.x; k < e0; k += blockDim.x) bel[k] = make_uint4(0u, 0u, 0u, 0u);
  if (kVecSrc) {
    uint4* wd = reinterpret_cast<uint4*>(const_cast<uint32_t*>(P.world) + m.world_off);
    const uint4* ws = reinterpret_cast<const uint4*>(world_src + m.world_off);
    share((int64_t)s * s / 128, b0, e0);
    for (int64_t k = b0 + threadIdx.x; k < e0; k += blockDim.x) wd[k] = ws[k];
  } else {
    uint32_t* wd = const_cast<uint32_t*>(P.world) + m.world_off;
    const uint32_t* ws = world_src + m.world_off;
    share((int64_t)s * s / 32, b0, e0);
    for (int64_t k = b0 + threadIdx.x; k < e0; k += blockDim.x) wd[k] = ws[k];
  }
  if (P.uses_visits) {
    share((int64_t)m.visit_side * m.visit_side, b0, e0);
    for (int64_t k = b0 + threadIdx.x; k < e0; k += blockDim.x) {
      P.visit_t[m.visit_off + k] = -1;
      P.visit_xy[2 * (m.visit_off + k)] = 0.0f;
      P.visit_xy[2 * (m.visit_off + k) + 1] = 0.0f;
      P.visit_last[m.visit_off + k] = -1;
    }
  }
  if (y != 0) return;
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      P.pose[3 * (int64_t)r + k] = init_pose[3 * (int64_t)r + k];
      P.est[3 * (int64_t)r + k] = init_pose[3 * (int64_t)r + k];
    }
    float* c = P.cov + 6 * (int64_t)r;
    c[0] = P.var0_xy; c[1] = 0.0f; c[2] = 0.0f;
    c[3] = P.var0_xy; c[4] = 0.0f; c[5] = P.var0_th;
    P.hq_total[r] = (int64_t)s * (int64_t)s * (int64_t)P.hq_lut[P.lclamp];
    P.step[r] = 0;
    P.last_lc[r] = -(1 << 30);
    P.prev_vcell[r] = -1;
    P.u_prev[r] = uncertainty(c);
    P.dcells[r] = 0.0;
    P.dmin_bits[r] = 0x7f800000;
    P.flags[2 * (int64_t)r] = 0;
    P.flags[2 * (int64_t)r + 1] = 0;
    P.counters[3 * (int64_t)r] = 0;
    P.counters[3 * (int64_t)r + 1] = 0;
    P.counters[3 * (int64_t)r + 2] = 0;
  }
  for (int32_t k = threadIdx.x; k < P.R; k += blockDim.x) P.raylen[(int64_t)r * P.R + k] = 0;
}

__global__ void k_observe(EnvParams P, const float* ranges, int16_t* crop, int32_t cs, float* scan, float* state,
                          float inv_r, float inv_pi, const float* u_new, double alpha) {
  const int32_t r = blockIdx.x;
  const RobotMeta m = P.meta[r];
  const int32_t s = m.side;
  const float* e = P.est + 3 * (int64_t)r;
  const int32_t ecx = to_q16(e[0], P.inv_c16) >> 16;
  const int32_t ecy = to_q16(e[1], P.inv_c16) >> 16;
  const int16_t* bel = P.belief + m.cell_off;
  int16_t* out = crop + (int64_t)r * cs * cs;
  // eight crop cells per item: cells i0 .. i0 + 7 of row j lie in the grid row's octets floor(i0 / 8)
  // and the next (rows start on 64-byte boundaries, s being a multiple of 32), so an item is two
  // aligned 16-byte loads (an octet outside the row reads as zeros, which are the cells off the grid)
  // funnel-shifted into place, and one 16-byte store when the crop side is a multiple of 8
  const int32_t chunks = (cs + 7) >> 3;
  const int32_t octs = s >> 3;
  for (int32_t q = threadIdx.x; q < cs * chunks; q += blockDim.x) {
    const int32_t jj = q / chunks, i8 = (q - jj * chunks) * 8;
    const int32_t j = ecy - cs / 2 + jj, i0 = ecx - cs / 2 + i8;
    uint64_t w[4] = {0ull, 0ull, 0ull, 0ull};
    if (j >= 0 && j < s) {
      const int32_t k0 = i0 >> 3;   // floor
      const uint4* row = reinterpret_cast<const uint4*>(bel + (int64_t)j * s);
      if (k0 >= 0 && k0 < octs) {
        const uint4 a = row[k0];
        w[0] = a.x | ((uint64_t)a.y << 32);
        w[1] = a.z | ((uint64_t)a.w << 32);
      }
      if (k0 + 1 >= 0 && k0 + 1 < octs) {
        const uint4 b = row[k0 + 1];
        w[2] = b.x | ((uint64_t)b.y << 32);
        w[3] = b.z | ((uint64_t)b.w << 32);
      }
    }
    // the eight cells start at bit 16 (i0 & 7) of the 256-bit concatenation w[0] .. w[3]
    const int32_t bit = 16 * (i0 & 7);
    const int32_t wi = bit >> 6, bs = bit & 63;
    const uint64_t x0 = wi ? w[1] : w[0], x1 = wi ? w[2] : w[1], x2 = wi ? w[3] : w[2];
    const uint64_t lo = bs ? (x0 >> bs) | (x1 << (64 - bs)) : x0;
    const uint64_t hi = bs ? (x1 >> bs) | (x2 << (64 - bs)) : x1;
    int16_t* dst = out + (int64_t)jj * cs + i8;
    if ((cs & 7) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
      *reinterpret_cast<uint4*>(dst) = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    } else {
      for (int e = 0; e < 8 && i8 + e < cs; ++e) dst[e] = (int16_t)((e < 4 ? lo >> (16 * e) : hi >> (16 * (e - 4))) & 0xffffu);
    }
  }
  for (int32_t k = threadIdx.x; k < P.R; k += blockDim.x)
    scan[(int64_t)r * P.R + k] = ranges[(int64_t)r * P.R + k] * inv_r;
  if (threadIdx.x == 0) {
    const float* c = P.cov + 6 * (int64_t)r;
    float* o = state + 12 * (int64_t)r;
    if (P.reward_mode == 1) {
      // Eq. (3): [LiDAR, yaw, U_t]; yaw of the true heading (IMU), U_t of the filter
      for (int k = 2; k < 12; ++k) o[k] = 0.0f;
      o[0] = P.pose[3 * (int64_t)r + 2] * inv_pi;
      double u = uncertainty(c);
      // uncertainty bridge (Sec. III-G): blend in the external estimator's U
      if (u_new) u = alpha * (double)u_new[r] + (1.0 - alpha) * u;
      o[1] = (float)u;
    } else {
      const float inv_ext = m.inv_ext;
      o[0] = e[0] * inv_ext; o[1] = e[1] * inv_ext; o[2] = e[2] * inv_pi;
      o[3] = c[0]; o[4] = c[1]; o[5] = c[2];
      o[6] = c[1]; o[7] = c[3]; o[8] = c[4];
      o[9] = c[2]; o[10] = c[4]; o[11] = c[5];
    }
  }
}

// ---------------------------------------------------------------- fixed-lag backend
//
// The step with the fixed-lag SLAM backbone of Sec. III-D in place of the EKF: motion, prediction and
// visits (k_motion), the LiDAR march (k_march), the scan-matching inputs (k_fl_prep), the correlative
// search, the alignment and the window's new pose and factors (k_fl_window), Gauss-Newton over the
// window, the weighted integration of the aligned scan, then the estimates and covariance back into the
// state and the reward of Eq. (7) (k_fl_post_reward).  The estimate is the aligned pose (integer work),
// the window only yields the covariance; see the C-ABI header for the rules.

// Predicted pose (Q16 x, y, heading index) and the scan: reported ranges of the rays that hit.
__global__ void k_fl_prep(EnvParams P, FixedLag F) {
  const int64_t total = (int64_t)P.n * P.R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / P.R;
    F.rho_q[i] = P.hitc[i] >= 0 ? P.rho[i] : -1;
    if (i - r * P.R == 0) {
      const float* e = P.est + 3 * r;
      F.pose_q[3 * r] = to_q16(e[0], P.inv_c16);
      F.pose_q[3 * r + 1] = to_q16(e[1], P.inv_c16);
      F.pose_q[3 * r + 2] = heading_index(e[2], P.k_ang);
    }
  }
}

// One wave per robot: the alignment, the estimate, and the window's new pose with its odometry and
// scan factors (the oldest pose leaves a full window, the next one taking the prior).  The slide of a
// full window moves up to 18 L doubles; the wave's lanes move them together, every value loaded before
// any is stored (the stores land below the loads, so none overwrites an element still to be read).
constexpr int kFlLanes = 64;
constexpr int kFlPer = (6 * slam::kMaxWindow + kFlLanes - 1) / kFlLanes;   // elements per lane and array

__device__ __forceinline__ void fl_shift_load(const double* a, int n, int off, int lane, double (&v)[kFlPer]) {
#pragma unroll
  for (int q = 0; q < kFlPer; ++q) {
    const int e = lane + kFlLanes * q;
    v[q] = e < n ? a[e + off] : 0.0;
  }
}

__device__ __forceinline__ void fl_shift_store(double* a, int n, int lane, const double (&v)[kFlPer]) {
#pragma unroll
  for (int q = 0; q < kFlPer; ++q) {
    const int e = lane + kFlLanes * q;
    if (e < n) a[e] = v[q];
  }
}

__global__ void k_fl_window(EnvParams P, FixedLag F) {
  const int32_t r = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kFlLanes);
  const int lane = (int)(threadIdx.x & (kFlLanes - 1));
  if (r >= P.n) return;   // uniform over the wave
  const int L = F.L;
  double* x = F.x + (int64_t)r * L * 3;
  double* od = F.odo + (int64_t)r * (L - 1) * 6;
  double* sc = F.scan + (int64_t)r * L * 6;
  double* sg = F.sig + (int64_t)r * L * 3;
  int c = F.count[r];
  if (c == L) {
    double vx[kFlPer], vs[kFlPer], vc[kFlPer], vo[kFlPer];
    fl_shift_load(x, 3 * (L - 1), 3, lane, vx);
    fl_shift_load(sg, 3 * (L - 1), 3, lane, vs);
    fl_shift_load(sc, 6 * (L - 1), 6, lane, vc);
    fl_shift_load(od, 6 * (L - 2), 6, lane, vo);
    fl_shift_store(x, 3 * (L - 1), lane, vx);
    fl_shift_store(sg, 3 * (L - 1), lane, vs);
    fl_shift_store(sc, 6 * (L - 1), lane, vc);
    fl_shift_store(od, 6 * (L - 2), lane, vo);
    if (lane < 3) {   // the new oldest pose's prior: its estimate, the inverse of its covariance diagonal
      double* pr = F.prior + 6 * (int64_t)r;
      pr[lane] = vx[0];
      pr[3 + lane] = 1.0 / vs[0];
    }
    c = L - 1;
  }
  if (lane != 0) return;
  const int32_t* m = F.match + 6 * (int64_t)r;
  const double w = slam::match_weight(m, F.l_max);
  const int64_t px = F.pose_q[3 * r], py = F.pose_q[3 * r + 1], ph = F.pose_q[3 * r + 2];
  int64_t ax = px, ay = py, ah = ph;
  if (w > 0.0) {
    ax = px + (int64_t)m[0] * F.step_xy;
    ay = py + (int64_t)m[1] * F.step_xy;
    ah = (ph + (int64_t)m[2] * F.step_h) % kNang;
    if (ah < 0) ah += kNang;
  }
  F.pose_al[3 * r] = (int32_t)ax;
  F.pose_al[3 * r + 1] = (int32_t)ay;
  F.pose_al[3 * r + 2] = (int32_t)ah;
  const double two_pi = 2.0 * M_PI;
  double th = (two_pi * (double)ah) / (double)kNang;
  th = th - two_pi * rint(th / two_pi);
  const double z[3] = {(double)ax / 65536.0 * F.cell, (double)ay / 65536.0 * F.cell, th};
  float* e = P.est + 3 * (int64_t)r;
  e[0] = (float)z[0];
  e[1] = (float)z[1];
  e[2] = (float)z[2];
  const double d = (double)P.odo_u[2 * (int64_t)r], phi = (double)P.odo_u[2 * (int64_t)r + 1];
  double* o = od + 6 * (c - 1);
  o[0] = d; o[1] = 0.0; o[2] = phi;
  o[3] = F.odo_info[0]; o[4] = F.odo_info[1]; o[5] = F.odo_info[2];
  for (int a = 0; a < 3; ++a) {
    sc[6 * c + a] = z[a];
    sc[6 * c + 3 + a] = w * F.scan_info[a];
    x[3 * c + a] = z[a];
  }
  F.count[r] = c + 1;
  F.wq[r] = (int32_t)rint(256.0 * (F.floor + (1.0 - F.floor) * w));
}

// One wave per robot, after the weighted integration: the window's solution back into the state (poses
// by all lanes); then lane 0 writes the FP32 covariance entries of the newest pose and its covariance
// diagonal (the prior the pose will carry as the oldest), and forms Eq. (7) with U_t of that covariance,
// done, terms, work counters and the draw counter.
__global__ void k_fl_post_reward(EnvParams P, StepArgs A, FixedLag F) {
  const int32_t r = (int32_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kFlLanes);
  const int lane = (int)(threadIdx.x & (kFlLanes - 1));
  if (r >= P.n) return;
  const int L = F.L, cnt = F.count[r];
  const double* xo = F.xout + (int64_t)r * L * 3;
  double* x = F.x + (int64_t)r * L * 3;
  for (int e = lane; e < 3 * cnt; e += kFlLanes) x[e] = xo[e];
  if (lane != 0) return;
  const double* S = F.covw + 9 * (int64_t)r;
  float* cv = P.cov + 6 * (int64_t)r;
  cv[0] = (float)S[0]; cv[1] = (float)S[1]; cv[2] = (float)S[2];
  cv[3] = (float)S[4]; cv[4] = (float)S[5]; cv[5] = (float)S[8];
  double* sg = F.sig + ((int64_t)r * L + (cnt - 1)) * 3;
  sg[0] = S[0]; sg[1] = S[4]; sg[2] = S[8];
  if (F.coded[r] > 0) P.counters[3 * (int64_t)r] += F.coded[r];
  const double det = cov_det(cv);
  const double ld = det > 0.0 ? log(det) : log(1.17549435e-38);
  const double u = det > 0.0 ? cbrt(det) : 0.0;
  const int32_t col = P.flags[2 * (int64_t)r];
  const double rew = paper_reward(P, col, P.dcells[r], P.u_prev[r], u, (double)__int_as_float(P.dmin_bits[r]));
  P.u_prev[r] = u;
  A.reward[r] = (float)rew;
  const int32_t t = P.step[r];
  A.done[r] = (uint8_t)(col || (P.episode_len > 0 && t >= P.episode_len));
  P.terms[2 * (int64_t)r] = 0.0f;
  P.terms[2 * (int64_t)r + 1] = (float)ld;
  P.draws[r] += 1;
}

// Masked reset of the windows: the initial pose with the prior (pose, 1 / var0), no scan factor.
__global__ void k_fl_reset(int32_t n, FixedLag F, const float* init_pose, const uint8_t* mask) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || (mask && !mask[r])) return;
  const int L = F.L;
  double* x = F.x + (int64_t)r * L * 3;
  double* pr = F.prior + 6 * (int64_t)r;
  double* sc = F.scan + (int64_t)r * L * 6;
  double* sg = F.sig + (int64_t)r * L * 3;
  for (int a = 0; a < 3; ++a) {
    x[a] = (double)init_pose[3 * (int64_t)r + a];
    pr[a] = x[a];
    pr[3 + a] = 1.0 / F.var0[a];
    sg[a] = F.var0[a];
  }
  for (int a = 0; a < 6; ++a) sc[a] = 0.0;
  F.count[r] = 1;
}

template <int NT>
hipError_t fixedlag_nt(const EnvParams& P, const StepArgs& A, const LdsPlan& L, const FixedLag& F, hipStream_t st) {
  k_motion<<<(unsigned)(((int64_t)P.n * kMotionLanes + 255) / 256), 256, 0, st>>>(P, A);
  k_march<NT><<<P.n, NT, L.total, st>>>(P, A, L);
  const int64_t items = (int64_t)P.n * P.R;
  k_fl_prep<<<(unsigned)std::min<int64_t>(4096, (items + 255) / 256), 256, 0, st>>>(P, F);
  hipError_t e = slam::launch_csm_match(P.dirtab, P.belief, F.cell_off, F.side, F.max_side, P.n, F.pose_q, F.rho_q,
                                        P.R, F.a_off, F.W, F.V, F.step_xy, F.step_h, F.match, st);
  if (e != hipSuccess) return e;
  const unsigned wave_blocks = (unsigned)(((int64_t)P.n * kFlLanes + 255) / 256);
  k_fl_window<<<wave_blocks, 256, 0, st>>>(P, F);
  e = slam::launch_fixedlag(P.n, F.L, F.count, F.x, F.prior, F.odo, F.scan, F.iters, F.xout, F.covw, st);
  if (e != hipSuccess) return e;
  e = slam::launch_csm_integrate(P.dirtab, P.belief, F.cell_off, F.side, P.n, F.pose_al, F.rho_q, P.R, F.a_off,
                                 F.max_side, P.rhat_q, nullptr, 0, 0, 1.0, P.lhit, P.lmiss, P.lclamp, F.coded, F.wq,
                                 st);
  if (e != hipSuccess) return e;
  k_fl_post_reward<<<wave_blocks, 256, 0, st>>>(P, A, F);
  return hipGetLastError();
}

template <int NT>
hipError_t plain_nt(const EnvParams& P, const StepArgs& A, const LdsPlan& L, hipStream_t st) {
  k_motion<<<(unsigned)(((int64_t)P.n * kMotionLanes + 255) / 256), 256, 0, st>>>(P, A);
  k_march<NT><<<P.n, NT, L.total, st>>>(P, A, L);
  if (L.mark_seg > 0) k_update<NT, true><<<P.n, NT, L.total, st>>>(P, A, L);
  else k_update<NT, false><<<P.n, NT, L.total, st>>>(P, A, L);
  return hipGetLastError();
}

template <int NT>
hipError_t fused_nt(const EnvParams& P, const StepArgs& A, const LdsPlan& L, int grid, bool order, hipStream_t st) {
  const bool seg = L.mark_seg > 0;
  if (order && P.n > 1) k_order<<<1, kOrderThreads, 0, st>>>(P.n, P.cost, P.order);
  if (grid >= P.n) {
    if (seg) k_fused<NT, true><<<P.n, NT, L.total, st>>>(P, A, L);
    else k_fused<NT, false><<<P.n, NT, L.total, st>>>(P, A, L);
  } else {
    if (seg) k_fused_persist<NT, true><<<grid, NT, L.total, st>>>(P, A, L);
    else k_fused_persist<NT, false><<<grid, NT, L.total, st>>>(P, A, L);
  }
  return hipGetLastError();
}

template <int NT>
hipError_t set_lds_nt(int bytes) {
  hipError_t e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_march<NT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  const void* fns[] = {reinterpret_cast<const void*>(&k_update<NT, false>),
                       reinterpret_cast<const void*>(&k_update<NT, true>),
                       reinterpret_cast<const void*>(&k_fused<NT, false>),
                       reinterpret_cast<const void*>(&k_fused<NT, true>),
                       reinterpret_cast<const void*>(&k_fused_persist<NT, false>),
                       reinterpret_cast<const void*>(&k_fused_persist<NT, true>)};
  for (const void* f : fns)
    if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace

constexpr int kResetSplit = 8;   // workgroups per reset robot

hipError_t launch_reset(const EnvParams& P, const uint32_t* world_src, const float* init_pose,
                        const uint8_t* mask, int32_t, hipStream_t stream) {
  const dim3 grid(P.n, kResetSplit);
  if ((reinterpret_cast<uintptr_t>(world_src) & 15) == 0) k_reset<true><<<grid, 256, 0, stream>>>(P, world_src, init_pose, mask);
  else k_reset<false><<<grid, 256, 0, stream>>>(P, world_src, init_pose, mask);
  return hipGetLastError();
}

hipError_t launch_step_plain(const EnvParams& P, const StepArgs& A, const LdsPlan& L, int threads,
                             hipStream_t stream) {
  switch (threads) {
    case 128: return plain_nt<128>(P, A, L, stream);
    case 192: return plain_nt<192>(P, A, L, stream);
    case 256: return plain_nt<256>(P, A, L, stream);
    case 384: return plain_nt<384>(P, A, L, stream);
    case 512: return plain_nt<512>(P, A, L, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_fused(const EnvParams& P, const StepArgs& A, const LdsPlan& L, int threads, int grid,
                             bool order, hipStream_t stream) {
  switch (threads) {
    case 128: return fused_nt<128>(P, A, L, grid, order, stream);
    case 192: return fused_nt<192>(P, A, L, grid, order, stream);
    case 256: return fused_nt<256>(P, A, L, grid, order, stream);
    case 384: return fused_nt<384>(P, A, L, grid, order, stream);
    case 512: return fused_nt<512>(P, A, L, grid, order, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_fixedlag(const EnvParams& P, const StepArgs& A, const LdsPlan& L, const FixedLag& F,
                                int threads, hipStream_t stream) {
  switch (threads) {
    case 128: return fixedlag_nt<128>(P, A, L, F, stream);
    case 192: return fixedlag_nt<192>(P, A, L, F, stream);
    case 256: return fixedlag_nt<256>(P, A, L, F, stream);
    case 384: return fixedlag_nt<384>(P, A, L, F, stream);
    case 512: return fixedlag_nt<512>(P, A, L, F, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reset_fixedlag(const EnvParams& P, const FixedLag& F, const float* init_pose, const uint8_t* mask,
                                 hipStream_t stream) {
  k_fl_reset<<<(P.n + 255) / 256, 256, 0, stream>>>(P.n, F, init_pose, mask);
  return hipGetLastError();
}

hipError_t launch_observe(const EnvParams& P, const float* ranges, int16_t* crop, int32_t cs, float* scan,
                          float* state, const float* u_new, double alpha, hipStream_t stream) {
  k_observe<<<P.n, 256, 0, stream>>>(P, ranges, crop, cs, scan, state, P.inv_rmax, P.inv_pi, u_new, alpha);
  return hipGetLastError();
}

hipError_t set_kernel_lds_limits(int bytes) {
  hipError_t e;
  if ((e = set_lds_nt<128>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_nt<192>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_nt<256>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_nt<384>(bytes)) != hipSuccess) return e;
  return set_lds_nt<512>(bytes);
}

}  // namespace aslam
