// slam.hip -- the fixed-lag SLAM backbone on gfx950 (arXiv 2603.25834, Sec. III-D).
//
// Four batched calls, one robot (or pose window) per workgroup or thread:
//  * correlative scan matching: every candidate of a (dx, dy, dheading) lattice around the predicted
//    pose scored against the robot's int16 log-odds grid -- exact integer arithmetic (Q16 positions,
//    the Q14 heading table), so results equal the definition bit for bit;
//  * the scan factor of a match: the best pose and an information matrix scaled by the normalised
//    score and the margin to the second-best separate peak;
//  * the fixed-lag pose graph: a few Gauss-Newton steps over a window of L poses (a prior on the
//    oldest, odometry factors between neighbours, unary scan factors) in FP64, solved by block
//    elimination of the block-tridiagonal normal equations; the newest pose's marginal covariance,
//    the last diagonal block of the inverse Hessian, is the inverse of the last Schur complement;
//  * the confidence-weighted map integration: the scan cast into the grid from the matched pose by
//    the exact traversal of the env step's map update, each coded cell's log-odds increment scaled by
//    the match weight quantised to 1/256.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "aslam.h"
#include "env_internal.h"
#include "slam_internal.h"

namespace aslam {
void set_last_error(const std::string& msg);
}

namespace {

using aslam::kDirOne;
using aslam::kNang;

int sfail(int code, const std::string& m) {
  aslam::set_last_error(m);
  return code;
}

#define SCHK(call)                                                            \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) return sfail(ASL_EHIP, hipGetErrorString(e_));      \
  } while (0)

constexpr int kCsmThreads = 256;
constexpr int kCsmMaxHalf = 8;                      // W, V <= 8
constexpr int kCsmMaxRayHeadings = 8192;            // (2V + 1) * R ray offsets staged in LDS
constexpr int kCsmMaxCand = (2 * kCsmMaxHalf + 1) * (2 * kCsmMaxHalf + 1) * (2 * kCsmMaxHalf + 1);
constexpr int64_t kCsmLdsBudget = 163840 - 64;      // dynamic LDS of the staged kernel (160 KB less its reductions)

// ------------------------------------------------------------------ correlative scan matching

// One workgroup per robot.  Stage: the endpoint offsets (Q16) of every ray under every heading
// candidate.  Score: each thread takes candidates t, t + 256, ... and sums the log-odds of its rays'
// endpoint cells (rays without a return and endpoints off the grid add nothing).  Then the best
// (highest, smallest index on ties) and the highest score at lattice Chebyshev distance >= 2 from it.
__global__ __launch_bounds__(kCsmThreads) void k_csm(const int16_t* __restrict__ belief,
                                                     const int64_t* __restrict__ cell_off,
                                                     const int32_t* __restrict__ side,
                                                     const int32_t* __restrict__ pose_q,
                                                     const int32_t* __restrict__ rho_q, int R,
                                                     const int32_t* __restrict__ a_off,
                                                     const int32_t* __restrict__ dirtab, int W, int V, int step_xy,
                                                     int step_h, int32_t* __restrict__ out) {
  __shared__ int2 s_off[kCsmMaxRayHeadings];
  __shared__ int32_t s_score[kCsmMaxCand];
  __shared__ int32_t s_red[kCsmThreads / 64][2];
  const int r = blockIdx.x;
  const int nw = 2 * W + 1, nk = 2 * V + 1, ncand = nk * nw * nw;
  const int32_t px = pose_q[3 * r], py = pose_q[3 * r + 1], ph = pose_q[3 * r + 2];
  const int32_t* rho = rho_q + (int64_t)r * R;
  int used = 0;
  for (int e = threadIdx.x; e < nk * R; e += kCsmThreads) {
    const int k = e / R, q = e - k * R;
    const int32_t rq = rho[q];
    int2 o = make_int2(INT32_MIN, 0);
    if (rq >= 0) {
      int64_t h = ((int64_t)ph + (int64_t)(k - V) * step_h + a_off[q]) % kNang;
      if (h < 0) h += kNang;
      const int32_t d = dirtab[h];
      const int32_t c = (int32_t)(int16_t)(d & 0xffff), s = d >> 16;
      o.x = (int32_t)(((int64_t)rq * c) >> 14);
      o.y = (int32_t)(((int64_t)rq * s) >> 14);
      if (k == 0) ++used;
    }
    s_off[e] = o;
  }
  __syncthreads();
  const int32_t sd = side[r];
  const int16_t* g = belief + cell_off[r];
  for (int c = threadIdx.x; c < ncand; c += kCsmThreads) {
    const int k = c / (nw * nw), rem = c - k * nw * nw, j = rem / nw, i = rem - j * nw;
    const int64_t x = (int64_t)px + (int64_t)(i - W) * step_xy, y = (int64_t)py + (int64_t)(j - W) * step_xy;
    const int2* o = s_off + k * R;
    int32_t sc = 0;
    if (sd > 0) {
      // eight rays per step with every read issued before any is used (reads from global memory);
      // a ray without a return or a cell off the grid reads cell 0 and adds nothing
      constexpr int kRays = 8;
      int q = 0;
      for (; q + kRays <= R; q += kRays) {
        int32_t t[kRays];
#pragma unroll
        for (int u = 0; u < kRays; ++u) {
          const int2 v = o[q + u];
          const int64_t cx = (x + v.x) >> 16, cy = (y + v.y) >> 16;
          const bool ok = v.x != INT32_MIN && cx >= 0 && cx < sd && cy >= 0 && cy < sd;
          const int32_t val = g[ok ? cy * sd + cx : 0];
          t[u] = ok ? val : 0;
        }
#pragma unroll
        for (int u = 0; u < kRays; ++u) sc += t[u];
      }
      for (; q < R; ++q) {
        const int2 v = o[q];
        if (v.x == INT32_MIN) continue;
        const int64_t cx = (x + v.x) >> 16, cy = (y + v.y) >> 16;
        if (cx >= 0 && cx < sd && cy >= 0 && cy < sd) sc += g[cy * sd + cx];
      }
    }
    s_score[c] = sc;
  }
  __syncthreads();
  // best: the highest score, the smallest index on ties
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t bs = INT32_MIN, bi = INT32_MAX;
  for (int c = threadIdx.x; c < ncand; c += kCsmThreads) {
    const int32_t v = s_score[c];
    if (v > bs || (v == bs && c < bi)) { bs = v; bi = c; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t os = __shfl_xor(bs, off, 64), oi = __shfl_xor(bi, off, 64);
    if (os > bs || (os == bs && oi < bi)) { bs = os; bi = oi; }
  }
  if (lane == 0) { s_red[wave][0] = bs; s_red[wave][1] = bi; }
  __syncthreads();
  bs = s_red[0][0]; bi = s_red[0][1];
  for (int w = 1; w < kCsmThreads / 64; ++w) {
    const int32_t os = s_red[w][0], oi = s_red[w][1];
    if (os > bs || (os == bs && oi < bi)) { bs = os; bi = oi; }
  }
  const int bk = bi / (nw * nw), brem = bi - bk * nw * nw, bj = brem / nw, bii = brem - bj * nw;
  // second: the highest score outside the best's 3 x 3 x 3 neighbourhood
  int32_t ss = INT32_MIN;
  for (int c = threadIdx.x; c < ncand; c += kCsmThreads) {
    const int k = c / (nw * nw), rem = c - k * nw * nw, j = rem / nw, i = rem - j * nw;
    const int dist = max(max(abs(i - bii), abs(j - bj)), abs(k - bk));
    if (dist >= 2) ss = max(ss, s_score[c]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ss = max(ss, __shfl_xor(ss, off, 64));
  // rays used: counted by the threads that staged heading candidate 0
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) used += __shfl_xor(used, off, 64);
  __syncthreads();
  if (lane == 0) { s_red[wave][0] = ss; s_red[wave][1] = used; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s2 = s_red[0][0], u = s_red[0][1];
    for (int w = 1; w < kCsmThreads / 64; ++w) { s2 = max(s2, s_red[w][0]); u += s_red[w][1]; }
    int32_t* o = out + 6 * (int64_t)r;
    o[0] = bii - W; o[1] = bj - W; o[2] = bk - V; o[3] = bs; o[4] = s2; o[5] = u;
  }
}

// The same with the robot's grid staged in LDS, for lattices of at most 9 translations per axis and
// 1024 candidates.  Only the part of the grid that some candidate's ray endpoint can reach is staged:
// the box of the rays' endpoint offsets over every heading candidate, widened by the translation
// lattice and clipped to the grid (its columns widened to multiples of 8 for 16-byte reads).  A box
// with more rows than the LDS holds is staged in bands of rows, each band scored in turn (an endpoint
// outside the band adds nothing in that pass), so any side can be staged.  A box row wider than the LDS
// is read from global memory instead.
// Thread (row, chunk) takes one (heading k, row j) line of nine x candidates over a chunk of the rays,
// so one offset read serves the whole line (the line's cells are read side by side); the chunks'
// partial sums are then added in chunk order.  Dynamic LDS: cap_cells int16 grid cells (a multiple of
// 8; the partial sums take this space after the last band), then the (2V + 1) R ray offsets.
constexpr int kCsmLdsThreads = 512;
constexpr int kCsmLdsMaxCand = 1024;
constexpr int kCsmLdsMaxLine = 9;                  // 2W + 1 <= 9
constexpr int kCsmLdsPad = 2;                      // cells between a staged row's end and the next row
constexpr int32_t kNoReturnY = -(1 << 30);        // y offset of a ray without a return: a negative row in every band

__global__ __launch_bounds__(kCsmLdsThreads) void k_csm_lds(const int16_t* __restrict__ belief,
                                                            const int64_t* __restrict__ cell_off,
                                                            const int32_t* __restrict__ side,
                                                            const int32_t* __restrict__ pose_q,
                                                            const int32_t* __restrict__ rho_q, int R,
                                                            const int32_t* __restrict__ a_off,
                                                            const int32_t* __restrict__ dirtab, int W, int V,
                                                            int step_xy, int step_h, int cap_cells,
                                                            int32_t* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  int16_t* s_grid = reinterpret_cast<int16_t*>(s_dyn);
  int32_t* s_part = reinterpret_cast<int32_t*>(s_dyn);
  int2* s_off = reinterpret_cast<int2*>(s_dyn + 2 * (int64_t)cap_cells);
  // s_red holds, until the scoring starts, the offsets' box: min x, max x, min y, max y
  __shared__ int32_t s_red[kCsmLdsThreads / 64][2];
  const int r = blockIdx.x;
  const int nw = 2 * W + 1, nk = 2 * V + 1, ncand = nk * nw * nw, nline = nk * nw;
  const int32_t px = pose_q[3 * r], py = pose_q[3 * r + 1], ph = pose_q[3 * r + 2];
  const int32_t* rho = rho_q + (int64_t)r * R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int used = 0;
  if (threadIdx.x == 0) {
    s_red[0][0] = INT32_MAX; s_red[0][1] = INT32_MIN; s_red[1][0] = INT32_MAX; s_red[1][1] = INT32_MIN;
  }
  __syncthreads();
  int32_t mnx = INT32_MAX, mxx = INT32_MIN, mny = INT32_MAX, mxy = INT32_MIN;
  for (int e = threadIdx.x; e < nk * R; e += kCsmLdsThreads) {
    const int k = e / R, q = e - k * R;
    const int32_t rq = rho[q];
    int2 o = make_int2(0, kNoReturnY);
    if (rq >= 0) {
      int64_t h = ((int64_t)ph + (int64_t)(k - V) * step_h + a_off[q]) % kNang;
      if (h < 0) h += kNang;
      const int32_t d = dirtab[h];
      const int32_t c = (int32_t)(int16_t)(d & 0xffff), s = d >> 16;
      o.x = (int32_t)(((int64_t)rq * c) >> 14);
      o.y = (int32_t)(((int64_t)rq * s) >> 14);
      mnx = min(mnx, o.x); mxx = max(mxx, o.x); mny = min(mny, o.y); mxy = max(mxy, o.y);
      if (k == 0) ++used;
    }
    s_off[e] = o;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mnx = min(mnx, __shfl_xor(mnx, off, 64)); mxx = max(mxx, __shfl_xor(mxx, off, 64));
    mny = min(mny, __shfl_xor(mny, off, 64)); mxy = max(mxy, __shfl_xor(mxy, off, 64));
  }
  if (lane == 0) {
    atomicMin(&s_red[0][0], mnx); atomicMax(&s_red[0][1], mxx);
    atomicMin(&s_red[1][0], mny); atomicMax(&s_red[1][1], mxy);
  }
  __syncthreads();
  mnx = s_red[0][0]; mxx = s_red[0][1]; mny = s_red[1][0]; mxy = s_red[1][1];
  const int32_t sd = side[r];
  const int64_t base = cell_off[r];
  // the cells any candidate's endpoint can reach, clipped to the grid (empty: every score is 0)
  const int64_t span = (int64_t)W * step_xy;
  int64_t bx0 = 0, bx1 = -1, by0 = 0, by1 = -1;
  if (mnx <= mxx && sd > 0) {
    bx0 = max<int64_t>(0, ((int64_t)px - span + mnx) >> 16);
    bx1 = min<int64_t>(sd - 1, ((int64_t)px + span + mxx) >> 16);
    by0 = max<int64_t>(0, ((int64_t)py - span + mny) >> 16);
    by1 = min<int64_t>(sd - 1, ((int64_t)py + span + mxy) >> 16);
  }
  const bool empty = bx0 > bx1 || by0 > by1;
  const bool vec = (reinterpret_cast<uintptr_t>(belief + base) & 15) == 0 && (sd & 7) == 0;
  const int64_t x0a = vec ? (bx0 & ~(int64_t)7) : bx0;
  const int64_t x1a = vec ? min<int64_t>(sd, (bx1 + 8) & ~(int64_t)7) : bx1 + 1;
  const int64_t pitch = x1a - x0a + kCsmLdsPad;
  // Staged grids are scored in 32-bit cell arithmetic, which needs the search centre within 2^28 and
  // the ray offsets within 2^29 (Q16): every coordinate relative to a band's origin then stays within
  // 2^31.  A robot beyond either bound (or with a box row wider than the LDS) is scored from global
  // memory in 64 bits.
  const bool near = mnx >= -(1 << 29) && mxx <= (1 << 29) && mny >= -(1 << 29) && mxy <= (1 << 29) &&
                    px > -(1 << 28) && px < (1 << 28) && py > -(1 << 28) && py < (1 << 28);
  const bool staged = near && pitch <= cap_cells;
  // lines x chunks of rays
  const int chunks = max(1, min(R, kCsmLdsThreads / nline));
  int32_t acc[kCsmLdsMaxLine];
#pragma unroll
  for (int i = 0; i < kCsmLdsMaxLine; ++i) acc[i] = 0;
  // consecutive threads take consecutive lines of one chunk, so a wave's lanes read the same ray at
  // the same time: neighbouring y candidates' endpoints are neighbouring rows, neighbouring headings'
  // the same or adjacent cells (fewer LDS bank conflicts than lanes on different rays)
  const int ch = threadIdx.x / nline, line = threadIdx.x - ch * nline;
  const bool active = ch < chunks;
  // One instance per memory, so that the reads of a staged grid compile to LDS reads (a pointer that
  // may point to either would make every read a flat access).  g holds rows [row0, row0 + nrows) and
  // columns [col0, col0 + ncols) of the grid, row y at (y - row0) * gp; coordinates are taken relative
  // to (col0, row0) in Q16 so that the bounds are two unsigned compares.  In 64-bit arithmetic a ray
  // without a return is skipped by its range; in 32 bits its y offset puts it above every row.
  auto score = [&](const int16_t* g, int64_t gp, int64_t row0, int64_t nrows, int64_t col0, int64_t ncols,
                   auto tag) {
    using I = decltype(tag);
    using U = std::make_unsigned_t<I>;
    constexpr bool kWide = sizeof(I) == 8;
    const int k = line / nw, j = line - k * nw;
    const int q0 = (int)((int64_t)ch * R / chunks), q1 = (int)((int64_t)(ch + 1) * R / chunks);
    const I x0 = (I)((int64_t)px - span - (col0 << 16));
    const I y = (I)((int64_t)py + (int64_t)(j - W) * step_xy - (row0 << 16));
    const U nr = (U)nrows, nc = (U)ncols;
    const I pit = (I)gp;
    const int2* o = s_off + k * R;
    // four rays per step, every read issued before any is used (the next step's offsets are read
    // before this step's cells, so one LDS round trip per step): a cell off the grid reads cell 0 of
    // the grid and adds nothing
    constexpr int kRays = 4;
    int q = q0;
    int2 nv[kRays];
    if (q + kRays <= q1) {
#pragma unroll
      for (int u = 0; u < kRays; ++u) nv[u] = o[q + u];
    }
    for (; q + kRays <= q1; q += kRays) {
      int2 cv[kRays];
#pragma unroll
      for (int u = 0; u < kRays; ++u) cv[u] = nv[u];
      if (q + 2 * kRays <= q1) {
#pragma unroll
        for (int u = 0; u < kRays; ++u) nv[u] = o[q + kRays + u];
      }
      int32_t val[kRays][kCsmLdsMaxLine];
#pragma unroll
      for (int u = 0; u < kRays; ++u) {
        const int2 v = cv[u];
        const I cy = (y + v.y) >> 16;
        bool row_ok = (U)cy < nr;
        if constexpr (kWide) row_ok = row_ok && rho[q + u] >= 0;
        const int16_t* grow = g + (row_ok ? cy : 0) * pit;
        const I ex = x0 + v.x;
#pragma unroll
        for (int i = 0; i < kCsmLdsMaxLine; ++i) {
          const I cx = (ex + (I)i * step_xy) >> 16;
          const bool ok = row_ok && i < nw && (U)cx < nc;
          const int32_t t = grow[ok ? cx : 0];
          val[u][i] = ok ? t : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < kRays; ++u)
#pragma unroll
        for (int i = 0; i < kCsmLdsMaxLine; ++i) acc[i] += val[u][i];
    }
    for (; q < q1; ++q) {
      const int2 v = o[q];
      const I cy = (y + v.y) >> 16;
      if ((U)cy >= nr) continue;
      if constexpr (kWide) {
        if (rho[q] < 0) continue;
      }
      const int16_t* grow = g + cy * pit;
      const I ex = x0 + v.x;
#pragma unroll
      for (int i = 0; i < kCsmLdsMaxLine; ++i) {
        if (i < nw) {
          const I cx = (ex + (I)i * step_xy) >> 16;
          if ((U)cx < nc) acc[i] += grow[cx];
        }
      }
    }
  };
  if (!empty && staged) {
    const int64_t band = cap_cells / pitch, ncols = x1a - x0a;
    for (int64_t r0 = by0; r0 <= by1; r0 += band) {
      const int64_t nrows = min<int64_t>(band, by1 + 1 - r0);
      if (vec) {
        // 8 cells per access: one 16-byte read, four 4-byte writes (pitch is even, so rows start on
        // 4-byte boundaries).  Thread t takes piece t mod p of rows t / p, t / p + rs, ... (p pieces a
        // row, rs = 512 / p rows a pass; a row of more than 512 pieces: pieces t, t + 512, ... of every
        // row), with kStage reads in flight before it writes any
        constexpr int kStage = 8;
        const uint4* src = reinterpret_cast<const uint4*>(belief + base + r0 * sd + x0a);
        const int per_row = (int)(ncols >> 3);
        const int64_t src_pitch = sd >> 3;
        const int rs = max(1, kCsmLdsThreads / per_row);
        const int first = per_row >= kCsmLdsThreads ? 0 : (int)threadIdx.x / per_row;
        const int piece0 = per_row >= kCsmLdsThreads ? (int)threadIdx.x : (int)threadIdx.x - first * per_row;
        if (first < rs) {
          for (int xp = piece0; xp < per_row; xp += kCsmLdsThreads) {
            for (int64_t y0 = first; y0 < nrows; y0 += (int64_t)kStage * rs) {
              const uint4* s0 = src + y0 * src_pitch + xp;
              uint32_t* d0 = reinterpret_cast<uint32_t*>(s_grid + y0 * pitch + 8 * xp);
              uint4 t[kStage];
#pragma unroll
              for (int u = 0; u < kStage; ++u)
                if (y0 + u * rs < nrows) t[u] = s0[(int64_t)u * rs * src_pitch];
#pragma unroll
              for (int u = 0; u < kStage; ++u) {
                if (y0 + u * rs < nrows) {
                  uint32_t* d = d0 + (u * rs * pitch) / 2;
                  d[0] = t[u].x; d[1] = t[u].y; d[2] = t[u].z; d[3] = t[u].w;
                }
              }
            }
          }
        }
      } else {
        const int64_t cells = nrows * ncols;
        for (int64_t e = threadIdx.x; e < cells; e += kCsmLdsThreads) {
          const int64_t yy = e / ncols, xx = e - yy * ncols;
          s_grid[yy * pitch + xx] = belief[base + (r0 + yy) * sd + x0a + xx];
        }
      }
      __syncthreads();
      if (active) score(s_grid, pitch, r0, nrows, x0a, ncols, int32_t{});
      __syncthreads();   // the band is read before the next one (or the partial sums) takes its space
    }
  } else if (!empty && active) {
    score(belief + base, sd, 0, sd, 0, sd, int64_t{});
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < kCsmLdsMaxLine; ++i)
      if (i < nw) s_part[ch * ncand + line * nw + i] = acc[i];
  }
  __syncthreads();
  int32_t sc[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int c = threadIdx.x + m * kCsmLdsThreads;
    sc[m] = INT32_MIN;
    if (c < ncand) {
      int32_t t = 0;
      for (int z = 0; z < chunks; ++z) t += s_part[z * ncand + c];
      sc[m] = t;
    }
  }
  int32_t bs = INT32_MIN, bi = INT32_MAX;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int c = threadIdx.x + m * kCsmLdsThreads;
    if (c < ncand && (sc[m] > bs || (sc[m] == bs && c < bi))) { bs = sc[m]; bi = c; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t os = __shfl_xor(bs, off, 64), oi = __shfl_xor(bi, off, 64);
    if (os > bs || (os == bs && oi < bi)) { bs = os; bi = oi; }
  }
  if (lane == 0) { s_red[wave][0] = bs; s_red[wave][1] = bi; }
  __syncthreads();
  bs = s_red[0][0]; bi = s_red[0][1];
  for (int w = 1; w < kCsmLdsThreads / 64; ++w) {
    const int32_t os = s_red[w][0], oi = s_red[w][1];
    if (os > bs || (os == bs && oi < bi)) { bs = os; bi = oi; }
  }
  const int bk = bi / (nw * nw), brem = bi - bk * nw * nw, bj = brem / nw, bii = brem - bj * nw;
  int32_t ss = INT32_MIN;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int c = threadIdx.x + m * kCsmLdsThreads;
    if (c >= ncand) continue;
    const int k = c / (nw * nw), rem = c - k * nw * nw, j = rem / nw, i = rem - j * nw;
    if (max(max(abs(i - bii), abs(j - bj)), abs(k - bk)) >= 2) ss = max(ss, sc[m]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ss = max(ss, __shfl_xor(ss, off, 64));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) used += __shfl_xor(used, off, 64);
  __syncthreads();
  if (lane == 0) { s_red[wave][0] = ss; s_red[wave][1] = used; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s2 = s_red[0][0], u = s_red[0][1];
    for (int w = 1; w < kCsmLdsThreads / 64; ++w) { s2 = max(s2, s_red[w][0]); u += s_red[w][1]; }
    int32_t* o = out + 6 * (int64_t)r;
    o[0] = bii - W; o[1] = bj - W; o[2] = bk - V; o[3] = bs; o[4] = s2; o[5] = u;
  }
}

// ------------------------------------------------------------------ scan factor

__device__ __forceinline__ double wrap_pi(double a) {
  const double two_pi = 6.283185307179586;
  return a - two_pi * rint(a / two_pi);
}

// Weight of a match: the normalised score times the margin to the second peak, both clamped to [0, 1].
using aslam::slam::match_weight;

__global__ void k_csm_factor(const int32_t* __restrict__ match, const int32_t* __restrict__ pose_q, int n,
                             int step_xy, int step_h, double cell_m, double l_max, double sig_xy, double sig_th,
                             double* __restrict__ meas, double* __restrict__ info) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t* m = match + 6 * (int64_t)r;
  const int32_t* p = pose_q + 3 * (int64_t)r;
  const double x = (double)((int64_t)p[0] + (int64_t)m[0] * step_xy) / 65536.0 * cell_m;
  const double y = (double)((int64_t)p[1] + (int64_t)m[1] * step_xy) / 65536.0 * cell_m;
  int64_t h = ((int64_t)p[2] + (int64_t)m[2] * step_h) % kNang;
  if (h < 0) h += kNang;
  const double th = wrap_pi(2.0 * 3.141592653589793 * (double)h / (double)kNang);
  const double w = match_weight(m, l_max);
  meas[3 * (int64_t)r] = x; meas[3 * (int64_t)r + 1] = y; meas[3 * (int64_t)r + 2] = th;
  info[3 * (int64_t)r] = w / (sig_xy * sig_xy);
  info[3 * (int64_t)r + 1] = w / (sig_xy * sig_xy);
  info[3 * (int64_t)r + 2] = w / (sig_th * sig_th);
}

// ------------------------------------------------------------------ weighted map integration

constexpr int kIntThreads = 512;
constexpr int kIntLdsMinWords = 4096;    // LDS bitmaps of at least 16 KB: a band holds a row of any side <= 65536
constexpr int kIntLdsMaxWords = 16384;   // and at most 64 KB
constexpr int kIntMaxSide = 32768;   // bit indices (row offset x row bits + column) stay below 2^31
constexpr int kIntInFlight = 4;          // octets (8 cells, 16 bytes) each thread keeps in flight in the apply pass
constexpr int kIntSortMax = 2048;        // rays are ordered by walk length when R <= this
constexpr int kIntBins = 64;             // length classes of 8 steps

// Saturating add of the increment of each coded cell of an octet (bit j of `any`: cell j coded, of `hit`:
// a HIT) to the 8 int16 values packed in v.
__device__ __forceinline__ int4 apply_octet(int4 v, uint32_t any, uint32_t hit, int32_t d_hit, int32_t d_miss,
                                            int32_t lc) {
  int32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int32_t lo = (int16_t)(w[j] & 0xffff), hi = w[j] >> 16;
    if ((any >> (2 * j)) & 1u) lo = min(max(lo + (((hit >> (2 * j)) & 1u) ? d_hit : d_miss), -lc), lc);
    if ((any >> (2 * j + 1)) & 1u) hi = min(max(hi + (((hit >> (2 * j + 1)) & 1u) ? d_hit : d_miss), -lc), lc);
    w[j] = (lo & 0xffff) | (hi << 16);
  }
  return make_int4(w[0], w[1], w[2], w[3]);
}

// One workgroup per robot.  The aligned pose is the predicted pose moved by the match's lattice
// offsets; the increments are round(w_q l / 256) with w_q = rint(256 w).  Rows are processed in bands
// whose two bitmaps fit the launch's LDS (sized for the largest side, up to 64 KB: a 512 x 512 grid is
// one band).  Per band: clear; one lane per ray walks it from the aligned origin with the exact
// traversal and sets MISS bits for the band's cells and the HIT bit of the end cell of a ray with a
// return that ended at its range; then the apply pass: one saturating add per coded cell (HIT beats
// MISS), an octet of 8 cells owned by one thread -- the result does not depend on ray or lane order,
// so lanes take the rays longest first (a counting sort on the walk's length bound), which keeps the
// rays of a wave alike in length and the workgroups that share a compute unit from issuing idle steps.
//
// The walk: with (a, b) the Q14 direction and the origin's fractional position, the k-th x crossing lies
// at axis distance ex0 + 65536 k and is within the range iff (ex0 + 65536 k) 2^14 <= rho |a|, so the
// numbers of x and y crossings allowed by the range and by the grid's edge are known up front; crossings
// are taken in order of distance by the sign of D = ex |b| - ey |a| (x first when D <= 0), a 32-bit
// value that stays in (-65536 |a|, 65536 |b|].  The walk stops at the first crossing that is not
// allowed; it ended at its range unless that crossing was barred by the grid's edge alone.
__global__ __launch_bounds__(kIntThreads) void k_csm_integrate(
    int16_t* __restrict__ belief, const int64_t* __restrict__ cell_off, const int32_t* __restrict__ side,
    const int32_t* __restrict__ pose_q, const int32_t* __restrict__ rho_q, int R, const int32_t* __restrict__ a_off,
    const int32_t* __restrict__ dirtab, int32_t rmax_q, const int32_t* __restrict__ match, int step_xy, int step_h,
    double l_max, int l_hit, int l_miss, int l_clamp, int32_t* __restrict__ coded, int lds_words,
    const int32_t* __restrict__ wq_in) {
  extern __shared__ __align__(16) uint32_t bits[];
  __shared__ int32_t s_cnt[kIntThreads / 64];
  __shared__ uint16_t s_perm[kIntSortMax];
  __shared__ int32_t s_hist[kIntBins];
  const int r = blockIdx.x;
  const int64_t s = side[r];
  const int64_t base = cell_off[r];
  int64_t ax = pose_q[3 * (int64_t)r], ay = pose_q[3 * (int64_t)r + 1], ah = pose_q[3 * (int64_t)r + 2];
  int32_t wq = 256;
  if (wq_in) {
    wq = wq_in[r];
  } else if (match) {
    const int32_t* m = match + 6 * (int64_t)r;
    ax += (int64_t)m[0] * step_xy;
    ay += (int64_t)m[1] * step_xy;
    ah += (int64_t)m[2] * step_h;
    wq = (int32_t)rint(256.0 * match_weight(m, l_max));
  }
  ah %= kNang;
  if (ah < 0) ah += kNang;
  const int32_t d_hit = (wq * l_hit + 128) >> 8, d_miss = (wq * l_miss + 128) >> 8;
  const int64_t ocx = ax >> 16, ocy = ay >> 16;
  if (s <= 0 || s > kIntMaxSide || ocx < 0 || ocx >= s || ocy < 0 || ocy >= s) {   // uniform over the workgroup
    if (coded && threadIdx.x == 0) coded[r] = s > kIntMaxSide ? -1 : 0;
    return;
  }
  const int32_t si = (int32_t)s, cx0 = (int32_t)ocx, cy0 = (int32_t)ocy;
  const int32_t fx = (int32_t)(ax - (ocx << 16)), fy = (int32_t)(ay - (ocy << 16));
  const int32_t nw = (si + 31) >> 5;
  const int32_t band = min(si, lds_words / (2 * nw));
  uint32_t* miss = bits;
  uint32_t* hitm = bits + band * nw;
  // 16-byte accesses when every row starts on an 8-cell boundary
  const bool vec = ((base | s) & 7) == 0;
  const bool sorted = R <= kIntSortMax;
  if (sorted) {
    // length class of a ray: its Manhattan length in cells (an upper bound of its steps) / 8
    auto ray_class = [&](int k) {
      const int32_t rho = rho_q[(int64_t)r * R + k];
      const int64_t lim = rho >= 0 ? (int64_t)rho : (int64_t)rmax_q;
      int64_t di = (ah + (int64_t)a_off[k]) % kNang;
      if (di < 0) di += kNang;
      const int32_t dv = dirtab[di];
      const int64_t ab = abs((int32_t)(int16_t)(dv & 0xffff)) + abs(dv >> 16);
      return (int32_t)min<int64_t>(kIntBins - 1, ((lim >> 16) * ab) >> 17);
    };
    constexpr int kPer = kIntSortMax / kIntThreads;
    int32_t cls[kPer];
    for (int i = threadIdx.x; i < kIntBins; i += kIntThreads) s_hist[i] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = threadIdx.x + u * kIntThreads;
      cls[u] = k < R ? ray_class(k) : 0;
      if (k < R) atomicAdd(&s_hist[cls[u]], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {   // start of each class, longest class first
      int32_t acc = 0;
      for (int c = kIntBins - 1; c >= 0; --c) {
        const int32_t h = s_hist[c];
        s_hist[c] = acc;
        acc += h;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = threadIdx.x + u * kIntThreads;
      if (k < R) s_perm[atomicAdd(&s_hist[cls[u]], 1)] = (uint16_t)k;
    }
    __syncthreads();
  }
  int32_t cnt = 0;
  for (int32_t by0 = 0; by0 < si; by0 += band) {
    const int32_t rows = min(band, si - by0);
    for (int32_t w = threadIdx.x; w < 2 * band * nw; w += kIntThreads) bits[w] = 0u;
    __syncthreads();
    // Each lane's walk length and end cell are known before it starts: the walk stops at the first
    // barred crossing in distance order -- x crossing #nx at axis distance ex0 + 65536 nx or y crossing
    // #ny, whichever comes first (x on a tie) -- after every crossing that precedes it.  The loop then
    // only selects the next crossing by the sign of D and marks the cell; trip counts are uniform over
    // the wave (lanes past their own length mark nothing), and while the band holds the whole grid and
    // every lane is within its length the marks need no test.
    const int32_t rowbits = nw << 5;
    const uint32_t band_bits = (uint32_t)(rows * rowbits);
    const bool one_band = band >= si;
    for (int j0 = 0; j0 < R; j0 += kIntThreads) {
      const int j = j0 + (int)threadIdx.x;
      const bool valid = j < R;
      int32_t rho = -1, dv = 0;
      if (valid) {
        const int k = sorted ? (int)s_perm[j] : j;
        rho = rho_q[(int64_t)r * R + k];
        int64_t di = (ah + (int64_t)a_off[k]) % kNang;
        if (di < 0) di += kNang;
        dv = dirtab[di];
      }
      const int64_t lim = rho >= 0 ? (int64_t)rho : (int64_t)rmax_q;
      const int32_t a = (int16_t)(dv & 0xffff), b = dv >> 16;
      const int32_t aa = abs(a), bb = abs(b);
      const int32_t ex0 = a > 0 ? 65536 - fx : fx, ey0 = b > 0 ? 65536 - fy : fy;
      const int64_t emx = (lim * aa) >> 14, emy = (lim * bb) >> 14;
      const int64_t nxl = (aa == 0 || emx < ex0) ? 0 : ((emx - ex0) >> 16) + 1;
      const int64_t nyl = (bb == 0 || emy < ey0) ? 0 : ((emy - ey0) >> 16) + 1;
      const int32_t nxg = a > 0 ? si - 1 - cx0 : cx0, nyg = b > 0 ? si - 1 - cy0 : cy0;
      const int32_t nx = (int32_t)min((int64_t)nxg, nxl), ny = (int32_t)min((int64_t)nyg, nyl);
      const bool gx = nxg < nxl, gy = nyg < nyl;
      int32_t kx, ky;     // x and y steps of the walk
      bool at_limit;      // the barred crossing is barred by the range (else by the grid's edge only)
      if (aa == 0) {
        kx = 0; ky = ny; at_limit = !gy;
      } else if (bb == 0) {
        kx = nx; ky = 0; at_limit = !gx;
      } else {
        const int64_t tx = ((int64_t)ex0 + ((int64_t)nx << 16)) * bb;   // barred x crossing (scaled)
        const int64_t ty = ((int64_t)ey0 + ((int64_t)ny << 16)) * aa;   // barred y crossing (scaled)
        if (tx <= ty) {   // stops at the x crossing: the y crossings strictly before it
          const int64_t X = tx - (int64_t)ey0 * aa, den = (int64_t)aa << 16;
          kx = nx;
          ky = X <= 0 ? 0 : (int32_t)min<int64_t>(ny, (X + den - 1) / den);
          at_limit = !gx;
        } else {          // stops at the y crossing: the x crossings at or before it
          const int64_t Y = ty - (int64_t)ex0 * bb, den = (int64_t)bb << 16;
          ky = ny;
          kx = Y < 0 ? 0 : (int32_t)min<int64_t>(nx, Y / den + 1);
          at_limit = !gy;
        }
      }
      const int32_t n = valid ? kx + ky : 0;
      const int32_t sxw = a > 0 ? 1 : -1, syw = b > 0 ? rowbits : -rowbits;
      const int32_t w0 = (cy0 - by0) * rowbits + cx0;   // bit of the origin cell (may lie outside the band)
      int32_t D = aa == 0 ? 1 : (bb == 0 ? -1 : ex0 * bb - ey0 * aa);
      const int32_t dX = bb == 0 ? 0 : bb << 16, dY = aa == 0 ? 0 : aa << 16;
      if (valid && (uint32_t)w0 < band_bits) atomicOr(&miss[w0 >> 5], 1u << (w0 & 31));
      int32_t nmax = n, nmin = n;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        nmax = max(nmax, __shfl_xor(nmax, o, 64));
        nmin = min(nmin, __shfl_xor(nmin, o, 64));
      }
      if (!one_band) nmin = 0;
      int32_t wi = w0, i = 0;
      for (; i < nmin; ++i) {
        const bool stepx = D <= 0;
        wi += stepx ? sxw : syw;
        D += stepx ? dX : -dY;
        atomicOr(&miss[wi >> 5], 1u << (wi & 31));
      }
      for (; i < nmax; ++i) {
        const bool stepx = D <= 0;
        wi += stepx ? sxw : syw;
        D += stepx ? dX : -dY;
        if (i < n && (uint32_t)wi < band_bits) atomicOr(&miss[wi >> 5], 1u << (wi & 31));
      }
      const int32_t we = w0 + kx * sxw + ky * syw;   // the end cell
      if (valid && rho >= 0 && at_limit && (uint32_t)we < band_bits) atomicOr(&hitm[we >> 5], 1u << (we & 31));
    }
    __syncthreads();
    // apply: octet o covers cells 8 (o mod 4nw) .. + 7 of band row o / 4nw
    const int32_t opr = 4 * nw, total = rows * opr;
    int16_t* band_base = belief + base + (int64_t)by0 * s;
    for (int32_t o0 = threadIdx.x; o0 < total; o0 += kIntInFlight * kIntThreads) {
      uint32_t any[kIntInFlight], hit[kIntInFlight];
      int64_t off[kIntInFlight];
#pragma unroll
      for (int u = 0; u < kIntInFlight; ++u) {
        const int32_t o = o0 + u * kIntThreads;
        any[u] = 0u;
        hit[u] = 0u;
        off[u] = 0;
        if (o < total) {
          const int32_t row = o / opr, oc = o - row * opr, sh = (oc & 3) * 8;
          const uint32_t wm = miss[row * nw + (oc >> 2)], wh = hitm[row * nw + (oc >> 2)];
          hit[u] = (wh >> sh) & 0xffu;
          any[u] = ((wm >> sh) & 0xffu) | hit[u];
          off[u] = (int64_t)row * s + 8 * oc;
        }
        cnt += __builtin_popcount(any[u]);
      }
      if (vec) {
        int4 v[kIntInFlight];
#pragma unroll
        for (int u = 0; u < kIntInFlight; ++u)
          if (any[u]) v[u] = *reinterpret_cast<const int4*>(band_base + off[u]);
#pragma unroll
        for (int u = 0; u < kIntInFlight; ++u)
          if (any[u])
            *reinterpret_cast<int4*>(band_base + off[u]) = apply_octet(v[u], any[u], hit[u], d_hit, d_miss, l_clamp);
      } else {
#pragma unroll
        for (int u = 0; u < kIntInFlight; ++u) {
          int16_t* c = band_base + off[u];
          int16_t v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if ((any[u] >> j) & 1u) v[j] = c[j];
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if ((any[u] >> j) & 1u)
              c[j] = (int16_t)min(max((int32_t)v[j] + (((hit[u] >> j) & 1u) ? d_hit : d_miss), -l_clamp), l_clamp);
        }
      }
    }
    __syncthreads();
  }
  if (coded) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t t = 0;
      for (int i = 0; i < kIntThreads / 64; ++i) t += s_cnt[i];
      coded[r] = t;
    }
  }
}

// ------------------------------------------------------------------ heading table

// Direction of heading step k, cos and sin of 2 pi k / 46080 rounded to Q14, packed (cos low, sin high).
void build_dirtab(std::vector<int32_t>& t) {
  t.resize(kNang);
  for (int k = 0; k < kNang; ++k) {
    const double ang = (2.0 * M_PI * (double)k) / (double)kNang;
    const int32_t c = (int32_t)std::llround(std::cos(ang) * (double)kDirOne);
    const int32_t sn = (int32_t)std::llround(std::sin(ang) * (double)kDirOne);
    t[k] = (int32_t)(((uint32_t)c & 0xffffu) | ((uint32_t)sn << 16));
  }
}

int check_csm_config(const aslam_csm_config* c, int32_t R) {
  if (!c) return sfail(ASL_EINVAL, "csm config is NULL");
  if (c->W < 0 || c->W > kCsmMaxHalf || c->V < 0 || c->V > kCsmMaxHalf)
    return sfail(ASL_EINVAL, "csm half-widths W and V must be in [0, 8]");
  if (c->step_xy_q < 1 || c->step_xy_q > (1 << 20) || c->step_h < 0 || c->step_h > kNang)
    return sfail(ASL_EINVAL, "csm steps out of range (step_xy_q in [1, 2^20], step_h in [0, 46080])");
  if (R < 1 || (int64_t)(2 * c->V + 1) * R > kCsmMaxRayHeadings)
    return sfail(ASL_EINVAL, "csm needs R >= 1 and (2V + 1) * R <= 8192");
  return ASL_OK;
}

}  // namespace

// The backbone's handle: the direction table on the device it was created on.
struct aslam_slam {
  int device = -1;
  int32_t* tab = nullptr;
};

namespace {

// The handle's table, checked to belong to the current device (a host query: no allocation, no sync).
int slam_table(const aslam_slam* h, const int32_t** tab) {
  if (!h || !h->tab) return sfail(ASL_EINVAL, "slam handle is NULL");
  int dev = 0;
  SCHK(hipGetDevice(&dev));
  if (dev != h->device) return sfail(ASL_ESTATE, "slam handle was created on another device");
  *tab = h->tab;
  return ASL_OK;
}

}  // namespace

namespace aslam {
namespace slam {

hipError_t launch_csm_match(const int32_t* tab, const int16_t* belief_dev, const int64_t* cell_off_dev,
                            const int32_t* side_dev, int32_t max_side, int32_t n, const int32_t* pose_q_dev,
                            const int32_t* rho_q_dev, int32_t R, const int32_t* a_off_dev, int W, int V,
                            int step_xy_q, int step_h, int32_t* out_dev, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int ncand = (2 * V + 1) * (2 * W + 1) * (2 * W + 1);
  if (ncand <= kCsmLdsMaxCand && 2 * W + 1 <= kCsmLdsMaxLine) {
    // LDS: the ray offsets and room for a whole grid of the largest side (rows padded) within the
    // CU's 160 KB, so one robot per CU; a box that does not fit is staged in bands.  (Smaller shares,
    // two or three robots per CU, were slower: at 360 rays the extra bands repeat the scoring, which
    // dominates.)  The grid space holds at least the chunks' partial sums.
    const int chunks = std::max(1, std::min((int)R, kCsmLdsThreads / ((2 * V + 1) * (2 * W + 1))));
    const int64_t off_bytes = (int64_t)(2 * V + 1) * R * (int64_t)sizeof(int2);
    const int64_t part_cells = (2 * (int64_t)ncand * chunks + 7) & ~(int64_t)7;
    const int64_t whole = (((int64_t)max_side + kCsmLdsPad) * max_side + 7) & ~(int64_t)7;
    const int64_t room = ((kCsmLdsBudget - off_bytes) / 2) & ~(int64_t)7;
    const int64_t cap_cells = std::max(part_cells, std::min(whole, room));
    const int bytes = (int)(2 * cap_cells + off_bytes);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_csm_lds),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    k_csm_lds<<<n, kCsmLdsThreads, bytes, stream>>>(belief_dev, cell_off_dev, side_dev, pose_q_dev, rho_q_dev, R,
                                                    a_off_dev, tab, W, V, step_xy_q, step_h, (int)cap_cells,
                                                    out_dev);
  } else {
    k_csm<<<n, kCsmThreads, 0, stream>>>(belief_dev, cell_off_dev, side_dev, pose_q_dev, rho_q_dev, R, a_off_dev, tab,
                                         W, V, step_xy_q, step_h, out_dev);
  }
  return hipGetLastError();
}

hipError_t launch_csm_integrate(const int32_t* tab, int16_t* belief_dev, const int64_t* cell_off_dev,
                                const int32_t* side_dev, int32_t n, const int32_t* pose_q_dev,
                                const int32_t* rho_q_dev, int32_t R, const int32_t* a_off_dev, int32_t max_side,
                                int32_t rmax_q, const int32_t* match_dev, int step_xy, int step_h, double l_max,
                                int32_t l_hit, int32_t l_miss, int32_t l_clamp, int32_t* coded_dev,
                                const int32_t* wq_dev, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  // bitmaps of one band holding the largest grid whole, within [16 KB, 64 KB]
  const int64_t nw_max = ((int64_t)std::min(max_side, kIntMaxSide) + 31) >> 5;
  const int words = (int)std::min<int64_t>(kIntLdsMaxWords, std::max<int64_t>(kIntLdsMinWords, 2 * nw_max * max_side));
  const int bytes = (int)sizeof(uint32_t) * words;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_csm_integrate),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  k_csm_integrate<<<n, kIntThreads, bytes, stream>>>(belief_dev, cell_off_dev, side_dev, pose_q_dev, rho_q_dev, R,
                                                     a_off_dev, tab, rmax_q, match_dev, step_xy, step_h,
                                                     match_dev ? l_max : 1.0, l_hit, l_miss, l_clamp, coded_dev,
                                                     words, wq_dev);
  return hipGetLastError();
}

}  // namespace slam
}  // namespace aslam

extern "C" {

int aslam_slam_create(aslam_slam** out) {
  if (!out) return sfail(ASL_EINVAL, "out is NULL");
  *out = nullptr;
  aslam_slam* h = new (std::nothrow) aslam_slam();
  if (!h) return sfail(ASL_ENOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&h->device);
  std::vector<int32_t> t;
  build_dirtab(t);
  if (e == hipSuccess) e = hipMalloc(&h->tab, sizeof(int32_t) * kNang);
  if (e == hipSuccess) e = hipMemcpy(h->tab, t.data(), sizeof(int32_t) * kNang, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (h->tab) (void)hipFree(h->tab);
    delete h;
    return sfail(e == hipErrorOutOfMemory ? ASL_ENOMEM : ASL_EHIP, hipGetErrorString(e));
  }
  *out = h;
  return ASL_OK;
}

int aslam_slam_destroy(aslam_slam* h) {
  if (!h) return sfail(ASL_EINVAL, "slam handle is NULL");
  if (h->tab) (void)hipFree(h->tab);
  delete h;
  return ASL_OK;
}

int aslam_csm_match(const aslam_slam* slam, const int16_t* belief_dev, const int64_t* cell_off_dev,
                    const int32_t* side_dev, int32_t max_side, int32_t n, const int32_t* pose_q_dev, const int32_t* rho_q_dev, int32_t R,
                    const int32_t* a_off_dev, const aslam_csm_config* cfg, int32_t* out_dev, aslam_stream_t stream) {
  int rc = check_csm_config(cfg, R);
  if (rc) return rc;
  if (n < 0) return sfail(ASL_EINVAL, "n must be >= 0");
  if (max_side < 0) return sfail(ASL_EINVAL, "max_side must be >= 0");
  if (n == 0) return ASL_OK;
  if (!belief_dev || !cell_off_dev || !side_dev || !pose_q_dev || !rho_q_dev || !a_off_dev || !out_dev)
    return sfail(ASL_EINVAL, "null argument to csm_match");
  const int32_t* tab = nullptr;
  rc = slam_table(slam, &tab);
  if (rc) return rc;
  SCHK(aslam::slam::launch_csm_match(tab, belief_dev, cell_off_dev, side_dev, max_side, n, pose_q_dev, rho_q_dev, R,
                                     a_off_dev, cfg->W, cfg->V, cfg->step_xy_q, cfg->step_h, out_dev,
                                     (hipStream_t)stream));
  return ASL_OK;
}

int aslam_csm_factor(const int32_t* match_dev, const int32_t* pose_q_dev, int32_t n, const aslam_csm_config* cfg,
                     double cell_m, double l_max, double sigma_xy, double sigma_th, double* meas_dev,
                     double* info_dev, aslam_stream_t stream) {
  if (!cfg) return sfail(ASL_EINVAL, "csm config is NULL");
  if (n < 0) return sfail(ASL_EINVAL, "n must be >= 0");
  if (!(cell_m > 0.0) || !(l_max > 0.0) || !(sigma_xy > 0.0) || !(sigma_th > 0.0))
    return sfail(ASL_EINVAL, "cell_m, l_max and the sigmas must be positive");
  if (n == 0) return ASL_OK;
  if (!match_dev || !pose_q_dev || !meas_dev || !info_dev) return sfail(ASL_EINVAL, "null argument to csm_factor");
  k_csm_factor<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(match_dev, pose_q_dev, n, cfg->step_xy_q,
                                                                  cfg->step_h, cell_m, l_max, sigma_xy, sigma_th,
                                                                  meas_dev, info_dev);
  SCHK(hipGetLastError());
  return ASL_OK;
}

int aslam_csm_integrate(const aslam_slam* slam, int16_t* belief_dev, const int64_t* cell_off_dev,
                        const int32_t* side_dev, int32_t n,
                        const int32_t* pose_q_dev, const int32_t* rho_q_dev, int32_t R, const int32_t* a_off_dev,
                        int32_t max_side, int32_t rmax_q, const int32_t* match_dev, const aslam_csm_config* cfg,
                        double l_max, int32_t l_hit, int32_t l_miss, int32_t l_clamp, int32_t* coded_dev,
                        aslam_stream_t stream) {
  if (n < 0) return sfail(ASL_EINVAL, "n must be >= 0");
  if (max_side < 0) return sfail(ASL_EINVAL, "max_side must be >= 0");
  if (R < 1 || R > (1 << 16)) return sfail(ASL_EINVAL, "R must be in [1, 65536]");
  if (rmax_q < 0) return sfail(ASL_EINVAL, "rmax_q must be >= 0");
  if (l_clamp < 1 || l_clamp > 32767 || l_hit < -32767 || l_hit > 32767 || l_miss < -32767 || l_miss > 32767)
    return sfail(ASL_EINVAL, "l_clamp must be in [1, 32767] and the increments in [-32767, 32767]");
  int step_xy = 0, step_h = 0;
  if (match_dev) {
    if (!cfg) return sfail(ASL_EINVAL, "csm config is NULL");
    if (cfg->step_xy_q < 1 || cfg->step_xy_q > (1 << 20) || cfg->step_h < 0 || cfg->step_h > kNang)
      return sfail(ASL_EINVAL, "csm steps out of range (step_xy_q in [1, 2^20], step_h in [0, 46080])");
    if (!(l_max > 0.0)) return sfail(ASL_EINVAL, "l_max must be positive");
    step_xy = cfg->step_xy_q;
    step_h = cfg->step_h;
  }
  if (n == 0) return ASL_OK;
  if (!belief_dev || !cell_off_dev || !side_dev || !pose_q_dev || !rho_q_dev || !a_off_dev)
    return sfail(ASL_EINVAL, "null argument to csm_integrate");
  const int32_t* tab = nullptr;
  const int rc = slam_table(slam, &tab);
  if (rc) return rc;
  SCHK(aslam::slam::launch_csm_integrate(tab, belief_dev, cell_off_dev, side_dev, n, pose_q_dev, rho_q_dev, R,
                                         a_off_dev, max_side, rmax_q, match_dev, step_xy, step_h, l_max, l_hit, l_miss,
                                         l_clamp, coded_dev, nullptr, (hipStream_t)stream));
  return ASL_OK;
}

int aslam_fixedlag_solve(int32_t n, int32_t L, const double* x0_dev, const double* prior_dev, const double* odo_dev,
                         const double* scan_dev, int32_t iters, double* x_dev, double* cov_dev,
                         aslam_stream_t stream) {
  if (n < 0 || L < 1 || L > aslam::slam::kMaxWindow || iters < 0 || iters > 100)
    return sfail(ASL_EINVAL, "need n >= 0, 1 <= L <= 64, 0 <= iters <= 100");
  if (n == 0) return ASL_OK;
  if (!x0_dev || !prior_dev || (L > 1 && !odo_dev) || !scan_dev || !x_dev || !cov_dev)
    return sfail(ASL_EINVAL, "null argument to fixedlag_solve");
  SCHK(aslam::slam::launch_fixedlag(n, L, nullptr, x0_dev, prior_dev, odo_dev, scan_dev, iters, x_dev, cov_dev,
                                    (hipStream_t)stream));
  return ASL_OK;
}

}  // extern "C"
