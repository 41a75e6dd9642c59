// fixedlag.hip -- the fixed-lag pose graph of the SLAM backbone (arXiv 2603.25834, Sec. III-D) on gfx950:
// a few Gauss-Newton steps over a window of L poses (a prior on the oldest, odometry factors between
// neighbours, unary scan factors) in FP64, solved by block elimination of the block-tridiagonal normal
// equations, and the newest pose's marginal covariance (the inverse of the last Schur complement).
//
// One wave runs each window's elimination chain alone on its SIMD, so the FP64 dependency latency
// between consecutive instructions, not the issue rate, sets its time (about 12 cycles per VALU
// instruction by the SQ counters).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "slam_internal.h"

namespace {

__device__ __forceinline__ double wrap_pi(double a) {
  const double two_pi = 6.283185307179586;
  return a - two_pi * rint(a / two_pi);
}

// ------------------------------------------------------------------ fixed-lag Gauss-Newton
//
// FP64 throughout, with multiply-adds fused (the solve is checked against the oracle to 1e-9, not bit
// for bit): the elimination chain of a window is serial over its poses, so its dependency depth per
// pose is the kernel's time; nine lanes share each pose's block arithmetic.
#pragma clang fp contract(fast)

struct M3 {
  double a[3][3];
};

// Inverse of a symmetric 3 x 3 matrix from its upper triangle (the result is symmetric): six cofactors,
// and the determinant's reciprocal by the hardware estimate refined with two Newton steps (about one
// ulp, against the dozen dependent operations of an IEEE division).
__device__ __forceinline__ M3 sym_inv3(const M3& m) {
  const double (*a)[3] = m.a;
  const double c00 = a[1][1] * a[2][2] - a[1][2] * a[1][2];
  const double c01 = a[0][2] * a[1][2] - a[0][1] * a[2][2];
  const double c02 = a[0][1] * a[1][2] - a[0][2] * a[1][1];
  const double c11 = a[0][0] * a[2][2] - a[0][2] * a[0][2];
  const double c12 = a[0][2] * a[0][1] - a[0][0] * a[1][2];
  const double c22 = a[0][0] * a[1][1] - a[0][1] * a[0][1];
  const double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
  double id = __builtin_amdgcn_rcp(det);
  id = id + id * (1.0 - det * id);
  id = id + id * (1.0 - det * id);
  M3 r;
  r.a[0][0] = c00 * id;
  r.a[0][1] = r.a[1][0] = c01 * id;
  r.a[0][2] = r.a[2][0] = c02 * id;
  r.a[1][1] = c11 * id;
  r.a[1][2] = r.a[2][1] = c12 * id;
  r.a[2][2] = c22 * id;
  return r;
}

// Odometry factor between poses xi and xj: residual, and its Jacobians Ji (wrt xi) and Jj (wrt xj).
__device__ __forceinline__ void odo_factor(const double* xi, const double* xj, const double* u, double r[3],
                                           double Ji[3][3], double Jj[3][3]) {
  double s, c;
  sincos(xi[2], &s, &c);
  const double dx = xj[0] - xi[0], dy = xj[1] - xi[1];
  r[0] = (c * dx + s * dy) - u[0];
  r[1] = (-s * dx + c * dy) - u[1];
  r[2] = wrap_pi(xj[2] - xi[2] - u[2]);
  Ji[0][0] = -c; Ji[0][1] = -s; Ji[0][2] = -s * dx + c * dy;
  Ji[1][0] = s;  Ji[1][1] = -c; Ji[1][2] = -c * dx - s * dy;
  Ji[2][0] = 0;  Ji[2][1] = 0;  Ji[2][2] = -1.0;
  Jj[0][0] = c;  Jj[0][1] = s;  Jj[0][2] = 0;
  Jj[1][0] = -s; Jj[1][1] = c;  Jj[1][2] = 0;
  Jj[2][0] = 0;  Jj[2][1] = 0;  Jj[2][2] = 1.0;
}

// acc += P^T diag(w) Q (3 x 3)
__device__ __forceinline__ void add_jtwj(double acc[3][3], const double P[3][3], const double* w, const double Q[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) t += P[k][a] * w[k] * Q[k][b];
      acc[a][b] += t;
    }
}

__device__ __forceinline__ void add_jtwr(double* acc, const double P[3][3], const double* w, const double* rr) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) t += P[k][a] * w[k] * rr[k];
    acc[a] += t;
  }
}

// One wavefront per window.  Each Gauss-Newton step linearises every pose in parallel, lane i < L
// forming the diagonal block A_i, the coupling B_i = H[i][i+1] and the gradient g_i from the factors
// that touch pose i (the prior on pose 0, its scan factor, the odometry factors to i-1 and to i+1,
// each with analytic Jacobians).  Lane 0 then eliminates the block-tridiagonal system pose by pose,
// D_i = A_i - B_{i-1}^T D_{i-1}^{-1} B_{i-1}, y_i = -g_i - B_{i-1}^T D_{i-1}^{-1} y_{i-1}, keeping
// D_i^{-1}, C_i = D_i^{-1} B_i and y_i, and back-substitutes delta_{L-1} = D_{L-1}^{-1} y_{L-1},
// delta_i = D_i^{-1} y_i - C_i delta_{i+1}.  After K steps one more linearisation and elimination at
// the result gives Sigma = D_{L-1}^{-1}, the last diagonal block of the inverse Hessian.  Everything
// lives in LDS: 45 L doubles per window.
constexpr int kLagThreads = 64;

__device__ __forceinline__ void linearise_pose(const double* x, int L, int i, const double* prior, const double* odo,
                                               const double* scan, double* A_out, double* B_out, double* g_out) {
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, B[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double g[3] = {0, 0, 0};
  const double* xi = x + 3 * i;
  if (i == 0) {
    const double r[3] = {xi[0] - prior[0], xi[1] - prior[1], wrap_pi(xi[2] - prior[2])};
#pragma unroll
    for (int a = 0; a < 3; ++a) { A[a][a] += prior[3 + a]; g[a] += prior[3 + a] * r[a]; }
  }
  const double* sc = scan + 6 * i;
  if (sc[3] != 0.0 || sc[4] != 0.0 || sc[5] != 0.0) {
    const double r[3] = {xi[0] - sc[0], xi[1] - sc[1], wrap_pi(xi[2] - sc[2])};
#pragma unroll
    for (int a = 0; a < 3; ++a) { A[a][a] += sc[3 + a]; g[a] += sc[3 + a] * r[a]; }
  }
  if (i > 0) {   // odometry factor (i-1, i): pose i's share
    const double* o = odo + 6 * (i - 1);
    double r[3], Ji[3][3], Jj[3][3];
    odo_factor(x + 3 * (i - 1), xi, o, r, Ji, Jj);
    add_jtwj(A, Jj, o + 3, Jj);
    add_jtwr(g, Jj, o + 3, r);
  }
  if (i + 1 < L) {   // odometry factor (i, i+1): pose i's share and the coupling
    const double* o = odo + 6 * i;
    double r[3], Ji[3][3], Jj[3][3];
    odo_factor(xi, x + 3 * (i + 1), o, r, Ji, Jj);
    add_jtwj(A, Ji, o + 3, Ji);
    add_jtwj(B, Ji, o + 3, Jj);
    add_jtwr(g, Ji, o + 3, r);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g_out[a] = g[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) { A_out[3 * a + b] = A[a][b]; B_out[3 * a + b] = B[a][b]; }
  }
}

// The elimination sweep spread over nine lanes, lane (a, b) owning entry (a, b) of the 3x3 blocks (every
// lane of the wave runs it; lane l works on entry l mod 9 and only lanes < 9 store): each lane forms its
// entry of the Schur complement D_i, the six upper entries are gathered to every lane by shuffles, every
// lane inverts D_i (so D_i^{-1} needs no exchange), forms its entry of C_i = D_i^{-1} B_i, and C_i and
// y_i are gathered for the next pose.  A lane's dependent chain per pose is a few operations and two
// shuffle rounds instead of the whole block arithmetic of one lane (about 4x shorter).
__device__ __forceinline__ double pick3(double x0, double x1, double x2, int k) {
  return k == 0 ? x0 : (k == 1 ? x1 : x2);
}

__device__ __forceinline__ void eliminate_sweep9(int L, int lane, const double* sA, const double* sB,
                                                 const double* sg, double* sDi, double* sC, double* sy, M3& last) {
  // a lane's operands are read from LDS at its own addresses (the previous pose's B, C and y there are
  // the ones the lanes stored one pose earlier: a wave's LDS accesses complete in order), so no register
  // array is indexed by the lane
  const int l = lane % 9, a = l / 3, b = l - 3 * a;
  for (int i = 0; i < L; ++i) {
    const double* Bi = sB + 9 * i;
    const double bb0 = Bi[b], bb1 = Bi[3 + b], bb2 = Bi[6 + b];   // column b of B_i
    double d = sA[9 * i + l];
    double ya = -sg[3 * i + a];
    if (i > 0) {
      const double* pB = sB + 9 * (i - 1);
      const double* pC = sC + 9 * (i - 1);
      const double* py = sy + 3 * (i - 1);
      d -= pB[a] * pC[b] + pB[3 + a] * pC[3 + b] + pB[6 + a] * pC[6 + b];
      ya -= pC[a] * py[0] + pC[3 + a] * py[1] + pC[6 + a] * py[2];
    }
    M3 D;   // the upper triangle is read by sym_inv3
    D.a[0][0] = __shfl(d, 0, 64);
    D.a[0][1] = __shfl(d, 1, 64);
    D.a[0][2] = __shfl(d, 2, 64);
    D.a[1][1] = __shfl(d, 4, 64);
    D.a[1][2] = __shfl(d, 5, 64);
    D.a[2][2] = __shfl(d, 8, 64);
    const M3 Di = sym_inv3(D);
    // row a of the (symmetric) inverse
    const double r0 = pick3(Di.a[0][0], Di.a[0][1], Di.a[0][2], a);
    const double r1 = pick3(Di.a[1][0], Di.a[1][1], Di.a[1][2], a);
    const double r2 = pick3(Di.a[2][0], Di.a[2][1], Di.a[2][2], a);
    const double c = r0 * bb0 + r1 * bb1 + r2 * bb2;
    if (lane < 9) {
      sDi[9 * i + l] = pick3(r0, r1, r2, b);
      sC[9 * i + l] = c;
      if (b == 0) sy[3 * i + a] = ya;
    }
    if (i == L - 1) last = Di;
  }
}

// counts (may be NULL): the poses of window r (<= Ls); the arrays are strided for Ls poses.
__global__ __launch_bounds__(kLagThreads) void k_fixedlag(int Ls, const int32_t* __restrict__ counts,
                                                          const double* __restrict__ x0,
                                                          const double* __restrict__ prior,
                                                          const double* __restrict__ odo,
                                                          const double* __restrict__ scan, int iters,
                                                          double* __restrict__ xout, double* __restrict__ cov) {
  extern __shared__ __align__(16) double s_lag[];
  double* sx = s_lag;
  double* sA = sx + 3 * Ls;
  double* sB = sA + 9 * Ls;
  double* sg = sB + 9 * Ls;
  double* sDi = sg + 3 * Ls;
  double* sC = sDi + 9 * Ls;
  double* sy = sC + 9 * Ls;
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int L = counts ? min(max(counts[r], 1), Ls) : Ls;   // uniform over the wavefront
  for (int e = lane; e < 3 * L; e += kLagThreads) sx[e] = x0[(int64_t)r * Ls * 3 + e];
  const double* pr = prior + 6 * (int64_t)r;
  const double* od = odo + (int64_t)r * (Ls > 1 ? Ls - 1 : 0) * 6;
  const double* sc = scan + (int64_t)r * Ls * 6;
  M3 last;
  for (int it = 0; it <= iters; ++it) {
    __syncthreads();
    for (int i = lane; i < L; i += kLagThreads) linearise_pose(sx, L, i, pr, od, sc, sA + 9 * i, sB + 9 * i, sg + 3 * i);
    __syncthreads();
    eliminate_sweep9(L, lane, sA, sB, sg, sDi, sC, sy, last);
    __syncthreads();
    if (it < iters) {
      // back-substitution over three lanes (lane a of 3 the component a of each pose's step); the
      // steps reach every lane by shuffles
      const int a = lane % 3;
      double dn0 = 0.0, dn1 = 0.0, dn2 = 0.0;
      for (int i = L - 1; i >= 0; --i) {
        const double* Di = sDi + 9 * i + 3 * a;
        const double* C = sC + 9 * i + 3 * a;
        const double* y = sy + 3 * i;
        double d = Di[0] * y[0] + Di[1] * y[1] + Di[2] * y[2];
        if (i < L - 1) d -= C[0] * dn0 + C[1] * dn1 + C[2] * dn2;
        if (lane < 3) sx[3 * i + a] += d;
        dn0 = __shfl(d, 0, 64);
        dn1 = __shfl(d, 1, 64);
        dn2 = __shfl(d, 2, 64);
      }
    } else if (lane == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) cov[9 * (int64_t)r + 3 * a + b] = last.a[a][b];
    }
  }
  __syncthreads();
  for (int e = lane; e < 3 * L; e += kLagThreads) xout[(int64_t)r * Ls * 3 + e] = sx[e];
}

#pragma clang fp contract(off)

}  // namespace

namespace aslam {
namespace slam {

hipError_t launch_fixedlag(int32_t n, int32_t L, const int32_t* counts, const double* x0, const double* prior,
                           const double* odo, const double* scan, int32_t iters, double* x, double* cov,
                           hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int bytes = (int)(sizeof(double) * 45 * L);
  k_fixedlag<<<n, kLagThreads, bytes, stream>>>(L, counts, x0, prior, odo, scan, iters, x, cov);
  return hipGetLastError();
}

}  // namespace slam
}  // namespace aslam
