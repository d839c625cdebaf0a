// Thin SVD of a tall matrix (the shooting Jacobian, N x n with n = M + 1 <= N) for the
// Levenberg-Marquardt driver (App. C: J = U S V^T, p~ = V^T p, r~ = U^T r).
//
// One-sided Jacobi (Hestenes): the columns of W = J are rotated in pairs until every
// pair is orthogonal to the tolerance; then W = U S and V holds the accumulated
// rotations.  A sweep visits every pair once in n2 - 1 rounds (n2 = n rounded up to an
// even count) of n2 / 2 disjoint pairs by the circle method, one workgroup per pair,
// so a round is one launch.  Dot products are reduced in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

#define SVD_NT 256

__device__ inline void svd_reduce3(double& a, double& b, double& c, double* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
    c += __shfl_xor(c, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[3 * w] = a;
    sh[3 * w + 1] = b;
    sh[3 * w + 2] = c;
  }
  __syncthreads();
  a = sh[0] + sh[3] + sh[6] + sh[9];
  b = sh[1] + sh[4] + sh[7] + sh[10];
  c = sh[2] + sh[5] + sh[8] + sh[11];
}

// Round `rd` (0 .. n2 - 2): pair q joins players (rd + q) and (rd - q) mod (n2 - 1), and
// pair 0 joins rd with the fixed player n2 - 1; players >= n are padding.
__global__ __launch_bounds__(SVD_NT) void k_jacobi_round(double* __restrict__ W, int N, double* __restrict__ V, int n,
                                                        int n2, int rd, double tol, int* __restrict__ flag) {
  __shared__ double sh[12];
  __shared__ double cs[2];
  __shared__ int rot;
  const int m = n2 - 1, q = blockIdx.x;
  int a = q == 0 ? rd : (rd + q) % m;
  int b = q == 0 ? m : (rd - q + m) % m;
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
  if (b >= n) return;   // (uniform per workgroup)
  double* wa = W + (size_t)a * N;
  double* wb = W + (size_t)b * N;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = threadIdx.x; i < N; i += SVD_NT) {
    const double x = wa[i], y = wb[i];
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  svd_reduce3(al, be, ga, sh);
  if (threadIdx.x == 0) {
    rot = 0;
    if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
      // the rotation that zeroes the off-diagonal of [[al, ga], [ga, be]]
      const double zeta = (be - al) / (2.0 * ga);
      const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + t * t);
      cs[0] = c;
      cs[1] = c * t;
      rot = 1;
      atomicOr(flag, 1);
    }
  }
  __syncthreads();
  if (!rot) return;
  const double c = cs[0], s = cs[1];
  for (int i = threadIdx.x; i < N; i += SVD_NT) {
    const double x = wa[i], y = wb[i];
    wa[i] = c * x - s * y;
    wb[i] = s * x + c * y;
  }
  double* va = V + (size_t)a * n;
  double* vb = V + (size_t)b * n;
  for (int i = threadIdx.x; i < n; i += SVD_NT) {
    const double x = va[i], y = vb[i];
    va[i] = c * x - s * y;
    vb[i] = s * x + c * y;
  }
}

// V = I (n x n)
__global__ void k_svd_eye(double* __restrict__ V, int n) {
  const size_t tot = (size_t)n * n;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x)
    V[idx] = (idx % (n + 1) == 0) ? 1.0 : 0.0;
}

// per column k of W: out_norm[k] = ||w_k||, out_dot[k] = w_k . r (r may be null)
__global__ __launch_bounds__(SVD_NT) void k_svd_cols(const double* __restrict__ W, int N, const double* __restrict__ r,
                                                    double* __restrict__ out_norm, double* __restrict__ out_dot) {
  __shared__ double sh[12];
  const double* w = W + (size_t)blockIdx.x * N;
  double a = 0.0, d = 0.0, z = 0.0;
  for (int i = threadIdx.x; i < N; i += SVD_NT) {
    const double x = w[i];
    a += x * x;
    if (r) d += x * r[i];
  }
  svd_reduce3(a, d, z, sh);
  if (threadIdx.x == 0) {
    if (out_norm) out_norm[blockIdx.x] = sqrt(a);
    if (out_dot) out_dot[blockIdx.x] = d;
  }
}

// U = W diag(1/sigma) with the columns in the order perm (sigma = 0: zero column)
__global__ void k_svd_u(const double* __restrict__ W, int N, const double* __restrict__ sig, const int* __restrict__ perm,
                        int n, double* __restrict__ U) {
  const size_t tot = (size_t)N * n;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx / N);
    const int i = (int)(idx - (size_t)k * N);
    const int src = perm[k];
    const double s = sig[src];
    U[idx] = s > 0.0 ? W[(size_t)src * N + i] / s : 0.0;
  }
}
