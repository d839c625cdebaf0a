// gfx950 kernels of the DtN / Jacobian hot path (Wilkening & Yu, overdetermined
// shooting for standing water waves).  FP64 throughout.
//
// Data layout (all device memory, column-major):
//   state column c (c = 0 base, c = 1..M Jacobian columns): 2N doubles,
//     [eta (N) | phi (N)], column stride 2N.
//   dense matrices A = I/2 + K/N and Gm = G/N: Np x Np, leading dimension Np, where
//     Np = N rounded up to the 64-row tile; the padding is the identity in A and zero
//     in Gm, so every blocked kernel works on whole 64x64 tiles.
//   solve arrays (right-hand sides, densities, gamma, DtN output): Np x R, ld Np.
//   per-point base arrays ("aux"): see AUX_* offsets.
#pragma once
#include <hip/hip_runtime.h>

#include "ww_fft.hpp"

#define WW_TB 64          // tile edge of the blocked LU / triangular solves / GEMM
#define WW_NT 256         // threads per workgroup

// per-point base quantities, each nmax doubles, at aux + AUX_x * nmax
enum {
  AUX_EX = 0,   // eta_x
  AUX_EXX,      // eta_xx
  AUX_PHS,      // varphi' (derivative of the surface potential along x)
  AUX_EP,       // exp(surface height)
  AUX_EM,       // exp(-surface height)
  AUX_U,        // phi_x on the surface
  AUX_V,        // phi_y on the surface
  AUX_W3,       // (1 + eta_x^2)^{3/2}
  AUX_COUNT
};

// Step coefficients in device memory (captured graphs stay valid when T changes):
//   coef[s * 16 + j] = a_sj dt,  coef[COEF_B + s] = b_s dt,  coef[COEF_DT] = dt
#define COEF_B 256
#define COEF_DT 300
#define COEF_SIZE 320

// -------------------------------------------------------------------------------------
// LDS helpers for real-signal pairs
// -------------------------------------------------------------------------------------

// z[t] = a[t] + i b[t] for t < N
__device__ __forceinline__ void load_pair(cplx* z, const double* a, const double* b, int N) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) z[t] = cmk(a ? a[t] : 0.0, b ? b[t] : 0.0);
}

// -------------------------------------------------------------------------------------
// state initialisation: q0 = q_fixed + basis @ params (column 0), Qdot(0) = basis
// -------------------------------------------------------------------------------------
__global__ void k_init_state(double* __restrict__ y, const double* __restrict__ basis,
                             const double* __restrict__ qfix, const double* __restrict__ params,
                             int N, int M) {
  const int R = M + 1;
  const int n2 = 2 * N;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n2 * R; idx += gridDim.x * blockDim.x) {
    const int c = idx / n2, i = idx - c * n2;
    if (c == 0) {
      double s = qfix ? qfix[i] : 0.0;
      for (int k = 0; k < M; ++k) s += basis[(size_t)k * n2 + i] * params[k];
      y[i] = s;
    } else {
      y[(size_t)c * n2 + i] = basis[(size_t)(c - 1) * n2 + i];
    }
  }
}

// -------------------------------------------------------------------------------------
// base stage prep (one workgroup).  Stage value of the base column
//   Y_s = y + sum_{j<s} a_sj dt k_j,
// then eta_x, eta_xx (spectral), varphi', exp(+-surface height) and the Dirichlet
// data varphi into column 0 of the solve array (rows N..Np-1 zero).
// Dynamic LDS: 4 N complex (three work buffers and the twiddles).
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_base_prep(
    const double* __restrict__ y, const double* __restrict__ K, double* __restrict__ Ys,
    const double* __restrict__ coef, int stage, size_t kstride, double* __restrict__ aux, int nmax,
    double* __restrict__ rhs0, int Np, const cplx* __restrict__ tw, int N, double hsurf) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  const int tid = threadIdx.x;
  load_twiddles(tws, tw, N);
  for (int i = tid; i < 2 * N; i += WW_NT) {
    double v = y[i];
    for (int j = 0; j < stage; ++j) v += coef[stage * 16 + j] * K[(size_t)j * kstride + i];
    Ys[i] = v;
  }
  __syncthreads();
  load_pair(Z, Ys, Ys + N, N);
  fft_lds(Z, S, tws, P, -1);   // spectrum of eta + i varphi
  for (int t = tid; t < N; t += WW_NT) {
    cplx E, F;
    split_pair(Z, t, N, E, F);
    const int k = wavenum(t, N);
    cplx ex = sym_deriv(E, k, N);
    cplx exx = sym_deriv(ex, k, N);
    W[t] = pack_pair(ex, exx);
    S[t] = sym_deriv(F, k, N);
  }
  fft_lds(W, Z, tws, P, +1);   // eta_x + i eta_xx
  fft_lds(S, Z, tws, P, +1);   // varphi' (imaginary part zero)
  for (int i = tid; i < N; i += WW_NT) {
    aux[AUX_EX * nmax + i] = W[i].x;
    aux[AUX_EXX * nmax + i] = W[i].y;
    aux[AUX_PHS * nmax + i] = S[i].x;
    const double s = Ys[i] + hsurf;
    aux[AUX_EP * nmax + i] = exp(s);
    aux[AUX_EM * nmax + i] = exp(-s);
    rhs0[i] = Ys[N + i];
  }
  for (int i = N + tid; i < Np; i += WW_NT) rhs0[i] = 0.0;
}

// -------------------------------------------------------------------------------------
// Kernel matrix assembly (Sec. 2.2 eq. (K1K2), App. A): A = I/2 + K/N, Gm = G/N.
//
// Entry (i, j), alpha_i - alpha_j = 2 pi d / N, d = (i - j) mod N:
//   C = cot((zeta_i - zeta_j)/2) by the branch formula of Sec. 2.2 with
//       cos x, sin x from a circulant table, cosh y, sinh y from exp(+-s_i) exp(-+s_j)
//   K1 = Im{zeta'_j C}/2,  G1 = Re{zeta'_i C}/2 - cot((alpha_i - alpha_j)/2)/2
//   diagonal: K1 = -Im{zeta''/(2 zeta')}, G1 = Re{zeta''/(2 zeta')}
//   finite depth (image surface conj zeta_j, all i, j):
//   D = cot((zeta_i - conj zeta_j)/2), K -= Im{conj(zeta'_j) D}/2, G -= Re{zeta'_i D}/2
// with zeta' = 1 + i eta_x, zeta'' = i eta_xx.  The image terms enter with a minus
// sign (the bracket of eq. (Phi) / (plemelj:1)-(plemelj:2)).
// One 64 x 64 tile per workgroup; thread (tx, ty) owns row tx and columns ty + 4m.
// -------------------------------------------------------------------------------------
__device__ __forceinline__ void cot_half_branch(double cx, double sx, double chy, double shy,
                                                double& re, double& im) {
  if (cx >= 0.0) {
    const double num = cx + chy;
    const double inv = 1.0 / (sx * sx + shy * shy);
    re = num * sx * inv;
    im = -num * shy * inv;
  } else {
    const double inv = 1.0 / (chy - cx);
    re = sx * inv;
    im = -shy * inv;
  }
}

__global__ __launch_bounds__(WW_NT) void k_assemble(
    const double* __restrict__ aux, int nmax, const double* __restrict__ cosT,
    const double* __restrict__ sinT, const double* __restrict__ c0T, double* __restrict__ A,
    double* __restrict__ Gm, float* __restrict__ A32, int N, int Np, int finite) {
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;
  const int i = blockIdx.x * WW_TB + tx;
  const int j0 = blockIdx.y * WW_TB;
  const double invN = 1.0 / (double)N;
  double exi = 0, exxi = 0, epi = 0, emi = 0;
  if (i < N) {
    exi = aux[AUX_EX * nmax + i];
    exxi = aux[AUX_EXX * nmax + i];
    epi = aux[AUX_EP * nmax + i];
    emi = aux[AUX_EM * nmax + i];
  }
  for (int jj = ty; jj < WW_TB; jj += 4) {
    const int j = j0 + jj;
    double a, gm;
    if (i >= N || j >= N) {
      a = (i == j) ? 1.0 : 0.0;
      gm = 0.0;
    } else {
      const double exj = aux[AUX_EX * nmax + j];
      const double epj = aux[AUX_EP * nmax + j];
      const double emj = aux[AUX_EM * nmax + j];
      int d = i - j;
      if (d < 0) d += N;
      const double cx = cosT[d], sx = sinT[d];
      double Kv, Gv;
      if (i != j) {
        const double e1 = epi * emj, e2 = emi * epj;   // exp(y), exp(-y), y = s_i - s_j
        const double chy = 0.5 * (e1 + e2), shy = 0.5 * (e1 - e2);
        double cre, cim;
        cot_half_branch(cx, sx, chy, shy, cre, cim);
        Kv = 0.5 * (cim + exj * cre);
        Gv = 0.5 * (cre - exi * cim) - c0T[d];
      } else {
        const double den = 1.0 / (1.0 + exi * exi);
        Kv = -0.5 * exxi * den;
        Gv = 0.5 * exxi * exi * den;
      }
      if (finite) {
        const double e1 = epi * epj, e2 = emi * emj;   // exp(+-(s_i + s_j))
        const double chy = 0.5 * (e1 + e2), shy = 0.5 * (e1 - e2);
        double dre, dim;
        cot_half_branch(cx, sx, chy, shy, dre, dim);
        Kv -= 0.5 * (dim - exj * dre);
        Gv -= 0.5 * (dre - exi * dim);
      }
      a = Kv * invN + (i == j ? 0.5 : 0.0);
      gm = Gv * invN;
    }
    if (i < Np && j < Np) {
      const size_t o = (size_t)j * Np + i;
      A[o] = a;
      Gm[o] = gm;
      if (A32) A32[o] = (float)a;
    }
  }
}

// -------------------------------------------------------------------------------------
// 64 x 64 tile routines.  LDS tiles are row-major with a pad column: T[r * TLD + c].
// Every routine is called by all WW_NT = 256 threads of the workgroup.
// -------------------------------------------------------------------------------------
#define TLD 65
#define TILE_DBL (64 * TLD)

// global (column-major, ld) -> LDS tile; all 16 loads of a thread are issued first
__device__ inline void tile_load(double* T, const double* __restrict__ G, size_t ld) {
  double v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    v[m] = G[(size_t)(idx >> 6) * ld + (idx & 63)];
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    T[(idx & 63) * TLD + (idx >> 6)] = v[m];
  }
}
// same for a tile of right-hand sides with ncol valid columns (the rest are zero)
__device__ inline void rhs_tile_load(double* T, const double* __restrict__ G, size_t ld, int ncol) {
  double v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    const int c = idx >> 6;
    v[m] = (c < ncol) ? G[(size_t)c * ld + (idx & 63)] : 0.0;
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    T[(idx & 63) * TLD + (idx >> 6)] = v[m];
  }
}
__device__ inline void tile_store(const double* T, double* __restrict__ G, size_t ld, int ncol = 64,
                                  double scale = 1.0) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    const int c = idx >> 6;
    if (c < ncol) G[(size_t)c * ld + (idx & 63)] = scale * T[(idx & 63) * TLD + c];
  }
}

// -------------------------------------------------------------------------------------
// MFMA 64 x 64 x 64 product of two LDS tiles: acc = As * Bs.
// Wave w computes the 32 x 32 quadrant (w >> 1, w & 1) as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64.  Operand layout (lane l): A[row l%16][k l/16],
// B[k l/16][col l%16]; result lane l holds column l%16, rows 4 i + l/16, i = 0..3.
// -------------------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

struct Acc64 {
  dbl4 v[2][2];
};

__device__ inline void acc_zero(Acc64& acc) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc.v[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
}

__device__ inline void mfma_tile(const double* As, const double* Bs, Acc64& acc) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < 64; k += 4) {
    const double a0 = As[(r0 + li) * TLD + k + lk];
    const double a1 = As[(r0 + 16 + li) * TLD + k + lk];
    const double b0 = Bs[(k + lk) * TLD + c0 + li];
    const double b1 = Bs[(k + lk) * TLD + c0 + 16 + li];
    acc.v[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.v[0][0], 0, 0, 0);
    acc.v[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.v[0][1], 0, 0, 0);
    acc.v[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.v[1][0], 0, 0, 0);
    acc.v[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.v[1][1], 0, 0, 0);
  }
}

// acc into an LDS tile: T = s * acc (mode 0) or T += s * acc (mode 1)
__device__ inline void acc_to_lds(const Acc64& acc, double* T, int mode, double s) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int col = lane & 15, rq = lane >> 4;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = r0 + 16 * a + 4 * i + rq;
        const int cc = c0 + 16 * b + col;
        if (mode == 0) T[rr * TLD + cc] = s * acc.v[a][b][i];
        else T[rr * TLD + cc] += s * acc.v[a][b][i];
      }
}

// -------------------------------------------------------------------------------------
// In-place Gauss-Jordan inverse of the 64 x 64 LDS tile T (no pivoting).  Thread
// (tr = tid & 15, tc = tid >> 4) keeps the 4 x 4 block rows 4tr.., columns 4tc.. in
// registers; per elimination step the pivot row and pivot column are published in
// LDS (double-buffered, one barrier per step).  Returns the smallest |pivot|.
// `pub` is LDS scratch of 4 * 64 doubles.
// -------------------------------------------------------------------------------------
__device__ inline double lds_gj_inverse(double* T, double* pub) {
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  const int R0 = 4 * tr, C0 = 4 * tc;
  double v[4][4];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) v[i][j] = T[(R0 + i) * TLD + C0 + j];
  double minpiv = 1e300;
  for (int pb = 0; pb < 16; ++pb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = 4 * pb + q;
      double* prow = pub + (p & 1) * 128;
      double* pcol = prow + 64;
      if (tr == pb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) prow[C0 + j] = v[q][j];
      }
      if (tc == pb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) pcol[R0 + i] = v[i][q];
      }
      __syncthreads();
      const double piv = prow[p];
      minpiv = fmin(minpiv, fabs(piv));
      const double ip = 1.0 / piv;
      double pr[4], pc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) pr[j] = prow[C0 + j] * ip;
#pragma unroll
      for (int i = 0; i < 4; ++i) pc[i] = pcol[R0 + i];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool prow_i = (R0 + i) == p;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool pcol_j = (C0 + j) == p;
          double x = v[i][j];
          if (prow_i) x = pcol_j ? ip : pr[j];
          else x = pcol_j ? -pc[i] * ip : x - pc[i] * pr[j];
          v[i][j] = x;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) T[(R0 + i) * TLD + C0 + j] = v[i][j];
  __syncthreads();
  return minpiv;
}

// -------------------------------------------------------------------------------------
// Block LU factorisation (Sec. 3.3: one factorisation of I/2 + K per stage), 64-blocks,
// no pivoting (A is diagonally dominant; a pivot guard reports violations):
//   A = Lt Ut,  Lt unit block-lower, Ut block-upper whose diagonal blocks are the
//   Schur-complement blocks A_kk^(k); D_k = (A_kk^(k))^{-1} by Gauss-Jordan.
// Step k:  Lt_ik = A_ik D_k (i > k),  A_ij -= Lt_ik A_kj (i, j > k).
// The block-triangular inverses X = Lt^{-1} and Z = Ut^{-1} are accumulated in the
// same launches, so every later solve A^{-1} B = Z (X B) is two MFMA GEMMs:
//   X_ij (i > j) = -sum_{m=j}^{i-1} Lt_im X_mj     (rows of X final after step i-1)
//   Z_kk = D_k,  Z_ik (i < k) = V_ik D_k,  V_ij = -sum_{m=i}^{j-1} Z_im Ut_mj.
// Launch per step k (one workgroup per 64-tile task):
//   role 1 (i, j > k):  L = A_ik D_k;  A_ij -= L A_kj;  (i, j) = (k+1, k+1) then
//                       inverts its updated tile: D_{k+1}
//   role 2 (i > k, j <= k): L = A_ik D_k;  X_ik = -L (j = k) or X_ij -= L X_kj
//   role 3 (i <= k, j > k): Z_ik = D_k (i = k) or V_ik D_k (stored when j = k+1);
//                       V_kj = -D_k A_kj (i = k) or V_ij -= Z_ik A_kj
// -------------------------------------------------------------------------------------
struct BluBufs {
  double* A;      // Np x Np, overwritten by the Schur complements
  double* X;      // Lt^{-1}, strictly lower blocks (unit diagonal implicit)
  double* Z;      // Ut^{-1}, upper blocks incl. diagonal
  double* V;      // accumulators of Z (upper blocks)
  double* Dinv;   // nb x 4096, D_k column-major
  int* status;
  int Np;
  double pivguard;
};

__device__ inline double* tileptr(double* M, int Np, int i, int j) {
  return M + (size_t)j * WW_TB * Np + (size_t)i * WW_TB;
}

__device__ inline void store_dinv(const double* T, double* D) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    D[idx] = T[(idx & 63) * TLD + (idx >> 6)];
  }
}

__global__ __launch_bounds__(WW_NT) void k_blu_init(BluBufs b) {
  extern __shared__ double sm[];
  double* T = sm;
  double* pub = sm + TILE_DBL;
  tile_load(T, b.A, b.Np);
  const double mp = lds_gj_inverse(T, pub);
  if (threadIdx.x == 0 && !(mp >= b.pivguard)) atomicOr(b.status, 1);
  store_dinv(T, b.Dinv);
  tile_store(T, b.Z, b.Np);
}

__global__ __launch_bounds__(WW_NT) void k_blu_step(BluBufs b, int k) {
  extern __shared__ double sm[];
  double* As = sm;
  double* Bs = sm + TILE_DBL;
  double* pub = sm + 2 * TILE_DBL;
  const int Np = b.Np, nb = Np / WW_TB;
  const int nt = nb - k - 1;
  const int n1 = nt * nt, n2 = nt * (k + 1);
  int bid = blockIdx.x;
  int role, i, j;
  if (bid < n1) {
    role = 1; i = k + 1 + bid / nt; j = k + 1 + bid % nt;
  } else if (bid < n1 + n2) {
    bid -= n1; role = 2; i = k + 1 + bid / (k + 1); j = bid % (k + 1);
  } else {
    bid -= n1 + n2; role = 3; i = bid / nt; j = k + 1 + bid % nt;
  }
  const double* Dk = b.Dinv + (size_t)k * 4096;
  Acc64 acc;
  // the left factor: L = A_ik D_k (roles 1, 2) or Z_ik (role 3) -> As
  if (role == 3 && i == k) {
    for (int idx = threadIdx.x; idx < 4096; idx += WW_NT) As[(idx & 63) * TLD + (idx >> 6)] = Dk[idx];
    __syncthreads();
  } else {
    tile_load(As, role == 3 ? tileptr(b.V, Np, i, k) : tileptr(b.A, Np, i, k), Np);
    for (int idx = threadIdx.x; idx < 4096; idx += WW_NT) Bs[(idx & 63) * TLD + (idx >> 6)] = Dk[idx];
    __syncthreads();
    acc_zero(acc);
    mfma_tile(As, Bs, acc);
    __syncthreads();
    acc_to_lds(acc, As, 0, 1.0);
    __syncthreads();
    if (role == 3 && j == k + 1) tile_store(As, tileptr(b.Z, Np, i, k), Np);
  }
  if (role == 2 && j == k) {
    tile_store(As, tileptr(b.X, Np, i, k), Np, 64, -1.0);
    return;
  }
  // right factor: A_kj (roles 1, 3) or X_kj (role 2)
  tile_load(Bs, role == 2 ? tileptr(b.X, Np, k, j) : tileptr(b.A, Np, k, j), Np);
  __syncthreads();
  acc_zero(acc);
  mfma_tile(As, Bs, acc);
  __syncthreads();
  double* dst = role == 1 ? tileptr(b.A, Np, i, j) : role == 2 ? tileptr(b.X, Np, i, j) : tileptr(b.V, Np, i, j);
  if (role == 3 && i == k) {
    acc_to_lds(acc, As, 0, -1.0);   // first contribution: V_kj = -D_k A_kj
  } else {
    tile_load(As, dst, Np);
    __syncthreads();
    acc_to_lds(acc, As, 1, -1.0);
  }
  __syncthreads();
  if (role == 1 && i == k + 1 && j == k + 1) {
    // Schur complement block of the next step: invert it (D_{k+1} = Z_{k+1,k+1})
    const double mp = lds_gj_inverse(As, pub);
    if (threadIdx.x == 0 && !(mp >= b.pivguard)) atomicOr(b.status, 1);
    store_dinv(As, b.Dinv + (size_t)(k + 1) * 4096);
    tile_store(As, tileptr(b.Z, Np, k + 1, k + 1), Np);
    return;
  }
  tile_store(As, dst, Np);
}

// last column block of Z: Z_i,nb-1 = V_i,nb-1 D_nb-1 (i < nb - 1)
__global__ __launch_bounds__(WW_NT) void k_blu_final(BluBufs b) {
  extern __shared__ double sm[];
  double* As = sm;
  double* Bs = sm + TILE_DBL;
  const int Np = b.Np, nb = Np / WW_TB;
  const int i = blockIdx.x, k = nb - 1;
  tile_load(As, tileptr(b.V, Np, i, k), Np);
  const double* Dk = b.Dinv + (size_t)k * 4096;
  for (int idx = threadIdx.x; idx < 4096; idx += WW_NT) Bs[(idx & 63) * TLD + (idx >> 6)] = Dk[idx];
  __syncthreads();
  Acc64 acc;
  acc_zero(acc);
  mfma_tile(As, Bs, acc);
  __syncthreads();
  acc_to_lds(acc, As, 0, 1.0);
  __syncthreads();
  tile_store(As, tileptr(b.Z, Np, i, k), Np);
}

// -------------------------------------------------------------------------------------
// Blocked GEMM with split K: part[s] = sum over the k-tiles of chunk s of
// T(rb, kt) * B(kt, :), 64 x 64 output tiles.  mode 0: all k-tiles (Gm Gamma);
// mode 1: kt < rb (strictly lower X); mode 2: kt >= rb (upper Z).
// k_gemm_reduce: out = add + sum_s part[s]  (add may be null).
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_gemm_part(const double* __restrict__ T, int Np, int mode,
                                                     const double* __restrict__ B, int R,
                                                     double* __restrict__ part, int kchunk) {
  extern __shared__ double sm[];
  double* As = sm;
  double* Bs = sm + TILE_DBL;
  const size_t ld = Np;
  const int rb = blockIdx.x;
  const int c0 = blockIdx.y * 64;
  const int s = blockIdx.z;
  const int ncol = min(64, R - c0);
  const int nkt = Np / WW_TB;
  int lo = s * kchunk, hi = min(nkt, lo + kchunk);
  if (mode == 1) hi = min(hi, rb);
  if (mode == 2) lo = max(lo, rb);
  Acc64 acc;
  acc_zero(acc);
  for (int kt = lo; kt < hi; ++kt) {
    __syncthreads();
    tile_load(As, T + (size_t)kt * WW_TB * ld + (size_t)rb * WW_TB, ld);
    rhs_tile_load(Bs, B + (size_t)c0 * ld + (size_t)kt * WW_TB, ld, ncol);
    __syncthreads();
    mfma_tile(As, Bs, acc);
  }
  __syncthreads();
  acc_to_lds(acc, As, 0, 1.0);
  __syncthreads();
  tile_store(As, part + (size_t)s * ld * R + (size_t)c0 * ld + (size_t)rb * WW_TB, ld, ncol);
}

__global__ void k_gemm_reduce(const double* __restrict__ part, int nsplit, const double* __restrict__ add,
                              double* __restrict__ out, int Np, int R) {
  const size_t n = (size_t)Np * R;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    double s = add ? add[idx] : 0.0;
    for (int p = 0; p < nsplit; ++p) s += part[(size_t)p * n + idx];
    out[idx] = s;
  }
}

// -------------------------------------------------------------------------------------
// gamma = d mu / d alpha and (1/2) H gamma for a pair of columns (eq. (G)):
// spectrum of mu_a + i mu_b, gamma_hat = i k mu_hat, (H gamma)_hat = |k| mu_hat
// (both zero at k = 0 and at Nyquist).  Rows N..Np-1 of the outputs are zero.
// Dynamic LDS: 4 N complex (three work buffers and the twiddles).
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_gamma(const double* __restrict__ Mu, int Np, int ncols,
                                                 double* __restrict__ Gam, double* __restrict__ HG,
                                                 const cplx* __restrict__ tw, int N) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  const int ca = 2 * blockIdx.x, cb = ca + 1;
  const bool hasb = cb < ncols;
  const int tid = threadIdx.x;
  for (int t = tid; t < N; t += WW_NT)
    Z[t] = cmk(Mu[(size_t)ca * Np + t], hasb ? Mu[(size_t)cb * Np + t] : 0.0);
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    cplx A, B;
    split_pair(Z, t, N, A, B);
    const int k = wavenum(t, N);
    const double hk = (k == 0 || 2 * k == N || 2 * k == -N) ? 0.0 : 0.5 * fabs((double)k);
    W[t] = pack_pair(sym_deriv(A, k, N), cscale(A, hk));
    S[t] = pack_pair(sym_deriv(B, k, N), cscale(B, hk));
  }
  fft_lds(W, Z, tws, P, +1);
  fft_lds(S, Z, tws, P, +1);
  for (int t = tid; t < Np; t += WW_NT) {
    const bool in = t < N;
    Gam[(size_t)ca * Np + t] = in ? W[t].x : 0.0;
    HG[(size_t)ca * Np + t] = in ? W[t].y : 0.0;
    if (hasb) {
      Gam[(size_t)cb * Np + t] = in ? S[t].x : 0.0;
      HG[(size_t)cb * Np + t] = in ? S[t].y : 0.0;
    }
  }
}

// -------------------------------------------------------------------------------------
// Base right-hand side (Sec. 2.1 eq. (ww), (uv:from:G)), one workgroup:
//   u = (varphi' - eta_x G phi)/(1 + eta_x^2),  v = (eta_x varphi' + G phi)/(1 + eta_x^2)
//   eta_t = G phi
//   varphi_t = P[v eta_t - u^2/2 - v^2/2 - g eta + tau d/dx(eta_x/sqrt(1 + eta_x^2))]
// both filtered; u, v, (1 + eta_x^2)^{3/2} are kept for the variational columns.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_base_rhs(const double* __restrict__ Ys, const double* __restrict__ Gphi,
                                                    double* __restrict__ aux, int nmax, double* __restrict__ Kout,
                                                    const cplx* __restrict__ tw, const double* __restrict__ sig,
                                                    int N, double g, double tau) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  const int tid = threadIdx.x;
  load_twiddles(tws, tw, N);
  for (int t = tid; t < N; t += WW_NT) {
    const double ex = aux[AUX_EX * nmax + t];
    const double ps = aux[AUX_PHS * nmax + t];
    const double G = Gphi[t];
    const double den = 1.0 + ex * ex;
    const double u = (ps - ex * G) / den;
    const double v = (ex * ps + G) / den;
    aux[AUX_U * nmax + t] = u;
    aux[AUX_V * nmax + t] = v;
    aux[AUX_W3 * nmax + t] = den * sqrt(den);
    const double eta = Ys[t];
    Z[t] = cmk(G, v * G - 0.5 * u * u - 0.5 * v * v - g * eta);
    S[t] = cmk(tau * ex / sqrt(den), 0.0);
  }
  fft_lds(Z, W, tws, P, -1);
  fft_lds(S, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    cplx A, C, F, dummy;
    split_pair(Z, t, N, A, C);
    split_pair(S, t, N, F, dummy);
    const int k = wavenum(t, N);
    const double sg = sig[t];
    cplx et = cscale(A, sg);
    cplx pt = (k == 0) ? cmk(0.0, 0.0) : cscale(cadd(C, sym_deriv(F, k, N)), sg);
    W[t] = pack_pair(et, pt);
  }
  fft_lds(W, Z, tws, P, +1);
  for (int t = tid; t < N; t += WW_NT) {
    Kout[t] = W[t].x;
    Kout[N + t] = W[t].y;
  }
}

// -------------------------------------------------------------------------------------
// Column stage values and Dirichlet data of the variational columns (App. B, (l4)):
//   Ydot_s = ydot + sum_{j<s} a_sj dt kdot_j,  psidot = phidot - phi_y etadot
// Psi column c-1 (ld Np, rows N..Np-1 zero) for state column c = 1..M.
// -------------------------------------------------------------------------------------
__global__ void k_col_pre(const double* __restrict__ y, const double* __restrict__ K, double* __restrict__ Ys,
                          const double* __restrict__ coef, int stage, size_t kstride,
                          const double* __restrict__ aux, int nmax, double* __restrict__ Psi, int Np, int N, int M) {
  const int n2 = 2 * N;
  const size_t tot = (size_t)Np * M;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / Np) + 1;
    const int i = (int)(idx - (size_t)(c - 1) * Np);
    if (i >= N) {
      Psi[idx] = 0.0;
      continue;
    }
    const size_t oe = (size_t)c * n2 + i, op = oe + N;
    double e = y[oe], p = y[op];
    for (int j = 0; j < stage; ++j) {
      const double a = coef[stage * 16 + j];
      e += a * K[(size_t)j * kstride + oe];
      p += a * K[(size_t)j * kstride + op];
    }
    Ys[oe] = e;
    Ys[op] = p;
    Psi[idx] = p - aux[AUX_V * nmax + i] * e;
  }
}

// -------------------------------------------------------------------------------------
// Variational right-hand side, one workgroup per column (App. B (l5a), (l6), (l6a)):
//   etadot_t = G psidot - d(etadot u)
//   phidot_t = P[-d(etadot u v) - u d psidot + v G psidot - g etadot
//               + tau d(d etadot / (1 + eta_x^2)^{3/2})]
// both filtered.  Spectral derivatives: pass 1 gives d psidot and d etadot; pass 2
// transforms the four real signals G psidot, etadot u, (undifferentiated terms of
// phidot_t) and (differentiated terms of phidot_t) and combines them spectrally.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_col_rhs(const double* __restrict__ Ys, const double* __restrict__ Gpsi,
                                                   int Np, const double* __restrict__ aux, int nmax,
                                                   double* __restrict__ Kout, const cplx* __restrict__ tw,
                                                   const double* __restrict__ sig, int N, double g, double tau) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  const int c = blockIdx.x + 1;
  const int tid = threadIdx.x;
  const double* ye = Ys + (size_t)c * 2 * N;
  const double* yp = ye + N;
  const double* gp = Gpsi + (size_t)(c - 1) * Np;
  const double* au = aux + AUX_U * nmax;
  const double* av = aux + AUX_V * nmax;
  const double* aw = aux + AUX_W3 * nmax;
  // pass 1: d psidot, d etadot
  for (int t = tid; t < N; t += WW_NT) Z[t] = cmk(yp[t] - av[t] * ye[t], ye[t]);
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    cplx A, B;
    split_pair(Z, t, N, A, B);
    const int k = wavenum(t, N);
    W[t] = pack_pair(sym_deriv(A, k, N), sym_deriv(B, k, N));
  }
  fft_lds(W, Z, tws, P, +1);
  // pass 2
  for (int t = tid; t < N; t += WW_NT) {
    const double e = ye[t], u = au[t], v = av[t], G = gp[t];
    const double dpsi = W[t].x, deta = W[t].y;
    Z[t] = cmk(G, e * u);
    S[t] = cmk(-u * dpsi + v * G - g * e, -e * u * v + tau * deta / aw[t]);
  }
  fft_lds(Z, W, tws, P, -1);
  fft_lds(S, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    cplx A, B, C, F;
    split_pair(Z, t, N, A, B);
    split_pair(S, t, N, C, F);
    const int k = wavenum(t, N);
    const double sg = sig[t];
    cplx et = cscale(csub(A, sym_deriv(B, k, N)), sg);
    cplx pt = (k == 0) ? cmk(0.0, 0.0) : cscale(cadd(C, sym_deriv(F, k, N)), sg);
    W[t] = pack_pair(et, pt);
  }
  fft_lds(W, Z, tws, P, +1);
  double* ko = Kout + (size_t)c * 2 * N;
  for (int t = tid; t < N; t += WW_NT) {
    ko[t] = W[t].x;
    ko[N + t] = W[t].y;
  }
}

// -------------------------------------------------------------------------------------
// End of step, one workgroup per state column: y <- S_F[y + sum_s b_s dt k_s]
// (the filter is applied to the solution after every step, Sec. 2.2).
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_step_end(double* __restrict__ y, const double* __restrict__ K,
                                                    size_t kstride, int nst, const double* __restrict__ coef,
                                                    const cplx* __restrict__ tw, const double* __restrict__ sig,
                                                    int N, int c0) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* tws = lds + 2 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  const int c = c0 + blockIdx.x;
  double* yc = y + (size_t)c * 2 * N;
  const int tid = threadIdx.x;
  for (int t = tid; t < N; t += WW_NT) {
    double e = yc[t], p = yc[N + t];
    for (int s = 0; s < nst; ++s) {
      const double b = coef[COEF_B + s];
      if (b != 0.0) {
        e += b * K[(size_t)s * kstride + (size_t)c * 2 * N + t];
        p += b * K[(size_t)s * kstride + (size_t)c * 2 * N + N + t];
      }
    }
    Z[t] = cmk(e, p);
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) Z[t] = cscale(Z[t], sig[t]);
  fft_lds(Z, W, tws, P, +1);
  for (int t = tid; t < N; t += WW_NT) {
    yc[t] = Z[t].x;
    yc[N + t] = Z[t].y;
  }
}

// -------------------------------------------------------------------------------------
// Outputs (eq. (f:phi), (Jik), (dfdT)): r = w varphi(T/4), J = w phidot(T/4),
// drdT = w varphi_t(T/4)/4, f = r.r/2, w = 1/sqrt(N).
// -------------------------------------------------------------------------------------
__global__ void k_outputs(const double* __restrict__ y, const double* __restrict__ kT, double* __restrict__ r,
                          double* __restrict__ J, double* __restrict__ drdT, int N, int M) {
  const double w = 1.0 / sqrt((double)N);
  const size_t tot = (size_t)N * (M + 1);
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / N);
    const int i = (int)(idx - (size_t)c * N);
    const double v = w * y[(size_t)c * 2 * N + N + i];
    if (c == 0) {
      r[i] = v;
      if (drdT && kT) drdT[i] = 0.25 * w * kT[N + i];
    } else if (J) {
      J[(size_t)(c - 1) * N + i] = v;
    }
  }
}

// f = r.r / 2: one workgroup, FP64 wavefront reduction
__global__ __launch_bounds__(WW_NT) void k_objective(const double* __restrict__ r, int N, double* __restrict__ f) {
  __shared__ double red[WW_NT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += WW_NT) s += r[i] * r[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < WW_NT / 64; ++w) t += red[w];
    f[0] = 0.5 * t;
  }
}

// copy between a dense N x R array (ld N) and a padded Np x R array (ld Np)
__global__ void k_pad_copy(const double* __restrict__ src, int lds_, double* __restrict__ dst, int ldd,
                           int nrows_src, int nrows_dst, int R) {
  const size_t tot = (size_t)nrows_dst * R;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / nrows_dst);
    const int i = (int)(idx - (size_t)c * nrows_dst);
    dst[(size_t)c * ldd + i] = (i < nrows_src) ? src[(size_t)c * lds_ + i] : 0.0;
  }
}

// non-finite scan of the state (failure detection): flag bit 2
__global__ void k_check_finite(const double* __restrict__ y, size_t n, int* __restrict__ status) {
  bool bad = false;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(y[idx])) bad = true;
  if (bad) atomicOr(status, 2);
}
