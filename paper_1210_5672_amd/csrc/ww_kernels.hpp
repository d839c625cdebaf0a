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

// Per-thread element sets: thread x owns t = x + 256 m, m < NPT.  Global loads go
// through clamped, unconditional register loads (all in flight at once); only the
// stores are guarded by t < N.
#define NPT (WW_NMAX / WW_NT)

__device__ __forceinline__ int tidx(int m) { return threadIdx.x + WW_NT * m; }
__device__ __forceinline__ int tclamp(int m, int N) {
  const int t = tidx(m);
  return t < N ? t : N - 1;
}
// Pin register values at this point (stops the compiler from sinking their loads into
// later guarded blocks, which would serialise them).
__device__ __forceinline__ void pin(const double (&v)[NPT]) {
#pragma unroll
  for (int m = 0; m < NPT; ++m) asm volatile("" ::"v"(v[m]));
}
__device__ __forceinline__ void gload(double (&v)[NPT], const double* __restrict__ p, int N) {
#pragma unroll
  for (int m = 0; m < NPT; ++m) v[m] = p[tclamp(m, N)];
}

// acc[m] = y[off + t_m] + sum_{j < stage} (a_sj dt) K[j][off + t_m]: stage values of the
// thread's elements; the loads of two stages for all elements are issued together.
// crow: the count weights (a_sj dt for a stage, b_s dt for the end of a step).
__device__ __forceinline__ void stage_combine_vec(double (&acc)[NPT], const double* __restrict__ y,
                                                  const double* __restrict__ K, size_t kstride, size_t off,
                                                  const double* __restrict__ crow, int count, int N) {
#pragma unroll
  for (int m = 0; m < NPT; ++m) acc[m] = y[off + tclamp(m, N)];
  for (int j0 = 0; j0 < count; j0 += 2) {
    const int j1 = (j0 + 1 < count) ? j0 + 1 : j0;
    const double a0 = crow[j0];
    const double a1 = (j0 + 1 < count) ? crow[j0 + 1] : 0.0;
    double k0[NPT], k1[NPT];
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      k0[m] = K[(size_t)j0 * kstride + off + tclamp(m, N)];
      k1[m] = K[(size_t)j1 * kstride + off + tclamp(m, N)];
    }
    pin(k0);
    pin(k1);
#pragma unroll
    for (int m = 0; m < NPT; ++m) acc[m] = fma(a1, k1[m], fma(a0, k0[m], acc[m]));
  }
}

// Stage value at one element (column kernels: many threads, one element each).
__device__ __forceinline__ double stage_combine(double y0, const double* __restrict__ K, size_t kstride,
                                                size_t off, const double* __restrict__ coef, int stage) {
  double acc = y0;
  for (int j0 = 0; j0 < stage; j0 += 4) {
    double kv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = (j0 + q < stage) ? j0 + q : j0;
      kv[q] = K[(size_t)j * kstride + off];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (j0 + q < stage) acc = fma(coef[stage * 16 + j0 + q], kv[q], acc);
  }
  return acc;
}

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
// The prep of one stage on LDS work buffers Z, W, S and the twiddles tws (loaded).
__device__ inline void base_prep_stage(cplx* Z, cplx* W, cplx* S, const cplx* tws, const FftPlan& P,
                                       const double* __restrict__ y, const double* __restrict__ K,
                                       double* __restrict__ Ys, const double* __restrict__ coef, int stage,
                                       size_t kstride, double* __restrict__ aux, int nmax, double* __restrict__ rhs0,
                                       int Np, int N, double hsurf, int* __restrict__ status) {
  const int tid = threadIdx.x;
  double ev[NPT], pv[NPT];
  stage_combine_vec(ev, y, K, kstride, 0, coef + stage * 16, stage, N);
  stage_combine_vec(pv, y, K, kstride, N, coef + stage * 16, stage, N);
  pin(ev);
  pin(pv);
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) {
      Ys[t] = ev[m];
      Ys[N + t] = pv[m];
      Z[t] = cmk(ev[m], pv[m]);
    }
  }
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
  bool bad = false, bed = false;
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int i = tidx(m);
    if (i < N) {
      aux[AUX_EX * nmax + i] = W[i].x;
      aux[AUX_EXX * nmax + i] = W[i].y;
      aux[AUX_PHS * nmax + i] = S[i].x;
      const double sh = ev[m] + hsurf;
      aux[AUX_EP * nmax + i] = exp(sh);
      aux[AUX_EM * nmax + i] = exp(-sh);
      rhs0[i] = pv[m];
      bad |= !isfinite(ev[m]) || !isfinite(pv[m]);
      bed |= hsurf > 0.0 && sh <= 0.0;   // (a NaN height is reported as non-finite)
    }
  }
  for (int i = N + tid; i < Np; i += WW_NT) rhs0[i] = 0.0;
  // failure detection: non-finite stage state (bit 2) or, at finite depth, a surface
  // through the bottom (bit 16); status[2] keeps the first 16 step + stage (status[1]
  // counts the completed steps)
  if (status && (bad || bed)) {
    atomicOr(status, (bad ? 2 : 0) | (bed ? 16 : 0));
    atomicMin(status + 2, status[1] * 16 + stage);
  }
}

__global__ __launch_bounds__(WW_NT) void k_base_prep(
    const double* __restrict__ y, const double* __restrict__ K, double* __restrict__ Ys,
    const double* __restrict__ coef, int stage, size_t kstride, double* __restrict__ aux, int nmax,
    double* __restrict__ rhs0, int Np, const cplx* __restrict__ tw, int N, double hsurf, int* __restrict__ status) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  const int tid = threadIdx.x;
  load_twiddles(tws, tw, N);
  base_prep_stage(Z, W, S, tws, P, y, K, Ys, coef, stage, kstride, aux, nmax, rhs0, Np, N, hsurf, status);
}

// -------------------------------------------------------------------------------------
// One row of y = add + sgn * M x over the 64-block range of `mode` (0 all, 1 strictly
// lower, 2 upper incl. diagonal) from the row-major M (element type T, accumulation in
// double), by one wave: contiguous row reads, sixteen loads in flight per lane, a
// fixed-order shuffle reduction.
// -------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void gemv_row_wave(const T* __restrict__ Mr, int Np, int mode, const double* __restrict__ x,
                                              const double* __restrict__ add, double sgn, double* __restrict__ y,
                                              int row, int lane) {
  const int rb = row / WW_TB;
  const int tri = mode & 3;
  const int lo = (tri == 2) ? rb * WW_TB : 0;
  const int hi = (tri == 1) ? rb * WW_TB : Np;
  const T* mr = Mr + (size_t)row * Np;
  double s0 = 0.0, s1 = 0.0;
  int j = lo + lane;
  for (; j + 15 * 64 < hi; j += 16 * 64) {   // sixteen loads of the row in flight per lane
    T m[16];
    double xv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      m[q] = mr[j + 64 * q];
      xv[q] = x[j + 64 * q];
    }
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
      s0 = fma((double)m[q], xv[q], s0);
      s1 = fma((double)m[q + 1], xv[q + 1], s1);
    }
  }
  for (; j < hi; j += 64) s0 = fma((double)mr[j], x[j], s0);
  double s = s0 + s1;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[row] = (add ? add[row] : 0.0) + sgn * s;
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
// One strip of 64 rows x 16 columns per workgroup; thread (tx, ty) owns row tx and
// columns ty + 4m.
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

// Launch: grid (Np / 64, Np / ASM_CW): one workgroup per strip of 64 rows x ASM_CW
// columns, several workgroups per 64-tile, so that enough waves are resident to hide
// the latency of the dependent FP64 chains (divisions of the cot branch formula).
// With a lagged inverse (Mx64 or Mx32, row-major), 16 more rows of workgroups follow
// the assembly grid: they form x0 = Mx psi (the first solve of the lagged-factor base
// chain, which does not need this stage's matrix), one wave per row.
// ASM_CW: columns per assembly workgroup (16 or 32)
template <int ASM_CW>
__global__ __launch_bounds__(WW_NT) void k_assemble(
    const double* __restrict__ aux, int nmax, const double* __restrict__ cosT,
    const double* __restrict__ sinT, const double* __restrict__ c0T, double* __restrict__ A,
    double* __restrict__ Gm, float* __restrict__ A32, double* __restrict__ Gmr, double* __restrict__ Ar, int N,
    int Np, int finite, const double* __restrict__ Mx64, const float* __restrict__ Mx32,
    const double* __restrict__ psi, double* __restrict__ x0) {
  if (blockIdx.y >= (unsigned)(Np / ASM_CW)) {
    // (uniform per workgroup: no barrier below is reached by these blocks)
    const int g = (blockIdx.y - Np / ASM_CW) * gridDim.x + blockIdx.x;
    const int row = g * (WW_NT / 64) + (threadIdx.x >> 6);
    if (row >= Np) return;
    if (Mx32)
      gemv_row_wave<float>(Mx32, Np, 0, psi, nullptr, 1.0, x0, row, threadIdx.x & 63);
    else if (Mx64)
      gemv_row_wave<double>(Mx64, Np, 0, psi, nullptr, 1.0, x0, row, threadIdx.x & 63);
    return;
  }
  // stage the per-point quantities of the strip's 64 rows and 16 columns and the 79
  // circulant table entries d = i - j it touches in LDS
  __shared__ double rt[WW_TB][ASM_CW + 1];   // the strip of Gm (then A) for the row-major copies
  __shared__ double rq[4][WW_TB];            // eta_x, eta_xx, exp(s), exp(-s) of rows
  __shared__ double cq[3][ASM_CW];           // eta_x, exp(s), exp(-s) of columns
  __shared__ double tb[3][WW_TB + ASM_CW];   // cos, sin, cot/2 of 2 pi d / N, d = i - j
  const int i0 = blockIdx.x * WW_TB, j0 = blockIdx.y * ASM_CW;
  const int t = threadIdx.x;
  {
    const int q = t >> 6, r = t & 63;   // 4 x 64 row quantities
    const int ir = i0 + r;
    rq[q][r] = (ir < N) ? aux[(q == 0 ? AUX_EX : q == 1 ? AUX_EXX : q == 2 ? AUX_EP : AUX_EM) * nmax + ir] : 0.0;
    if (q < 3 && r < ASM_CW) {
      const int jc = j0 + r;
      cq[q][r] = (jc < N) ? aux[(q == 0 ? AUX_EX : q == 1 ? AUX_EP : AUX_EM) * nmax + jc] : 0.0;
    }
    // table entries e = 0..78 <-> d = (i0 - j0 - 15 + e) mod N
    constexpr int NE = WW_TB + ASM_CW - 1;
    for (int e = t; e < 3 * NE; e += WW_NT) {
      const int which = e / NE, ee = e - which * NE;
      int d = (i0 - j0 - (ASM_CW - 1) + ee) % N;
      if (d < 0) d += N;
      tb[which][ee] = which == 0 ? cosT[d] : which == 1 ? sinT[d] : c0T[d];
    }
  }
  __syncthreads();
  const int tx = t & 63;
  const int ty = t >> 6;
  const int i = i0 + tx;
  const double invN = 1.0 / (double)N;
  const double exi = rq[0][tx], exxi = rq[1][tx], epi = rq[2][tx], emi = rq[3][tx];
#pragma unroll
  for (int jj = ty; jj < ASM_CW; jj += 4) {
    const int j = j0 + jj;
    double a, gm;
    if (i >= N || j >= N) {
      a = (i == j) ? 1.0 : 0.0;
      gm = 0.0;
    } else {
      const double exj = cq[0][jj], epj = cq[1][jj], emj = cq[2][jj];
      const int e = tx - jj + (ASM_CW - 1);
      const double cx = tb[0][e], sx = tb[1][e];
      double Kv, Gv;
      if (i != j) {
        const double e1 = epi * emj, e2 = emi * epj;   // exp(y), exp(-y), y = s_i - s_j
        const double chy = 0.5 * (e1 + e2), shy = 0.5 * (e1 - e2);
        double cre, cim;
        cot_half_branch(cx, sx, chy, shy, cre, cim);
        Kv = 0.5 * (cim + exj * cre);
        Gv = 0.5 * (cre - exi * cim) - tb[2][e];
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
    const size_t o = (size_t)j * Np + i;
    A[o] = a;
    if (Gm) Gm[o] = gm;
    if (A32) A32[o] = (float)a;
    rt[tx][jj] = gm;
  }
  // row-major copies (Gmr always, Ar when given): 16 contiguous doubles per row
  __syncthreads();
  for (int idx = t; idx < WW_TB * ASM_CW; idx += WW_NT) {
    const int r = idx / ASM_CW, cc = idx % ASM_CW;
    Gmr[(size_t)(i0 + r) * Np + j0 + cc] = rt[r][cc];
  }
  if (!Ar) return;
  __syncthreads();
  for (int jj = ty; jj < ASM_CW; jj += 4) rt[tx][jj] = A[(size_t)(j0 + jj) * Np + i];
  __syncthreads();
  for (int idx = t; idx < WW_TB * ASM_CW; idx += WW_NT) {
    const int r = idx / ASM_CW, cc = idx % ASM_CW;
    Ar[(size_t)(i0 + r) * Np + j0 + cc] = rt[r][cc];
  }
}

// -------------------------------------------------------------------------------------
// 64 x 64 tile routines, templated on the element type T (double: FP64 path; float:
// the factorisation of the mixed-precision path).  LDS tiles are row-major with a pad
// column: T[r * TLD + c].  Every routine is called by all WW_NT = 256 threads.
// -------------------------------------------------------------------------------------
#define TLD 65
#define TILE_DBL (64 * TLD)

// global (column-major, ld, element type S) -> LDS tile of T; ncol valid columns, the
// rest zero; all 16 loads of a thread are issued before the stores
template <typename T, typename S>
__device__ inline void tile_load(T* Ts, const S* __restrict__ G, size_t ld, int ncol = 64) {
  S v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    const int c = idx >> 6;
    v[m] = (c < ncol) ? G[(size_t)c * ld + (idx & 63)] : S(0);
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    Ts[(idx & 63) * TLD + (idx >> 6)] = (T)v[m];
  }
}
template <typename T>
__device__ inline void rhs_tile_load(T* Ts, const double* __restrict__ G, size_t ld, int ncol) {
  tile_load<T, double>(Ts, G, ld, ncol);
}
template <typename T, typename S>
__device__ inline void tile_store(const T* Ts, S* __restrict__ G, size_t ld, int ncol = 64, T scale = T(1)) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    const int c = idx >> 6;
    if (c < ncol) G[(size_t)c * ld + (idx & 63)] = (S)(scale * Ts[(idx & 63) * TLD + c]);
  }
}

// LDS tile -> row-major global copy (the row-major matrix pointer already offset to the
// tile), coalesced along the rows
template <typename T>
__device__ inline void tile_store_rm(const T* Ts, T* __restrict__ G, size_t ld, T scale = T(1)) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    const int r = idx >> 6, c = idx & 63;
    G[(size_t)r * ld + c] = scale * Ts[r * TLD + c];
  }
}

// -------------------------------------------------------------------------------------
// MFMA 64 x 64 x 64 product of two LDS tiles: acc = As * Bs (accumulating).
// Wave w computes the 32 x 32 quadrant (w >> 1, w & 1) as 2 x 2 blocks of 16 x 16 x 4
// MFMAs (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).  Operand layout (lane l):
// A[row l%16][k l/16], B[k l/16][col l%16].  Result lane l holds column l%16 and rows
// 4 i + l/16 (f64) or 4 (l/16) + i (f32), i = 0..3.
// -------------------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef dbl4 V;
  static __device__ __forceinline__ V step(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int rq) { return 4 * i + rq; }
  // element index and lane group (lane >> 4) of the result entries in row p
  static __device__ __forceinline__ int row_elem(int p) { return p >> 2; }
  static __device__ __forceinline__ int row_grp(int p) { return p & 3; }
};
template <> struct Mfma<float> {
  typedef flt4 V;
  static __device__ __forceinline__ V step(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int i, int rq) { return 4 * rq + i; }
  static __device__ __forceinline__ int row_elem(int p) { return p & 3; }
  static __device__ __forceinline__ int row_grp(int p) { return p >> 2; }
};

template <typename T>
struct Acc64 {
  typename Mfma<T>::V v[2][2];
};

template <typename T>
__device__ inline void acc_zero(Acc64<T>& acc) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc.v[a][b] = typename Mfma<T>::V{T(0), T(0), T(0), T(0)};
}

// The operands of a wave are read from LDS a quarter of the inner dimension at a time,
// all reads of a quarter issued before its MFMAs, so that the MFMAs run back to back
// instead of each waiting for its own LDS read.
template <typename T>
__device__ inline void mfma_tile(const T* As, const T* Bs, Acc64<T>& acc) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int h = 0; h < 64; h += 16) {
    T a0[4], a1[4], b0[4], b1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = h + 4 * q;
      a0[q] = As[(r0 + li) * TLD + k + lk];
      a1[q] = As[(r0 + 16 + li) * TLD + k + lk];
      b0[q] = Bs[(k + lk) * TLD + c0 + li];
      b1[q] = Bs[(k + lk) * TLD + c0 + 16 + li];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc.v[0][0] = Mfma<T>::step(a0[q], b0[q], acc.v[0][0]);
      acc.v[0][1] = Mfma<T>::step(a0[q], b1[q], acc.v[0][1]);
      acc.v[1][0] = Mfma<T>::step(a1[q], b0[q], acc.v[1][0]);
      acc.v[1][1] = Mfma<T>::step(a1[q], b1[q], acc.v[1][1]);
    }
  }
}

// acc into an LDS tile: T = s * acc (mode 0) or T += s * acc (mode 1)
template <typename T>
__device__ inline void acc_to_lds(const Acc64<T>& acc, T* Ts, int mode, T s) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int col = lane & 15, rq = lane >> 4;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = r0 + 16 * a + Mfma<T>::row(i, rq);
        const int cc = c0 + 16 * b + col;
        if (mode == 0) Ts[rr * TLD + cc] = s * acc.v[a][b][i];
        else Ts[rr * TLD + cc] += s * acc.v[a][b][i];
      }
}

// The same product with the operands' roles swapped (the MFMA computes (A B)^T), which
// leaves the result in the column layout: lane (cl = lane & 15, rq = lane >> 4) of wave w
// holds in acc.v[a][b][i] the entry (r0 + 16 a + cl, c0 + 16 b + Mfma<T>::row(i, rq)),
// r0 = 32 (w >> 1), c0 = 32 (w & 1).  In that layout the 16 lanes of a row group hold 16
// consecutive rows of one column, so a column-major tile is read and written straight
// from and to the accumulators, 128-byte segments per row group.
template <typename T>
__device__ inline void mfma_tile_t(const T* As, const T* Bs, Acc64<T>& acc) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int h = 0; h < 64; h += 16) {
    T a0[4], a1[4], b0[4], b1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = h + 4 * q;
      a0[q] = As[(r0 + li) * TLD + k + lk];
      a1[q] = As[(r0 + 16 + li) * TLD + k + lk];
      b0[q] = Bs[(k + lk) * TLD + c0 + li];
      b1[q] = Bs[(k + lk) * TLD + c0 + 16 + li];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc.v[0][0] = Mfma<T>::step(b0[q], a0[q], acc.v[0][0]);
      acc.v[0][1] = Mfma<T>::step(b1[q], a0[q], acc.v[0][1]);
      acc.v[1][0] = Mfma<T>::step(b0[q], a1[q], acc.v[1][0]);
      acc.v[1][1] = Mfma<T>::step(b1[q], a1[q], acc.v[1][1]);
    }
  }
}

// column-major 64 x 64 global tile (leading dimension ld) <-> column-layout accumulators
template <typename T>
__device__ inline void acc_load_cm(Acc64<T>& acc, const T* __restrict__ G, size_t ld) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int cl = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc.v[a][b][i] = G[(size_t)(c0 + 16 * b + Mfma<T>::row(i, rq)) * ld + r0 + 16 * a + cl];
}
template <typename T>
__device__ inline void acc_store_cm(const Acc64<T>& acc, T* __restrict__ G, size_t ld) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int cl = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        G[(size_t)(c0 + 16 * b + Mfma<T>::row(i, rq)) * ld + r0 + 16 * a + cl] = acc.v[a][b][i];
}
// column-layout accumulators into an LDS tile: T = acc
template <typename T>
__device__ inline void acc_t_to_lds(const Acc64<T>& acc, T* Ts) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int cl = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) Ts[(r0 + 16 * a + cl) * TLD + c0 + 16 * b + Mfma<T>::row(i, rq)] = acc.v[a][b][i];
}

// -------------------------------------------------------------------------------------
// In-place Gauss-Jordan inverse of the 64 x 64 LDS tile, without pivoting.  Thread
// (tr = tid & 15, tc = tid >> 4) keeps the 4 x 4 block of rows 4tr.., columns 4tc.. in
// registers.  For pivot p every entry follows one rule,  a_rc <- a_rc - kap_r rho_c,
//   rho_c = a_pc / a_pp (c != p),  rho_p = 1 + 1/a_pp,
//   kap_r = a_rp (r != p),         kap_p = a_pp - 1,
// which yields A_QQ - a_Qp a_pQ / a_pp, a_pQ / a_pp, -a_Qp / a_pp and 1/a_pp on the four
// parts.  The pivot row and column are published in LDS (double-buffered, one barrier
// per pivot).  1/a_pp: hardware reciprocal refined by Newton steps.  `pub` is LDS
// scratch of 256 elements.  Returns the smallest |pivot|.
// -------------------------------------------------------------------------------------
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

template <typename T>
__device__ inline double lds_gj_inverse(T* Ts, T* pub) {
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  const int R0 = 4 * tr, C0 = 4 * tc;
  T v[4][4];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) v[i][j] = Ts[(R0 + i) * TLD + C0 + j];
  T minpiv = T(1e30);
  for (int pb = 0; pb < 16; ++pb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = 4 * pb + q;
      T* prow = pub + (q & 1) * 128;
      T* pcol = prow + 64;
      if (tr == pb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) prow[C0 + j] = v[q][j];
      }
      if (tc == pb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) pcol[R0 + i] = v[i][q];
      }
      __syncthreads();
      const T piv = prow[p];
      minpiv = fmin(minpiv, fabs(piv));
      const T ip = recip(piv);
      T rho[4], kap[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) rho[j] = prow[C0 + j] * ip;
#pragma unroll
      for (int i = 0; i < 4; ++i) kap[i] = pcol[R0 + i];
      if (tc == pb) rho[q] = T(1) + ip;
      if (tr == pb) kap[q] = piv - T(1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i][j] = fma(-kap[i], rho[j], v[i][j]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Ts[(R0 + i) * TLD + C0 + j] = v[i][j];
  __syncthreads();
  return (double)minpiv;
}

// -------------------------------------------------------------------------------------
// In-place inverse of the 64 x 64 LDS tile by Gauss-Jordan over 16 x 16 blocks, without
// pivoting (the rule above, applied to blocks).  Wave w keeps row band w (rows 16w ..
// 16w + 15) in registers as four 16 x 16 blocks in the MFMA result layout.  Block step P:
// wave P inverts its diagonal block in registers (the scalar rule across the wave's
// lanes: the pivot entry by a lane read, pivot row and column by lane shuffles, no
// workgroup barrier), replaces its other blocks by D B_PJ (D = B_PP^-1) and publishes
// the band; after one barrier every other wave updates B_wJ <- B_wJ - B_wP (D B_PJ) and
// B_wP <- -B_wP D, all 16 x 16 x 16 MFMA products.  The pivots are those of the scalar
// elimination.  `scr`: LDS scratch of GJ_SCR elements; it may start at Ts (each wave
// keeps its rows in registers in between).  Returns the smallest |pivot|.
// -------------------------------------------------------------------------------------
#define GJ_SLD 65
#define GJ_BAND (16 * GJ_SLD)
#define GJ_SCR (6 * GJ_BAND + 8)
static_assert(GJ_SCR <= 2 * TILE_DBL, "the inverse scratch must fit in two LDS tiles");

__device__ __forceinline__ double lane_read(double x, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float lane_read(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Broadcast of lane n of each 16-lane row to the whole row (DPP row_newbcast on the
// 64-bit move of CDNA3/4; a float travels in the low half).  n must fold to a
// constant (unrolled loops): the switch then reduces to one move.
template <int CTRL>
__device__ __forceinline__ long long dpp64(long long v) {
  return __builtin_amdgcn_update_dpp(0LL, v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ long long bits64(double v) { return __double_as_longlong(v); }
__device__ __forceinline__ long long bits64(float v) { return (long long)(unsigned)__float_as_int(v); }
__device__ __forceinline__ void from_bits64(long long u, double& v) { v = __longlong_as_double(u); }
__device__ __forceinline__ void from_bits64(long long u, float& v) { v = __int_as_float((int)(unsigned)u); }
template <typename T>
__device__ __forceinline__ T row_bcast(T v, int n) {
  const long long u = bits64(v);
  long long r;
  switch (n & 15) {
    case 0: r = dpp64<0x150>(u); break;
    case 1: r = dpp64<0x151>(u); break;
    case 2: r = dpp64<0x152>(u); break;
    case 3: r = dpp64<0x153>(u); break;
    case 4: r = dpp64<0x154>(u); break;
    case 5: r = dpp64<0x155>(u); break;
    case 6: r = dpp64<0x156>(u); break;
    case 7: r = dpp64<0x157>(u); break;
    case 8: r = dpp64<0x158>(u); break;
    case 9: r = dpp64<0x159>(u); break;
    case 10: r = dpp64<0x15a>(u); break;
    case 11: r = dpp64<0x15b>(u); break;
    case 12: r = dpp64<0x15c>(u); break;
    case 13: r = dpp64<0x15d>(u); break;
    case 14: r = dpp64<0x15e>(u); break;
    default: r = dpp64<0x15f>(u); break;
  }
  T out;
  from_bits64(r, out);
  return out;
}

// Gauss-Jordan inverse of one 16 x 16 block held by a whole wave in the MFMA result
// layout (lane: column lane & 15, rows Mfma<T>::row(i, lane >> 4)).  The pivot column
// entries a lane needs sit in lane p of its own 16-lane row (row broadcasts); the
// pivot row entry sits in another row (one lane shuffle); the pivot by a lane read.
template <typename T>
__device__ __forceinline__ void leaf_gj16(typename Mfma<T>::V& x, T& minpiv) {
  const int lane = threadIdx.x & 63;
  const int cl = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int pe = Mfma<T>::row_elem(p), pg = Mfma<T>::row_grp(p);
    const T piv = lane_read(x[pe], pg * 16 + p);     // a_pp
    const T rsrc = __shfl(x[pe], pg * 16 + cl);      // a_p,cl
    T ksrc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ksrc[i] = row_bcast(x[i], p);   // a_row(i),p
    minpiv = fmin(minpiv, fabs(piv));
    const T ip = recip(piv);
    const T rho = (cl == p) ? T(1) + ip : rsrc * ip;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T kap = (Mfma<T>::row(i, rq) == p) ? piv - T(1) : ksrc[i];
      x[i] = fma(-kap, rho, x[i]);
    }
  }
}

// The step loop stays rolled (one copy of the leaf code); blocks of the band are only
// addressed with compile-time indices under uniform branches on P (a select on P
// would be turned into a dynamically indexed private array).
template <typename T>
__device__ __forceinline__ double blk_gj_inverse(T* Ts, T* scr) {
  typedef typename Mfma<T>::V V;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cl = lane & 15, rq = lane >> 4;
  T* stg = scr + w * GJ_BAND;       // this wave's staging band
  T* pubs = scr + 4 * GJ_BAND;      // two published bands (by step parity)
  T* red = scr + 6 * GJ_BAND;       // smallest pivot of each wave's leaf
  const V zero = V{T(0), T(0), T(0), T(0)};
  V v[4];
  __syncthreads();
#pragma unroll
  for (int J = 0; J < 4; ++J)
#pragma unroll
    for (int i = 0; i < 4; ++i) v[J][i] = Ts[(16 * w + Mfma<T>::row(i, rq)) * TLD + 16 * J + cl];
  __syncthreads();   // the tile is in registers: scr may overlay Ts
  T minpiv = T(1e30);
#pragma unroll 1
  for (int P = 0; P < 4; ++P) {
    T* pub = pubs + (P & 1) * GJ_BAND;
    if (w == P) {
      // stage the band, invert the diagonal block (read back from the staging copy)
      __syncwarp();
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int i = 0; i < 4; ++i) stg[Mfma<T>::row(i, rq) * GJ_SLD + 16 * J + cl] = v[J][i];
      __syncwarp();
      V x;
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = stg[Mfma<T>::row(i, rq) * GJ_SLD + 16 * P + cl];
      leaf_gj16<T>(x, minpiv);
#pragma unroll
      for (int i = 0; i < 4; ++i) stg[Mfma<T>::row(i, rq) * GJ_SLD + 16 * P + cl] = x[i];
      __syncwarp();
#pragma unroll
      for (int J = 0; J < 4; ++J) {
        if (J == P) {
          v[J] = x;
        } else {
          V acc = zero;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            acc = Mfma<T>::step(stg[cl * GJ_SLD + 16 * P + 4 * kk + rq], stg[(4 * kk + rq) * GJ_SLD + 16 * J + cl], acc);
          v[J] = acc;
        }
      }
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int i = 0; i < 4; ++i) pub[Mfma<T>::row(i, rq) * GJ_SLD + 16 * J + cl] = v[J][i];
    }
    __syncthreads();
    if (w != P) {
      __syncwarp();
#pragma unroll
      for (int J = 0; J < 4; ++J)
        if (J == P) {
#pragma unroll
          for (int i = 0; i < 4; ++i) stg[Mfma<T>::row(i, rq) * GJ_SLD + cl] = v[J][i];   // L = B_wP
        }
      __syncwarp();
      T a[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) a[kk] = -stg[cl * GJ_SLD + 4 * kk + rq];
#pragma unroll
      for (int J = 0; J < 4; ++J) {
        V acc = (J == P) ? zero : v[J];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = Mfma<T>::step(a[kk], pub[(4 * kk + rq) * GJ_SLD + 16 * J + cl], acc);
        v[J] = acc;
      }
    }
  }
  if (lane == 0) red[w] = minpiv;
  __syncthreads();   // every wave is done with the bands before Ts is rewritten
#pragma unroll
  for (int J = 0; J < 4; ++J)
#pragma unroll
    for (int i = 0; i < 4; ++i) Ts[(16 * w + Mfma<T>::row(i, rq)) * TLD + 16 * J + cl] = v[J][i];
  __syncthreads();
  const T mp = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
  return (double)mp;
}

// -------------------------------------------------------------------------------------
// Block LU factorisation (Sec. 3.3: one factorisation of I/2 + K per stage), 64-blocks,
// no pivoting (A is diagonally dominant; a pivot guard reports violations):
//   A = Lt Ut,  Lt unit block-lower, Ut block-upper whose diagonal blocks are the
//   Schur-complement blocks A_kk^(k); D_k = (A_kk^(k))^{-1} by Gauss-Jordan.
// Step k:  Lt_ik = A_ik D_k (i > k),  A_ij -= Lt_ik A_kj (i, j > k).
// The block-triangular inverses X = Lt^{-1} and Z = Ut^{-1} are accumulated in the
// same launches, so every later solve A^{-1} B = Z (B + X B) is two MFMA GEMMs:
//   X_ij (i > j) = -sum_{m=j}^{i-1} Lt_im X_mj     (rows of X final after step i-1)
//   Z_kk = D_k,  Z_ik (i < k) = V_ik D_k,  V_ij = -sum_{m=i}^{j-1} Z_im Ut_mj.
// Launch per step k (one workgroup per 64-tile task):
//   role 1 (i, j > k):  L = A_ik D_k;  A_ij -= L A_kj;  (i, j) = (k+1, k+1) then
//                       inverts its updated tile: D_{k+1}
//   role 2 (i > k, j <= k): L = A_ik D_k;  X_ik = -L (j = k) or X_ij -= L X_kj
//   role 3 (i <= k, j > k): Z_ik = D_k (i = k) or V_ik D_k (stored when j = k+1);
//                       the diagonal Z_kk = D_k is stored here (step k), not by the
//                       workgroup that inverted the block (k_blu_final stores the last)
//                       V_kj = -D_k A_kj (i = k) or V_ij -= Z_ik A_kj
// T = double (FP64 path) or float (mixed path: factor of an FP32 copy of A).
// -------------------------------------------------------------------------------------
template <typename T>
struct BluBufs {
  T* A;      // Np x Np, overwritten by the Schur complements
  T* X;      // Lt^{-1}, strictly lower blocks (unit diagonal implicit)
  T* Z;      // Ut^{-1}, upper blocks incl. diagonal
  T* V;      // accumulators of Z (upper blocks)
  T* Dinv;   // nb x 4096, D_k column-major
  T* Xr;     // row-major copies of X and Z (one-vector solves read rows), or null
  T* Zr;
  int* status;
  int Np;
  double pivguard;
};

// Several matrices factored by one launch sequence (the lagged-factor march factors
// consecutive stages together): block b of a launch works on matrix b % count, task
// b / count, so the critical tasks (the next diagonal block of every matrix) come first.
#define BLU_GMAX 4
template <typename T>
struct BluGroup {
  BluBufs<T> m[BLU_GMAX];
  int count;
  int strip;   // tiles per strip task of a step (1..BLU_STRIP_MAX)
};
// Field by field, each a select among kernel-argument values: selecting whole structs
// makes the compiler copy the argument block into per-lane scratch memory.
template <typename T>
__device__ __forceinline__ BluBufs<T> blu_pick(const BluGroup<T>& g, int m) {
#define BLU_SEL(f) (m == 0 ? g.m[0].f : m == 1 ? g.m[1].f : m == 2 ? g.m[2].f : g.m[3].f)
  BluBufs<T> b;
  b.A = BLU_SEL(A);
  b.X = BLU_SEL(X);
  b.Z = BLU_SEL(Z);
  b.V = BLU_SEL(V);
  b.Dinv = BLU_SEL(Dinv);
  b.Xr = BLU_SEL(Xr);
  b.Zr = BLU_SEL(Zr);
  b.status = BLU_SEL(status);
  b.Np = BLU_SEL(Np);
  b.pivguard = BLU_SEL(pivguard);
#undef BLU_SEL
  return b;
}

template <typename T>
__device__ inline T* tileptr(T* M, int Np, int i, int j) {
  return M + (size_t)j * WW_TB * Np + (size_t)i * WW_TB;
}

template <typename T>
__device__ inline T* rmptr(T* M, int Np, int i, int j) {
  return M + (size_t)i * WW_TB * Np + (size_t)j * WW_TB;
}

template <typename T>
__device__ inline void store_dinv(const T* Ts, T* D) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    D[idx] = Ts[(idx & 63) * TLD + (idx >> 6)];
  }
}

template <typename T>
__global__ __launch_bounds__(WW_NT) void k_blu_init(BluGroup<T> g) {
  const BluBufs<T> b = blu_pick(g, blockIdx.x);
  extern __shared__ double sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  T* Ts = sm;
  tile_load<T, T>(Ts, b.A, b.Np);
  const double mp = blk_gj_inverse<T>(Ts, sm + TILE_DBL);
  if (threadIdx.x == 0 && !(mp >= b.pivguard)) atomicOr(b.status, 1);
  store_dinv<T>(Ts, b.Dinv);
  if (b.Np == WW_TB) {   // one block: no step launch stores Z_00
    tile_store<T, T>(Ts, b.Z, b.Np);
    if (b.Zr) tile_store_rm<T>(Ts, b.Zr, b.Np);
  }
}

// One 64 x 64 column-major tile into registers (thread t holds entries t + 256 m, m =
// 0..15, of the column-major order), then into an LDS tile; the same thread owns the
// same entries in tile_put, tile_store and tile_store_sum, so a tile kept in registers
// can be combined with an LDS tile without a barrier.
template <typename T>
__device__ inline void tile_fetch(T (&v)[16], const T* __restrict__ G, size_t ld) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    v[m] = G[(size_t)(idx >> 6) * ld + (idx & 63)];
  }
}
template <typename T>
__device__ inline void tile_put(T* Ts, const T (&v)[16]) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    Ts[(idx & 63) * TLD + (idx >> 6)] = v[m];
  }
}
// Ts += v (each thread its own entries)
template <typename T>
__device__ inline void tile_add_own(T* Ts, const T (&v)[16]) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    Ts[(idx & 63) * TLD + (idx >> 6)] += v[m];
  }
}
// G = Ts + v
template <typename T>
__device__ inline void tile_store_sum(const T* Ts, const T (&v)[16], T* __restrict__ G, size_t ld) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int idx = threadIdx.x + WW_NT * m;
    G[(size_t)(idx >> 6) * ld + (idx & 63)] = Ts[(idx & 63) * TLD + (idx >> 6)] + v[m];
  }
}

// Tasks of step k (per matrix of a group).  Task 0 updates the next diagonal tile
// (k+1, k+1) and inverts it (the critical path of the factorisation).  Every other task
// is a strip of at most `strip` tiles of one row i: it forms the row's left factor
// once (A_ik D_k for i > k; V_ik D_k for i < k; D_k itself for i = k) and applies it to
// each tile of its strip, so no product is repeated across the tiles of a row.  Row i
// > k runs over j = k+1 .. nb-1 (role 1: A_ij -= L A_kj; row k+1 without the diagonal
// tile) and then j = 0 .. k (role 2: X_ik = -L, X_ij -= L X_kj); row i <= k over
// j = k+1 .. nb-1 (role 3: V_ij -= L A_kj, V_kj = -D_k A_kj; the strip starting at
// j = k+1 also stores Z_ik = L).
#define BLU_STRIP_MAX 16
__host__ __device__ inline int blu_row_len(int nb, int k, int i) {
  return i > k ? (i == k + 1 ? nb - 1 : nb) : nb - k - 1;
}
__host__ __device__ inline int blu_step_tasks(int nb, int k, int strip) {
  int n = 1;
  for (int i = 0; i < nb; ++i) n += (blu_row_len(nb, k, i) + strip - 1) / strip;
  return n;
}

// Two LDS tiles per workgroup (two workgroups share a CU): S0 holds the negated left
// factor -L, S1 the right factor R of the current tile.  The tile C being updated goes
// from global memory straight into the MFMA accumulators (column layout), which then
// accumulate -L R and are stored straight back: C - L R summed into C in increasing
// inner index.  The next tile's R and C are in flight during the current product.
template <typename T>
__global__ __launch_bounds__(WW_NT) void k_blu_step(BluGroup<T> g, int k) {
  extern __shared__ double sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  T* S0 = sm;
  T* S1 = sm + TILE_DBL;
  const BluBufs<T> b = blu_pick(g, (int)(blockIdx.x % g.count));
  const int Np = b.Np, nb = Np / WW_TB;
  const int nt = nb - k - 1;
  const T* Dk = b.Dinv + (size_t)k * 4096;
  int q = blockIdx.x / g.count;
  Acc64<T> acc;
  if (q == 0) {
    // the next diagonal tile: L = A_{k+1,k} D_k, A_{k+1,k+1} -= L A_{k,k+1}, then its
    // inverse D_{k+1} (the inverse's scratch overlays both slots)
    T vl[16], vd[16], vr[16];
    tile_fetch<T>(vl, tileptr(b.A, Np, k + 1, k), Np);
    tile_fetch<T>(vd, Dk, 64);
    tile_fetch<T>(vr, tileptr(b.A, Np, k, k + 1), Np);
    tile_put<T>(S0, vl);
    tile_put<T>(S1, vd);
    __syncthreads();
    acc_zero(acc);
    mfma_tile(S0, S1, acc);
    __syncthreads();
    acc_to_lds(acc, S0, 0, T(-1));   // S0 = -L
    tile_put<T>(S1, vr);
    acc_load_cm<T>(acc, tileptr(b.A, Np, k + 1, k + 1), Np);
    __syncthreads();
    mfma_tile_t(S0, S1, acc);
    __syncthreads();
    acc_t_to_lds(acc, S0);
    const double mp = blk_gj_inverse<T>(S0, sm);
    if (threadIdx.x == 0 && !(mp >= b.pivguard)) atomicOr(b.status, 1);
    store_dinv<T>(S0, b.Dinv + (size_t)(k + 1) * 4096);   // Z_{k+1,k+1} is stored one step later
    return;
  }
  // the strip: row i, positions p0 .. p0 + len - 1 of the row's tile list
  q -= 1;
  int i = -1, p0 = 0, len = 0;
  for (int r = 0; r < nb; ++r) {
    const int n = blu_row_len(nb, k, r);
    const int ch = (n + g.strip - 1) / g.strip;
    if (q < ch) {
      i = r;
      p0 = q * g.strip;
      len = min(g.strip, n - p0);
      break;
    }
    q -= ch;
  }
  if (i < 0 || len <= 0) return;
  const bool low = i > k;      // roles 1 and 2
  const bool ldiag = i == k;   // role 3 on row k: the left factor is D_k
  const bool vfirst = ldiag;   // V_kj = -D_k A_kj: nothing to accumulate into
  // the tile (i, j) of position p
  auto col_of = [&](int p) {
    if (!low) return k + 1 + p;
    const int nrt = (i == k + 1) ? nt - 1 : nt;   // tiles right of column k in this row
    const int jr0 = (i == k + 1) ? k + 2 : k + 1;
    return p < nrt ? jr0 + p : p - nrt;
  };
  auto dst_of = [&](int j) {
    return (low && j <= k) ? tileptr(b.X, Np, i, j) : (low ? tileptr(b.A, Np, i, j) : tileptr(b.V, Np, i, j));
  };
  // right factor (registers) and current value (accumulator layout) of the tile at
  // position p; the X_ik = -L position reads nothing
  auto fetch = [&](int p, T (&vr)[16], Acc64<T>& cn) {
    const int j = col_of(p);
    const bool role2 = low && j <= k;
    if (role2 && j == k) return;
    tile_fetch<T>(vr, role2 ? tileptr(b.X, Np, k, j) : tileptr(b.A, Np, k, j), Np);
    if (vfirst)
      acc_zero(cn);
    else
      acc_load_cm<T>(cn, dst_of(j), Np);
  };
  T vr[16];
  Acc64<T> cn;
  {
    T vl[16], vd[16];
    tile_fetch<T>(vl, ldiag ? Dk : (low ? tileptr(b.A, Np, i, k) : tileptr(b.V, Np, i, k)), ldiag ? 64 : Np);
    if (!ldiag) tile_fetch<T>(vd, Dk, 64);
    fetch(p0, vr, cn);
    if (ldiag) {
#pragma unroll
      for (int m = 0; m < 16; ++m) vl[m] = -vl[m];
    }
    tile_put<T>(S0, vl);
    if (!ldiag) tile_put<T>(S1, vd);
    __syncthreads();
    if (!ldiag) {
      acc_zero(acc);
      mfma_tile(S0, S1, acc);
      __syncthreads();
      acc_to_lds(acc, S0, 0, T(-1));   // S0 = -L
    }
  }
  if (!low && p0 == 0) {
    __syncthreads();
    tile_store<T, T>(S0, tileptr(b.Z, Np, i, k), Np, 64, T(-1));   // Z_ik = L (Z_kk = D_k)
  }
  for (int p = p0; p < p0 + len; ++p) {
    const int j = col_of(p);
    if (low && j == k) {   // X_ik = -L (final); the last position of its row
      __syncthreads();
      tile_store<T, T>(S0, tileptr(b.X, Np, i, k), Np);
      continue;
    }
    __syncthreads();   // S1 is free (every wave is done with the previous product)
    tile_put<T>(S1, vr);
    acc = cn;
    __syncthreads();
    if (p + 1 < p0 + len) fetch(p + 1, vr, cn);
    mfma_tile_t(S0, S1, acc);
    acc_store_cm<T>(acc, dst_of(j), Np);
  }
}

// last column block of Z: Z_i,nb-1 = V_i,nb-1 D_nb-1 (i < nb - 1)
template <typename T>
__global__ __launch_bounds__(WW_NT) void k_blu_final(BluGroup<T> g) {
  extern __shared__ double sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  T* As = sm;
  T* Bs = sm + TILE_DBL;
  const BluBufs<T> b = blu_pick(g, (int)(blockIdx.x % g.count));
  const int Np = b.Np, nb = Np / WW_TB;
  const int i = blockIdx.x / g.count, k = nb - 1;
  tile_load<T, T>(As, tileptr(b.V, Np, i, k), Np);
  tile_load<T, T>(Bs, b.Dinv + (size_t)k * 4096, 64);
  __syncthreads();
  if (i == 0) {   // Z of the last diagonal block = D_{nb-1}
    tile_store<T, T>(Bs, tileptr(b.Z, Np, k, k), Np);
    if (b.Zr) tile_store_rm<T>(Bs, rmptr(b.Zr, Np, k, k), Np);
  }
  Acc64<T> acc;
  acc_zero(acc);
  mfma_tile(As, Bs, acc);
  __syncthreads();
  acc_to_lds(acc, As, 0, T(1));
  __syncthreads();
  tile_store<T, T>(As, tileptr(b.Z, Np, i, k), Np);
  if (b.Zr) tile_store_rm<T>(As, rmptr(b.Zr, Np, i, k), Np);
}

// -------------------------------------------------------------------------------------
// Explicit inverse from the block LU: A^{-1} = Ut^{-1} Lt^{-1} = Z (I + X), written
// row-major (the one-vector products read it along rows, the column products read
// row-major tiles), so that every later solve is one product.  Output tile (i, j):
//   [i <= j] Z_ij + sum_{m = max(i, j+1)}^{nb-1} Z_im X_mj,
// one tile per task, the sum in increasing m (fixed order).  The next pair of tiles is in
// flight in registers during the MFMAs of the current one.
// -------------------------------------------------------------------------------------
// Matrices of a group (Z, X, Mr of matrix z).
template <typename T>
struct MinvGroup {
  const T* Z[BLU_GMAX];
  const T* X[BLU_GMAX];
  T* Mr[BLU_GMAX];
  float* Mr32[BLU_GMAX];   // optional FP32 row-major copy of the inverse (null: none)
  int count;
};

// Tile of rank r in decreasing order of work: level m = max(i, j + 1) holds the 2m
// tiles (m, 0..m-1) and (0..m-1, m-1) with nb - m products each (m < nb), level nb the
// nb tiles (0..nb-1, nb-1) with none; level m starts at rank m (m - 1).
__host__ __device__ inline void minv_tile(int r, int nb, int& i, int& j) {
  if (r >= nb * (nb - 1)) {
    i = r - nb * (nb - 1);
    j = nb - 1;
    return;
  }
  int m = (int)((1.0 + sqrt(1.0 + 4.0 * (double)r)) * 0.5);
  while (m > 1 && m * (m - 1) > r) --m;
  while ((m + 1) * m <= r) ++m;
  const int idx = r - m * (m - 1);
  if (idx < m) {
    i = m;
    j = idx;
  } else {
    i = idx - m;
    j = m - 1;
  }
}

// A fixed grid works through the tiles of every matrix of the group, longest sums
// first, so that the launch occupies a bounded number of compute units: the inverse is
// not on the critical path of the march (it is first read `lag` stages later) and the
// units it leaves free serve the latency-bound base chain.
template <typename T>
__global__ __launch_bounds__(WW_NT) void k_minv(MinvGroup<T> gr, int Np) {
  extern __shared__ double sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  T* As = sm;
  T* Bs = sm + TILE_DBL;
  const int nb = Np / WW_TB;
  const int ntask = nb * nb * gr.count;
  for (int task = blockIdx.x; task < ntask; task += gridDim.x) {
    const int z = task % gr.count;
    int i, j;
    minv_tile(task / gr.count, nb, i, j);
    const T* __restrict__ Z = z == 0 ? gr.Z[0] : z == 1 ? gr.Z[1] : z == 2 ? gr.Z[2] : gr.Z[3];
    const T* __restrict__ X = z == 0 ? gr.X[0] : z == 1 ? gr.X[1] : z == 2 ? gr.X[2] : gr.X[3];
    T* __restrict__ Mr = z == 0 ? gr.Mr[0] : z == 1 ? gr.Mr[1] : z == 2 ? gr.Mr[2] : gr.Mr[3];
    float* __restrict__ Mr32 = z == 0 ? gr.Mr32[0] : z == 1 ? gr.Mr32[1] : z == 2 ? gr.Mr32[2] : gr.Mr32[3];
    const int m0 = max(i, j + 1);
    Acc64<T> acc;
    acc_zero(acc);
    T za[16], xb[16];
    if (m0 < nb) {
      tile_fetch<T>(za, tileptr(Z, Np, i, m0), Np);
      tile_fetch<T>(xb, tileptr(X, Np, m0, j), Np);
    }
    for (int m = m0; m < nb; ++m) {
      __syncthreads();
      tile_put<T>(As, za);
      tile_put<T>(Bs, xb);
      __syncthreads();
      if (m + 1 < nb) {
        tile_fetch<T>(za, tileptr(Z, Np, i, m + 1), Np);
        tile_fetch<T>(xb, tileptr(X, Np, m + 1, j), Np);
      }
      mfma_tile(As, Bs, acc);
    }
    __syncthreads();
    if (i <= j) {
      tile_load<T, T>(As, tileptr(Z, Np, i, j), Np);
      __syncthreads();
      acc_to_lds(acc, As, 1, T(1));
    } else {
      acc_to_lds(acc, As, 0, T(1));
    }
    __syncthreads();
    tile_store_rm<T>(As, rmptr(Mr, Np, i, j), Np);
    if (Mr32) {
      float* G = rmptr(Mr32, Np, i, j);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int idx = threadIdx.x + WW_NT * m;
        const int r = idx >> 6, c = idx & 63;
        G[(size_t)r * Np + c] = (float)As[r * TLD + c];
      }
    }
  }
}

// -------------------------------------------------------------------------------------
// Pivoting fallback.  The paper factors A without discussing pivoting (Sec. 3.3); A is
// diagonally dominant for the surfaces it treats, and the block LU above runs without
// interchanges behind a pivot guard.  When a pivot falls below the guard, Gaussian
// elimination with partial pivoting (largest magnitude in the column, first row on
// ties) fixes a row order P; the block LU then factors P A, whose elimination pivots
// are the partial-pivoting ones, and every solve gathers its right-hand side by P.
// Two launches per column of the leading N x N block of W (column-major, ld Np):
// k_plu_pivot (one workgroup) picks the pivot, interchanges the two rows over all
// columns, records the interchange in perm ((P A) row i = A row perm[i]) and forms the
// multipliers; k_plu_update subtracts the rank-one update from the trailing block.
// Status bit 8: the largest candidate of a column is below the guard.
// -------------------------------------------------------------------------------------
#define PLU_NT 1024
__global__ __launch_bounds__(PLU_NT) void k_plu_pivot(double* __restrict__ W, int Np, int N, int k,
                                                       int* __restrict__ perm, double guard, int* __restrict__ status) {
  __shared__ double sv[PLU_NT / 64];
  __shared__ int si[PLU_NT / 64];
  __shared__ int sp;
  double* col = W + (size_t)k * Np;
  double bv = -1.0;
  int bi = N;
  for (int i = k + (int)threadIdx.x; i < N; i += PLU_NT) {   // rising rows: ties keep the first
    const double v = fabs(col[i]);
    if (v > bv) {
      bv = v;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sv[w] = bv;
    si[w] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = sv[0];
    int p = si[0];
    for (int q = 1; q < PLU_NT / 64; ++q)
      if (sv[q] > v || (sv[q] == v && si[q] < p)) {
        v = sv[q];
        p = si[q];
      }
    if (!(v >= guard)) atomicOr(status, 8);
    if (p < k || p >= N) p = k;   // no finite candidate (NaN column): keep the order
    sp = p;
    if (p != k) {
      const int t = perm[k];
      perm[k] = perm[p];
      perm[p] = t;
    }
  }
  __syncthreads();
  const int p = sp;
  if (p != k)
    for (int j = threadIdx.x; j < Np; j += PLU_NT) {
      double* cj = W + (size_t)j * Np;
      const double t = cj[k];
      cj[k] = cj[p];
      cj[p] = t;
    }
  __syncthreads();
  const double piv = col[k];
  for (int i = k + 1 + (int)threadIdx.x; i < N; i += PLU_NT) col[i] = col[i] / piv;
}

// W[i][j] -= W[i][k] W[k][j] for k < i, j < N: 64 rows x 16 columns per workgroup
__global__ __launch_bounds__(256) void k_plu_update(double* __restrict__ W, int Np, int N, int k) {
  const int i = k + 1 + blockIdx.x * 64 + (threadIdx.x & 63);
  if (i >= N) return;
  const double l = W[(size_t)k * Np + i];
  const int j0 = k + 1 + blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + q;
    if (j < N) W[(size_t)j * Np + i] -= l * W[(size_t)j * Np + k];
  }
}

__global__ void k_iota(int* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// rows of an Np x ncols column-major array (ld Np) by perm: gather dst[i] = src[perm[i]]
// (P x), or scatter dst[perm[i]] = src[i] (P^T x)
__global__ void k_permute_rows(const double* __restrict__ src, double* __restrict__ dst, const int* __restrict__ perm,
                               int Np, int ncols, int scatter) {
  const size_t tot = (size_t)Np * ncols;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t c = idx / Np;
    const int i = (int)(idx - c * Np);
    const int q = perm[i];
    if (scatter) dst[c * Np + q] = src[c * Np + i];
    else dst[c * Np + i] = src[c * Np + q];
  }
}

// -------------------------------------------------------------------------------------
// One right-hand side: y = add + sgn * M x over the 64-block range of `mode` (0 all,
// 1 strictly lower, 2 upper incl. diagonal), from the row-major copy Mr (element type
// T, accumulation in double).  One wave per row: contiguous row reads, eight loads in
// flight per lane, a fixed-order shuffle reduction (no cross-workgroup reduction).
// -------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(WW_NT) void k_gemv_row(const T* __restrict__ Mr, int Np, int mode,
                                                    const double* __restrict__ x, const double* __restrict__ add,
                                                    double sgn, double* __restrict__ y) {
  const int row = (blockIdx.x * WW_NT + threadIdx.x) >> 6;
  if (row >= Np) return;
  gemv_row_wave<T>(Mr, Np, mode, x, add, sgn, y, row, threadIdx.x & 63);
}


// -------------------------------------------------------------------------------------
// Product with a row-major matrix for R right-hand sides:  out = add + sgn * M B
// (M: Np x Np row-major, element type T; B, add, out: Np x R column-major doubles,
// ld Np; B is rounded to T on load).  One workgroup per TR x 32 output tile: the inner
// dimension is split over GSPLIT wave groups (group g takes the 64-wide steps g,
// g + GSPLIT, ...), in each group every wave computes one 16 x 16 block with
// 16 x 16 x 4 MFMAs, the next step's operands in flight in
// registers during the MFMAs; the partial tiles are summed in LDS in a fixed order,
// ((g0 + g1) + g2) + g3, so each entry is one deterministic sum (no partials in
// memory, no second launch).  The result is stored along the columns.
// -------------------------------------------------------------------------------------
#define GT 32           // output tile edge
#define GK 64           // inner step
#define GA_LD (GK + 1)  // LDS pitch of the M tile (TR rows x 64) and of the B tile (32 columns x 64)
// GSPLIT: wave groups splitting the inner dimension (2 or 4); TR: rows of the output
// tile (32, or 16 for twice the workgroups at the same columns); a group has TR / 8
// waves, each computing one 16 x 16 block of the TR x 32 tile.
template <typename T, int GSPLIT, int TR>
__global__ __launch_bounds__(8 * TR * GSPLIT) void k_gemm_rm(const T* __restrict__ M, int Np,
                                                          const double* __restrict__ B, int R,
                                                          const double* __restrict__ add, double sgn,
                                                          double* __restrict__ out) {
  constexpr int WPG = TR / 8;         // waves per group
  constexpr int TPG = 64 * WPG;       // threads per group
  constexpr int MA = TR * 64 / TPG;   // M-tile entries per thread and step (8)
  constexpr int MB = 32 * 64 / TPG;   // B-tile entries per thread and step (8 or 16)
  // operand tiles of the groups; after the inner loop the same memory holds the
  // partial output tiles
  constexpr int OPER = GSPLIT * (TR + GT) * GA_LD * (int)sizeof(T);
  constexpr int PART = GSPLIT * GT * (TR + 1) * (int)sizeof(double);
  __shared__ double smem[(OPER > PART ? OPER : PART) / 8];
  T* const tiles = reinterpret_cast<T*>(smem);
  double (*Cs)[GT * (TR + 1)] = reinterpret_cast<double (*)[GT * (TR + 1)]>(smem);
  typedef typename Mfma<T>::V V;
  const int r0 = blockIdx.x * TR, c0 = blockIdx.y * GT;
  const int tid = threadIdx.x;
  const int grp = tid / TPG, gt = tid % TPG;   // wave group and thread within it
  const int lane = gt & 63, w = gt >> 6;
  const int wr = (TR == 32 ? (w >> 1) : 0) * 16, wc = (w & 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  T* as = tiles + (size_t)grp * (TR + GT) * GA_LD;
  T* bs = as + TR * GA_LD;
  // loads of one inner step by the threads of a group: MA entries of the M tile (rows
  // r0 + w + WPG m, columns k0..) and MB of the B tile (columns c0 + w + WPG m)
  T ma[MA];
  double bv[MB];
  auto fetch = [&](int k0) {
    const int kk = gt & 63;
#pragma unroll
    for (int m = 0; m < MA; ++m) ma[m] = M[(size_t)(r0 + (gt >> 6) + WPG * m) * Np + k0 + kk];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int cc = c0 + (gt >> 6) + WPG * m;
      bv[m] = cc < R ? B[(size_t)cc * Np + k0 + kk] : 0.0;
    }
  };
  // two accumulators (even and odd 4-steps of the inner dimension): two independent
  // MFMA chains per wave, summed once at the end
  V acc = V{T(0), T(0), T(0), T(0)};
  V acc1 = V{T(0), T(0), T(0), T(0)};
  const int nsteps = Np / GK;
  if (grp < nsteps) fetch(grp * GK);
  // every group runs the same number of iterations (barriers are workgroup-wide); a
  // group without a step in an iteration only waits
  for (int it = 0; it * GSPLIT < nsteps; ++it) {
    const int st = it * GSPLIT + grp;
    const bool have = st < nsteps;
    __syncthreads();
    if (have) {
      const int kk = gt & 63;
#pragma unroll
      for (int m = 0; m < MA; ++m) as[((gt >> 6) + WPG * m) * GA_LD + kk] = ma[m];
#pragma unroll
      for (int m = 0; m < MB; ++m) bs[((gt >> 6) + WPG * m) * GA_LD + kk] = (T)bv[m];
    }
    __syncthreads();
    if (have && st + GSPLIT < nsteps) fetch((st + GSPLIT) * GK);
    if (have) {
#pragma unroll
      for (int h = 0; h < GK; h += 32) {
        T a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a[q] = as[(wr + li) * GA_LD + h + 4 * q + lk];
          b[q] = bs[(wc + li) * GA_LD + h + 4 * q + lk];
        }
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
          acc = Mfma<T>::step(a[q], b[q], acc);
          acc1 = Mfma<T>::step(a[q + 1], b[q + 1], acc1);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] += acc1[i];
  __syncthreads();   // every group is done with its operand tiles
#pragma unroll
  for (int i = 0; i < 4; ++i) Cs[grp][(wc + li) * (TR + 1) + wr + Mfma<T>::row(i, lk)] = (double)acc[i];
  __syncthreads();
  if (grp == 0) {
    // column c0 + gt / (TR / 4), rows r0 + 4 (gt % (TR / 4)) .. + 3
    const int cc = c0 + gt / (TR / 4);
    if (cc < R) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = 4 * (gt % (TR / 4)) + q;
        const int e = (gt / (TR / 4)) * (TR + 1) + rr;
        double s = Cs[0][e];
#pragma unroll
        for (int g2 = 1; g2 < GSPLIT; ++g2) s += Cs[g2][e];
        const size_t o = (size_t)cc * Np + r0 + rr;
        out[o] = (add ? add[o] : 0.0) + sgn * s;
      }
    }
  }
}

// -------------------------------------------------------------------------------------
// gamma = d mu / d alpha and (1/2) H gamma for a pair of columns (eq. (G)):
// spectrum of mu_a + i mu_b, gamma_hat = i k mu_hat, (H gamma)_hat = |k| mu_hat
// (both zero at k = 0 and at Nyquist).  Rows N..Np-1 of the outputs are zero.
// Dynamic LDS: 4 N complex (three work buffers and the twiddles).
// -------------------------------------------------------------------------------------
__device__ inline void refine_check_col(const double* __restrict__ rc, const double* __restrict__ bc, int N,
                                        double tol, int* __restrict__ status, int flag);

__global__ __launch_bounds__(WW_NT) void k_gamma(const double* __restrict__ Mu, int Np, int ncols,
                                                 double* __restrict__ Gam, double* __restrict__ HG,
                                                 const cplx* __restrict__ tw, int N,
                                                 const double* __restrict__ chk_r, const double* __restrict__ chk_b,
                                                 double chk_tol, int* __restrict__ status, int chk_flag) {
  // the refinement test of the solve that produced Mu's first column, when chk_r is
  // given (the check kernel's work, folded into this launch)
  if (chk_r && blockIdx.x == 0) refine_check_col(chk_r, chk_b, N, chk_tol, status, chk_flag);
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
  {
    double va[NPT], vb[NPT];
    gload(va, Mu + (size_t)ca * Np, N);
    gload(vb, Mu + (size_t)(hasb ? cb : ca) * Np, N);
    pin(va);
    pin(vb);
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      if (t < N) Z[t] = cmk(va[m], hasb ? vb[m] : 0.0);
    }
  }
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
  if (hasb) fft_lds(S, Z, tws, P, +1);
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
// Base DtN output of a lagged-factor stage in one launch (eq. (G)): every workgroup
// forms gamma = d mu/d alpha and (1/2) H gamma of the base density mu in LDS (one
// forward and one inverse FFT of its own), then, for its rows i (one wave per row),
//   G phi_i = (1/2) H gamma_i + sum_j Gm_ij gamma_j          (row-major Gm)
//   r_i     = psi_i - sum_j A_ij mu_j                          (row-major A)
// the FP64 residual of the refined solve.  The convergence test of that solve
// (max |r| <= tol max |psi|) needs both maxima over all rows: each wave folds its own
// into chk[0] = max |r|, chk[1] = max |psi| with an atomic maximum on the bit patterns
// (non-negative doubles order like their bits; a NaN residual is larger than any
// finite one), and the next kernel on the stream (k_base_rhs) takes the decision and
// clears chk.  Rows N..Np-1 of Gphi are zero.  Dynamic LDS: 4 N complex.  A workgroup
// takes `rows` consecutive rows (a multiple of 4; grid ceil(Np / rows)).
// -------------------------------------------------------------------------------------
// NR: entries of a row per lane, N <= 64 NR (16 up to N = 1024, 32 above), so that the
// row prefetch holds no more registers than the grid needs.
template <int NR>
__global__ __launch_bounds__(WW_NT) void k_base_dtn(const double* __restrict__ mu, const double* __restrict__ psi,
                                                    const double* __restrict__ Gmr, const double* __restrict__ Ar,
                                                    int Np, const cplx* __restrict__ tw, int N,
                                                    double* __restrict__ Gphi,
                                                    unsigned long long* __restrict__ chk, int rows) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* tws = lds + 2 * N;
  double* xs = reinterpret_cast<double*>(lds + 3 * N);   // mu (N doubles)
  double* gs = xs + N;                                   // gamma (N doubles)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  // a row's entries of Gm and A, all in flight at once (clamped, unconditional loads);
  // the first row's loads are issued before the transforms, which they do not need
  double gv[NR], av[NR];
  auto load_row = [&](int row) {
    const int rr = row < N ? row : N - 1;
    const double* gr = Gmr + (size_t)rr * Np;
    const double* ar = Ar + (size_t)rr * Np;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const int j = lane + 64 * m;
      const int jj = j < N ? j : N - 1;
      gv[m] = gr[jj];
      av[m] = ar[jj];
    }
  };
  const int row0 = blockIdx.x * rows + wv;
  load_row(row0);
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  {
    double va[NPT];
    gload(va, mu, N);
    pin(va);
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      if (t < N) {
        Z[t] = cmk(va[m], 0.0);
        xs[t] = va[m];
      }
    }
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    const int k = wavenum(t, N);
    const double hk = (k == 0 || 2 * k == N || 2 * k == -N) ? 0.0 : 0.5 * fabs((double)k);
    // Z holds the spectrum of the real signal mu: gamma_hat = i k mu_hat, (H gamma / 2)_hat
    // = |k| mu_hat / 2; both real signals travel as one complex signal
    W[t] = pack_pair(sym_deriv(Z[t], k, N), cscale(Z[t], hk));
  }
  fft_lds(W, Z, tws, P, +1);
  for (int t = tid; t < N; t += WW_NT) gs[t] = W[t].x;
  __syncthreads();
  double mr = 0.0, mb = 0.0;
  for (int q = 0; q < rows / 4; ++q) {
    const int row = blockIdx.x * rows + q * 4 + wv;
    if (row >= Np) break;
    if (q > 0) load_row(row);
    if (row >= N) {
      if (lane == 0) Gphi[row] = 0.0;
      continue;
    }
    double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int m = 0; m < NR; m += 2) {
      const int j0 = lane + 64 * m, j1 = j0 + 64;
      if (j0 < N) {
        s0 = fma(gv[m], gs[j0], s0);
        t0 = fma(av[m], xs[j0], t0);
      }
      if (j1 < N) {
        s1 = fma(gv[m + 1], gs[j1], s1);
        t1 = fma(av[m + 1], xs[j1], t1);
      }
    }
    double s = s0 + s1, t = t0 + t1;
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_down(s, off, 64);
      t += __shfl_down(t, off, 64);
    }
    if (lane == 0) {
      Gphi[row] = W[row].y + s;
      const double r = psi[row] - t;
      mr = fmax(mr, fabs(r));
      if (r != r) mr = INFINITY;
      mb = fmax(mb, fabs(psi[row]));
    }
  }
  if (lane == 0 && chk) {
    atomicMax(chk, (unsigned long long)__double_as_longlong(mr));
    atomicMax(chk + 1, (unsigned long long)__double_as_longlong(mb));
  }
}

// The convergence test of a lagged-factor solve from the maxima left by k_base_dtn
// (one thread), then the maxima are cleared for the next stage.
__device__ __forceinline__ void lagged_check(unsigned long long* __restrict__ chk, double tol, int* __restrict__ status,
                                             int flag) {
  if (!chk || threadIdx.x != 0) return;
  const double mr = __longlong_as_double((long long)chk[0]);
  const double mb = __longlong_as_double((long long)chk[1]);
  if (!(mr <= tol * mb)) atomicOr(status, flag);
  chk[0] = 0ull;
  chk[1] = 0ull;
}

// -------------------------------------------------------------------------------------
// Base right-hand side (Sec. 2.1 eq. (ww), (uv:from:G)), one workgroup:
//   u = (varphi' - eta_x G phi)/(1 + eta_x^2),  v = (eta_x varphi' + G phi)/(1 + eta_x^2)
//   eta_t = G phi
//   varphi_t = P[v eta_t - u^2/2 - v^2/2 - g eta + tau d/dx(eta_x/sqrt(1 + eta_x^2))]
// both filtered; u, v, (1 + eta_x^2)^{3/2} are kept for the variational columns.
// -------------------------------------------------------------------------------------
// The right-hand side of one stage on LDS work buffers Z, W, S and the twiddles tws.
__device__ inline void base_rhs_stage(cplx* Z, cplx* W, cplx* S, const cplx* tws, const FftPlan& P,
                                      const double* __restrict__ Ys, const double* __restrict__ Gphi,
                                      double* __restrict__ aux, int nmax, double* __restrict__ Kout,
                                      const double* __restrict__ sig, int N, double g, double tau) {
  const int tid = threadIdx.x;
  {
    double exv[NPT], psv[NPT], Gv[NPT], etv[NPT];
    gload(exv, aux + AUX_EX * nmax, N);
    gload(psv, aux + AUX_PHS * nmax, N);
    gload(Gv, Gphi, N);
    gload(etv, Ys, N);
    pin(exv);
    pin(psv);
    pin(Gv);
    pin(etv);
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      if (t < N) {
        const double ex = exv[m], ps = psv[m], G = Gv[m];
        const double den = 1.0 + ex * ex;
        const double u = (ps - ex * G) / den;
        const double v = (ex * ps + G) / den;
        aux[AUX_U * nmax + t] = u;
        aux[AUX_V * nmax + t] = v;
        aux[AUX_W3 * nmax + t] = den * sqrt(den);
        Z[t] = cmk(G, v * G - 0.5 * u * u - 0.5 * v * v - g * etv[m]);
        S[t] = cmk(tau * ex / sqrt(den), 0.0);
      }
    }
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

__global__ __launch_bounds__(WW_NT) void k_base_rhs(const double* __restrict__ Ys, const double* __restrict__ Gphi,
                                                    double* __restrict__ aux, int nmax, double* __restrict__ Kout,
                                                    unsigned long long* __restrict__ chk, double chk_tol,
                                                    int* __restrict__ status,
                                                    const cplx* __restrict__ tw, const double* __restrict__ sig,
                                                    int N, double g, double tau) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  const int tid = threadIdx.x;
  lagged_check(chk, chk_tol, status, 32);
  load_twiddles(tws, tw, N);
  base_rhs_stage(Z, W, S, tws, P, Ys, Gphi, aux, nmax, Kout, sig, N, g, tau);
}

// The right-hand side of stage s and, in the same workgroup, the prep of stage s + 1
// (s + 1 < stages of the step): one launch and one twiddle load fewer on the march's
// critical path.  The prep reads K_s through global memory after a barrier.
__global__ __launch_bounds__(WW_NT) void k_base_rhs_prep(
    const double* __restrict__ Gphi, double* __restrict__ aux_cur, double* __restrict__ Kcur,
    unsigned long long* __restrict__ chk, double chk_tol, const double* __restrict__ sig, double g, double tau,
    const double* __restrict__ y, const double* __restrict__ K, double* __restrict__ Ys,
    const double* __restrict__ coef, int stage_next, size_t kstride, double* __restrict__ aux_next,
    double* __restrict__ rhs0, int Np, double hsurf, int nmax, const cplx* __restrict__ tw, int N,
    int* __restrict__ status) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  lagged_check(chk, chk_tol, status, 32);
  load_twiddles(tws, tw, N);
  base_rhs_stage(Z, W, S, tws, P, Ys, Gphi, aux_cur, nmax, Kcur, sig, N, g, tau);
  __syncthreads();   // K_s (global) and the LDS buffers are complete
  base_prep_stage(Z, W, S, tws, P, y, K, Ys, coef, stage_next, kstride, aux_next, nmax, rhs0, Np, N, hsurf, status);
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
    const double e = stage_combine(y[oe], K, kstride, oe, coef, stage);
    const double p = stage_combine(y[op], K, kstride, op, coef, stage);
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
  double ev[NPT], pv[NPT], vv[NPT];
  gload(ev, ye, N);
  gload(pv, yp, N);
  gload(vv, av, N);
  pin(ev);
  pin(pv);
  pin(vv);
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) Z[t] = cmk(pv[m] - vv[m] * ev[m], ev[m]);
  }
  double uv[NPT], gv[NPT], wv[NPT];   // in flight during pass 1
  gload(uv, au, N);
  gload(gv, gp, N);
  gload(wv, aw, N);
  pin(uv);
  pin(gv);
  pin(wv);
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    cplx A, B;
    split_pair(Z, t, N, A, B);
    const int k = wavenum(t, N);
    W[t] = pack_pair(sym_deriv(A, k, N), sym_deriv(B, k, N));
  }
  fft_lds(W, Z, tws, P, +1);
  // pass 2
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) {
      const double e = ev[m], u = uv[m], v = vv[m], G = gv[m];
      const double dpsi = W[t].x, deta = W[t].y;
      Z[t] = cmk(G, e * u);
      S[t] = cmk(-u * dpsi + v * G - g * e, -e * u * v + tau * deta / wv[m]);
    }
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
                                                    int N, int c0, int* __restrict__ status) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* tws = lds + 2 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  const int c = c0 + blockIdx.x;
  double* yc = y + (size_t)c * 2 * N;
  const int tid = threadIdx.x;
  {
    double ev[NPT], pv[NPT];
    stage_combine_vec(ev, y + (size_t)c * 2 * N, K + (size_t)c * 2 * N, kstride, 0, coef + COEF_B, nst, N);
    stage_combine_vec(pv, y + (size_t)c * 2 * N, K + (size_t)c * 2 * N, kstride, N, coef + COEF_B, nst, N);
    pin(ev);
    pin(pv);
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      if (t < N) Z[t] = cmk(ev[m], pv[m]);
    }
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) Z[t] = cscale(Z[t], sig[t]);
  fft_lds(Z, W, tws, P, +1);
  for (int t = tid; t < N; t += WW_NT) {
    yc[t] = Z[t].x;
    yc[N + t] = Z[t].y;
  }
  if (status && c == 0 && tid == 0) status[1] += 1;   // steps completed (with the base column)
}

// status word of a call: bits, step counter, first failing 16 step + stage
__global__ void k_status_reset(int* __restrict__ status) {
  if (threadIdx.x == 0) {
    status[0] = 0;
    status[1] = 0;
    status[2] = 0x7fffffff;
    // status[4..7]: the two maxima of the lagged-solve test (k_base_dtn, k_base_rhs)
    status[4] = status[5] = status[6] = status[7] = 0;
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

// f = r.r / 2 and, when d is given, df/dT = r.d (Sec. 3.2 eq. (dfdT) with d = dr/dT)
// into f[1]: one workgroup, FP64 wavefront reductions in a fixed order
__global__ __launch_bounds__(WW_NT) void k_objective(const double* __restrict__ r, int N, double* __restrict__ f,
                                                     const double* __restrict__ d) {
  __shared__ double red[2][WW_NT / 64];
  double s = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < N; i += WW_NT) {
    s += r[i] * r[i];
    if (d) t += r[i] * d[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    t += __shfl_down(t, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < WW_NT / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    f[0] = 0.5 * a;
    if (d) f[1] = b;
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

// =====================================================================================
// Discrete adjoint (Sec. 3.2 and App. B, discrete form): the exact transpose of the
// tangent march above.  For one right-hand-side operator L = S_F DF(Y) of a stage,
//   psidot = phidot - v etadot,  G = (H/2 + Gm) D A^{-1} psidot,
//   etadot_t = G - D(u etadot),
//   phidot_t = P[-D(u v etadot) - u D psidot + v G - g etadot + tau D(w3^{-1} D etadot)],
// the transpose, with D^T = -D, H^T = -H, P^T = P, S_F^T = S_F, is, for adjoint data
// (alpha, beta) of (etadot_t, phidot_t):
//   a = S_F alpha,  b = P S_F beta,  gt = a + v b,
//   psit = A^{-T} D (H gt / 2 - Gm^T gt) + D(u b),
//   etat = u D a + u v D b - g b + tau D(w3^{-1} D b) - v psit,   phit = psit.
// A^{-T} = (Z (I + X))^T = (I + X^T) Z^T with the stored block-triangular inverses.
// =====================================================================================

// adjoint stage, part 1 (one workgroup):  kappa = wb * mu + sum_{i > s} wa_i upsilon_i
// (the stage weights come from coef), then the spectral pieces of the transpose.
// Outputs (ld Np where noted): gt (Np, zero padded), hd = D(H gt / 2), e1, q.
__global__ __launch_bounds__(WW_NT) void k_adj_pre(const double* __restrict__ mu, const double* __restrict__ ups,
                                                   size_t ustride, const double* __restrict__ coef, int stage,
                                                   int nst, const double* __restrict__ saux, const cplx* __restrict__ tw,
                                                   const double* __restrict__ sig, int N, int Np, double g, double tau,
                                                   double* __restrict__ gt, double* __restrict__ hd,
                                                   double* __restrict__ e1, double* __restrict__ q) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  const int tid = threadIdx.x;
  const double* u = saux;
  const double* v = saux + N;
  const double* w3 = saux + 2 * N;
  // kappa_s = b_s dt mu + sum_{i > s} a_is dt upsilon_i
  const double wb = coef[COEF_B + stage];
  for (int t = tid; t < 2 * N; t += WW_NT) {
    double kv = wb * mu[t];
    for (int i = stage + 1; i < nst; ++i) kv += coef[i * 16 + stage] * ups[(size_t)i * ustride + t];
    if (t < N) Z[t].x = kv;
    else Z[t - N].y = kv;
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) {
    cplx Al, Be;
    split_pair(Z, t, N, Al, Be);
    const int k = wavenum(t, N);
    const double sg = sig[t];
    cplx a = cscale(Al, sg);
    cplx b = (k == 0) ? cmk(0.0, 0.0) : cscale(Be, sg);
    W[t] = pack_pair(a, b);
    S[t] = pack_pair(sym_deriv(a, k, N), sym_deriv(b, k, N));
  }
  fft_lds(W, Z, tws, P, +1);   // a + i b
  fft_lds(S, Z, tws, P, +1);   // D a + i D b
  // physical: gt = a + v b ; f1 = D b / w3 ; f2 = u b   (kept in registers between passes)
  double av[NPT], bv[NPT], dav[NPT], dbv[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tclamp(m, N);
    av[m] = W[t].x;
    bv[m] = W[t].y;
    dav[m] = S[t].x;
    dbv[m] = S[t].y;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) {
      const double gg = av[m] + v[t] * bv[m];
      Z[t] = cmk(gg, dbv[m] / w3[t]);
      S[t] = cmk(u[t] * bv[m], 0.0);
      gt[t] = gg;
    }
  }
  for (int t = N + tid; t < Np; t += WW_NT) gt[t] = 0.0;
  fft_lds(Z, W, tws, P, -1);
  fft_lds(S, W, tws, P, -1);
  {
    // split_pair reads the mirrored bin N - t of S, which another thread (or this
    // thread's next m) would overwrite: read everything first, write after a barrier
    cplx wo[NPT], so[NPT];
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tclamp(m, N);
      cplx Gh, F1, F2, dm;
      split_pair(Z, t, N, Gh, F1);
      split_pair(S, t, N, F2, dm);
      const int k = wavenum(t, N);
      // D(H gt / 2): symbol (i k)(-i sgn k)/2 = |k|/2, zero at Nyquist
      const double hk = (2 * k == N || 2 * k == -N) ? 0.0 : 0.5 * fabs((double)k);
      wo[m] = pack_pair(cscale(Gh, hk), sym_deriv(F1, k, N));
      so[m] = sym_deriv(F2, k, N);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      if (t < N) {
        W[t] = wo[m];
        S[t] = so[m];
      }
    }
  }
  fft_lds(W, Z, tws, P, +1);   // D(H gt/2) + i D f1
  fft_lds(S, Z, tws, P, +1);   // D f2
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) {
      const double uu = u[t], vv = v[t];
      hd[t] = W[t].x;
      e1[t] = uu * dav[m] + uu * vv * dbv[m] - g * bv[m] + tau * W[t].y;
      q[t] = S[t].x;
    }
  }
}

// adjoint stage, part 2 (one workgroup): zeta = hd - D(g2), g2 = Gm^T gt (ld Np);
// zeta padded with zeros to Np.
__global__ __launch_bounds__(WW_NT) void k_adj_mid(const double* __restrict__ g2, const double* __restrict__ hd,
                                                   const cplx* __restrict__ tw, int N, int Np,
                                                   double* __restrict__ zeta) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* tws = lds + 2 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = cmk(g2[t], 0.0);
  fft_lds(Z, W, tws, P, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = sym_deriv(Z[t], wavenum(t, N), N);
  fft_lds(Z, W, tws, P, +1);
  for (int t = threadIdx.x; t < Np; t += WW_NT) zeta[t] = (t < N) ? hd[t] - Z[t].x : 0.0;
}

// y = add + M^T x for one vector (M column-major, ld Np): y_i = sum_j M[j, i] x_j over
// j in the block range of the mode: 0 all; 1 blk(j) > blk(i) (transpose of the strictly
// lower X); 2 blk(j) <= blk(i) (transpose of the upper Z).  One wave per output.
__global__ __launch_bounds__(WW_NT) void k_gemv_t(const double* __restrict__ M, int Np, int mode,
                                                  const double* __restrict__ x, const double* __restrict__ add,
                                                  double* __restrict__ y) {
  const int wave = (blockIdx.x * WW_NT + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= Np) return;
  const int i = wave;
  const int bi = i / WW_TB;
  int lo = 0, hi = Np;
  if (mode == 1) lo = (bi + 1) * WW_TB;
  if (mode == 2) hi = (bi + 1) * WW_TB;
  const double* col = M + (size_t)i * Np;
  double s = 0.0;
  for (int j = lo + lane; j < hi; j += 64) s = fma(col[j], x[j], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[i] = (add ? add[i] : 0.0) + s;
}

// adjoint stage, part 3: psit = y + q;  upsilon = (e1 - v psit, psit)
__global__ void k_adj_post(const double* __restrict__ yv, const double* __restrict__ q, const double* __restrict__ e1,
                           const double* __restrict__ saux, int N, double* __restrict__ ups) {
  const double* v = saux + N;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < N; t += gridDim.x * blockDim.x) {
    const double ps = yv[t] + q[t];
    ups[t] = e1[t] - v[t] * ps;
    ups[N + t] = ps;
  }
}

// adjoint of the end of a step: lambda_n = mu + sum_s upsilon_s, then (for the step
// before) mu = S_F lambda.  One workgroup; first = 1 starts from lambda (no upsilon).
__global__ __launch_bounds__(WW_NT) void k_adj_step(double* __restrict__ lam, double* __restrict__ mu,
                                                    const double* __restrict__ ups, size_t ustride, int nst,
                                                    int first, const cplx* __restrict__ tw,
                                                    const double* __restrict__ sig, int N) {
  extern __shared__ cplx lds[];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* tws = lds + 2 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  for (int t = threadIdx.x; t < 2 * N; t += WW_NT) {
    double l = first ? lam[t] : mu[t];
    if (!first)
      for (int s = 0; s < nst; ++s) l += ups[(size_t)s * ustride + t];
    lam[t] = l;
    if (t < N) Z[t].x = l;
    else Z[t - N].y = l;
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = cscale(Z[t], sig[t]);
  fft_lds(Z, W, tws, P, +1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    mu[t] = Z[t].x;
    mu[N + t] = Z[t].y;
  }
}

// gradient: grad_k = <basis_k, lambda_0>  (one wave per parameter)
__global__ __launch_bounds__(WW_NT) void k_adj_grad(const double* __restrict__ basis, const double* __restrict__ lam,
                                                    int N, int M, double* __restrict__ grad) {
  const int k = (blockIdx.x * WW_NT + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= M) return;
  const double* bk = basis + (size_t)k * 2 * N;
  double s = 0.0;
  for (int t = lane; t < 2 * N; t += 64) s = fma(bk[t], lam[t], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) grad[k] = s;
}

// lambda at T/4: (0, w r)
__global__ void k_adj_seed(const double* __restrict__ r, int N, double* __restrict__ lam) {
  const double w = 1.0 / sqrt((double)N);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * N; t += gridDim.x * blockDim.x)
    lam[t] = (t < N) ? 0.0 : w * r[t - N];
}

// copy of the stage's u, v, (1 + eta_x^2)^{3/2} for the reverse sweep
__global__ void k_save_aux(const double* __restrict__ aux, int nmax, int N, double* __restrict__ saux) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < N; t += gridDim.x * blockDim.x) {
    saux[t] = aux[AUX_U * nmax + t];
    saux[N + t] = aux[AUX_V * nmax + t];
    saux[2 * N + t] = aux[AUX_W3 * nmax + t];
  }
}

// -------------------------------------------------------------------------------------
// Convergence test of a mixed-precision solve (one workgroup per column): with the
// FP64 residual r = B - A X of the final X, max|r| <= tol * max|B| over the N rows
// (a relative residual, which bounds the normwise backward error); a column that
// fails, or a NaN, sets status bit 4 (reported as WW_EREFINE).
// -------------------------------------------------------------------------------------
__device__ inline void refine_check_col(const double* __restrict__ rc, const double* __restrict__ bc, int N,
                                        double tol, int* __restrict__ status, int flag) {
  __shared__ double rr[WW_NT], rb[WW_NT];
  double mr = 0.0, mb = 0.0;
  for (int i = threadIdx.x; i < N; i += WW_NT) {
    mr = fmax(mr, fabs(rc[i]));
    mb = fmax(mb, fabs(bc[i]));
    if (rc[i] != rc[i]) mr = INFINITY;
  }
  rr[threadIdx.x] = mr;
  rb[threadIdx.x] = mb;
  __syncthreads();
  for (int off = WW_NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      rr[threadIdx.x] = fmax(rr[threadIdx.x], rr[threadIdx.x + off]);
      rb[threadIdx.x] = fmax(rb[threadIdx.x], rb[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(rr[0] <= tol * rb[0])) atomicOr(status, flag);
}

__global__ __launch_bounds__(WW_NT) void k_refine_check(const double* __restrict__ r, const double* __restrict__ B,
                                                        int Np, int N, double tol, int* __restrict__ status,
                                                        int flag) {
  refine_check_col(r + (size_t)blockIdx.x * Np, B + (size_t)blockIdx.x * Np, N, tol, status, flag);
}

// -------------------------------------------------------------------------------------
// Measurement stamp (not part of the method): one thread reads the GPU's constant-rate
// wall clock.  which = 0 keeps the start tick of a slot; which = 1 adds the ticks since
// that start to the slot's running sum and counts the interval.  Slots are
// [start, sum, count]; a slot is only touched by work on one stream, in order.
// -------------------------------------------------------------------------------------
__global__ void k_stamp(unsigned long long* __restrict__ st, int slot, int which) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long t = (unsigned long long)wall_clock64();
  unsigned long long* s = st + 3 * (size_t)slot;
  if (which == 0) {
    s[0] = t;
  } else {
    s[1] += t - s[0];
    s[2] += 1;
  }
}
