// gfx950 kernels of the non-uniform mesh x = xi(alpha) and the time segments
// (Wilkening & Yu, Sec. 2.2 eq. (xi), (rho:def)).  The state, the Jacobian columns and
// every per-point array hold values at x_j = xi(alpha_j) of the uniform alpha grid;
// spectral operators act in alpha, and x-derivatives are (1/E) d/dalpha, E = xi'.
// Used by the segmented march only; the uniform-grid kernels are unchanged.
#pragma once
#include "ww_kernels.hpp"

// per-point mesh tables, each nmax doubles at mesh + MESH_x * nmax
enum {
  MESH_XI = 0,   // x_j = xi(alpha_j)
  MESH_E,        // E = xi'
  MESH_EINV,     // 1 / E
  MESH_EP,       // E' = xi''
  MESH_COUNT
};

// The change of variables of eq. (xi): E = 1 - A (s - 3/8) with s = sin^4(alpha/2)
// (side 0: refined near x = pi) or cos^4(alpha/2) (side 1: refined near x = 0); 3/8 is
// the mean of s, so E has mean one and xi(2 pi) = 2 pi.  A = 8 (1 - rho)/(5 + 3 rho).
__device__ __forceinline__ void mesh_eval(double a, double A, int side, double* xi, double* E, double* Ep) {
  double sh, ch;
  sincos(0.5 * a, &sh, &ch);
  const double p = side == 0 ? sh : ch;   // sin(a/2) or cos(a/2)
  const double q = side == 0 ? ch : -sh;  // its derivative times 2
  const double p2 = p * p;
  if (E) *E = 1.0 - A * (p2 * p2 - 0.375);
  if (Ep) *Ep = -A * 2.0 * p2 * p * q;
  if (xi) {
    // int_0^a (s - 3/8) = -sin(a)/2 + sin(2a)/16 (side 0), sin(a)/2 + sin(2a)/16 (side 1)
    double s1, c1;
    sincos(a, &s1, &c1);
    const double s2 = 2.0 * s1 * c1;
    *xi = a - A * ((side == 0 ? -0.5 : 0.5) * s1 + 0.0625 * s2);
  }
}

__global__ void k_mesh_tables(double* __restrict__ mesh, int nmax, int N, double A, int side) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const double a = 2.0 * M_PI * (double)j / (double)N;
    double xi, E, Ep;
    mesh_eval(a, A, side, &xi, &E, &Ep);
    mesh[MESH_XI * nmax + j] = xi;
    mesh[MESH_E * nmax + j] = E;
    mesh[MESH_EINV * nmax + j] = 1.0 / E;
    mesh[MESH_EP * nmax + j] = Ep;
  }
}

// -------------------------------------------------------------------------------------
// Assembly on the mapped grid (eq. (K1K2) for the curve zeta = xi + i eta):
//   zeta' = E + i eta_alpha,  zeta'' = E' + i eta_alphaalpha,  x_ij = xi_i - xi_j
//   C = cot((zeta_i - zeta_j)/2):  K1 = Im{zeta'_j C}/2 = (E_j Im C + eta'_j Re C)/2
//                                  G1 = Re{zeta'_i C}/2 - cot((alpha_i - alpha_j)/2)/2
//   diagonal: zeta''/zeta' = (E' + i eta'')(E - i eta')/(E^2 + eta'^2)
//   finite depth: D = cot((zeta_i - conj zeta_j)/2), K -= Im{conj(zeta'_j) D}/2,
//                 G -= Re{zeta'_i D}/2
// The regularising cot((alpha_i - alpha_j)/2)/2 stays on the uniform alpha grid (the
// circulant table).  cos x_ij and sin x_ij are evaluated per entry.  One strip of 64
// rows x 16 columns per workgroup (grid Np/64 x Np/16); writes what k_assemble writes.
// With a lagged inverse (Mx64 or Mx32, row-major) 16 more rows of workgroups form
// x0 = Mx psi, the first solve of the lagged-factor base chain, one wave per row.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_assemble_map(const double* __restrict__ aux, const double* __restrict__ mesh,
                                                        int nmax, const double* __restrict__ c0T,
                                                        double* __restrict__ A, double* __restrict__ Gm,
                                                        float* __restrict__ A32, double* __restrict__ Gmr,
                                                        double* __restrict__ Ar, int N, int Np, int finite,
                                                        const double* __restrict__ Mx64, const float* __restrict__ Mx32,
                                                        const double* __restrict__ psi, double* __restrict__ x0) {
  constexpr int CW = 16;
  if (blockIdx.y >= (unsigned)(Np / CW)) {
    // (uniform per workgroup: no barrier below is reached by these blocks)
    const int g = (blockIdx.y - Np / CW) * gridDim.x + blockIdx.x;
    const int row = g * (WW_NT / 64) + (threadIdx.x >> 6);
    if (row >= Np) return;
    if (Mx32)
      gemv_row_wave<float>(Mx32, Np, 0, psi, nullptr, 1.0, x0, row, threadIdx.x & 63);
    else if (Mx64)
      gemv_row_wave<double>(Mx64, Np, 0, psi, nullptr, 1.0, x0, row, threadIdx.x & 63);
    return;
  }
  __shared__ double rt[WW_TB][CW + 1];
  __shared__ double rq[7][WW_TB];   // eta', eta'', exp(s), exp(-s), xi, E, E' of the rows
  __shared__ double cq[5][CW];      // eta', exp(s), exp(-s), xi, E of the columns
  __shared__ double c0s[WW_TB + CW];
  const int i0 = blockIdx.x * WW_TB, j0 = blockIdx.y * CW;
  const int t = threadIdx.x;
  for (int e = t; e < 7 * WW_TB; e += WW_NT) {
    const int q = e / WW_TB, r = e - q * WW_TB, ir = i0 + r;
    const double* src = q == 0 ? aux + AUX_EX * nmax
                        : q == 1 ? aux + AUX_EXX * nmax
                        : q == 2 ? aux + AUX_EP * nmax
                        : q == 3 ? aux + AUX_EM * nmax
                        : q == 4 ? mesh + MESH_XI * nmax
                        : q == 5 ? mesh + MESH_E * nmax
                                 : mesh + MESH_EP * nmax;
    rq[q][r] = ir < N ? src[ir] : 0.0;
  }
  for (int e = t; e < 5 * CW; e += WW_NT) {
    const int q = e / CW, r = e - q * CW, jc = j0 + r;
    const double* src = q == 0 ? aux + AUX_EX * nmax
                        : q == 1 ? aux + AUX_EP * nmax
                        : q == 2 ? aux + AUX_EM * nmax
                        : q == 3 ? mesh + MESH_XI * nmax
                                 : mesh + MESH_E * nmax;
    cq[q][r] = jc < N ? src[jc] : 0.0;
  }
  for (int e = t; e < WW_TB + CW - 1; e += WW_NT) {
    int d = (i0 - j0 - (CW - 1) + e) % N;
    if (d < 0) d += N;
    c0s[e] = c0T[d];
  }
  __syncthreads();
  const int tx = t & 63, ty = t >> 6;
  const int i = i0 + tx;
  const double invN = 1.0 / (double)N;
  const double exi = rq[0][tx], exxi = rq[1][tx], epi = rq[2][tx], emi = rq[3][tx];
  const double xii = rq[4][tx], Ei = rq[5][tx], Epi = rq[6][tx];
  for (int jj = ty; jj < CW; jj += 4) {
    const int j = j0 + jj;
    double a, gm;
    if (i >= N || j >= N) {
      a = (i == j) ? 1.0 : 0.0;
      gm = 0.0;
    } else {
      const double exj = cq[0][jj], epj = cq[1][jj], emj = cq[2][jj], Ej = cq[4][jj];
      double sx, cx;
      sincos(xii - cq[3][jj], &sx, &cx);
      double Kv, Gv;
      if (i != j) {
        const double e1 = epi * emj, e2 = emi * epj;
        const double chy = 0.5 * (e1 + e2), shy = 0.5 * (e1 - e2);
        double cre, cim;
        cot_half_branch(cx, sx, chy, shy, cre, cim);
        Kv = 0.5 * (Ej * cim + exj * cre);
        Gv = 0.5 * (Ei * cre - exi * cim) - c0s[tx - jj + (CW - 1)];
      } else {
        const double den = 1.0 / (Ei * Ei + exi * exi);
        Kv = -0.5 * (exxi * Ei - Epi * exi) * den;
        Gv = 0.5 * (Epi * Ei + exxi * exi) * den;
      }
      if (finite) {
        const double e1 = epi * epj, e2 = emi * emj;
        const double chy = 0.5 * (e1 + e2), shy = 0.5 * (e1 - e2);
        double dre, dim;
        cot_half_branch(cx, sx, chy, shy, dre, dim);
        Kv -= 0.5 * (Ej * dim - exj * dre);
        Gv -= 0.5 * (Ei * dre - exi * dim);
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
  __syncthreads();
  for (int idx = t; idx < WW_TB * CW; idx += WW_NT) {
    const int r = idx / CW, cc = idx % CW;
    Gmr[(size_t)(i0 + r) * Np + j0 + cc] = rt[r][cc];
  }
  if (!Ar) return;
  __syncthreads();
  for (int jj = ty; jj < CW; jj += 4) rt[tx][jj] = A[(size_t)(j0 + jj) * Np + i];
  __syncthreads();
  for (int idx = t; idx < WW_TB * CW; idx += WW_NT) {
    const int r = idx / CW, cc = idx % CW;
    Ar[(size_t)(i0 + r) * Np + j0 + cc] = rt[r][cc];
  }
}

// Sum over the workgroup of one value per thread, in a fixed order (each wave by
// shuffles, then the four wave sums in turn); every thread receives the sum.
__device__ inline double block_sum_fixed(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < WW_NT / 64; ++w) s += red[w];
  return s;
}

// -------------------------------------------------------------------------------------
// Base right-hand side on the mapped grid (one workgroup), eq. (ww), (uv:from:G):
//   eta_x = eta_alpha / E,  varphi' = varphi_alpha / E,  G phi = (H gamma/2 + Gm gamma)/E
//   u, v as on the uniform grid; eta_t = G phi
//   varphi_t = P[v eta_t - u^2/2 - v^2/2 - g eta + tau (1/E) d/dalpha(eta_x/sqrt(1 + eta_x^2))]
// with P the zero-mean projection in x (the E-weighted mean removed), then both
// filtered in alpha.  Gphi holds H gamma/2 + Gm gamma (without the 1/E).
// Dynamic LDS: 4 N complex.
// -------------------------------------------------------------------------------------
// The right-hand side of one stage on LDS work buffers Z, W and the twiddles tws.
__device__ inline void base_rhs_map_stage(cplx* Z, cplx* W, const cplx* tws, const FftPlan& P, double* red,
                                          const double* __restrict__ Ys, const double* __restrict__ Gphi,
                                          double* __restrict__ aux, const double* __restrict__ mesh, int nmax,
                                          double* __restrict__ Kout, const double* __restrict__ sig, int N, double g,
                                          double tau) {
  const int tid = threadIdx.x;
  double Gv[NPT], pre[NPT], iv[NPT];
  {
    double exv[NPT], psv[NPT], etv[NPT];
    gload(exv, aux + AUX_EX * nmax, N);
    gload(psv, aux + AUX_PHS * nmax, N);
    gload(Gv, Gphi, N);
    gload(etv, Ys, N);
    gload(iv, mesh + MESH_EINV * nmax, N);
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      const double ex = exv[m] * iv[m], ps = psv[m] * iv[m];
      const double G = Gv[m] * iv[m];
      const double den = 1.0 + ex * ex;
      const double u = (ps - ex * G) / den;
      const double v = (ex * ps + G) / den;
      Gv[m] = G;
      pre[m] = v * G - 0.5 * u * u - 0.5 * v * v - g * etv[m];
      if (t < N) {
        aux[AUX_U * nmax + t] = u;
        aux[AUX_V * nmax + t] = v;
        aux[AUX_W3 * nmax + t] = den * sqrt(den);
        Z[t] = cmk(tau * ex / sqrt(den), 0.0);
      }
    }
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) W[t] = sym_deriv(Z[t], wavenum(t, N), N);
  fft_lds(W, Z, tws, P, +1);
  double ew[NPT];
  gload(ew, mesh + MESH_E * nmax, N);
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) {
      pre[m] += W[t].x * iv[m];
      s += ew[m] * pre[m];
    }
  }
  const double mean = block_sum_fixed(s, red) / (double)N;
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) Z[t] = cmk(Gv[m], pre[m] - mean);
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) Z[t] = cscale(Z[t], sig[t]);
  fft_lds(Z, W, tws, P, +1);
  for (int t = tid; t < N; t += WW_NT) {
    Kout[t] = Z[t].x;
    Kout[N + t] = Z[t].y;
  }
}

// chk (optional): the two maxima of a lagged-factor solve's test (see k_base_dtn)
__global__ __launch_bounds__(WW_NT) void k_base_rhs_map(const double* __restrict__ Ys, const double* __restrict__ Gphi,
                                                        double* __restrict__ aux, const double* __restrict__ mesh,
                                                        int nmax, double* __restrict__ Kout,
                                                        unsigned long long* __restrict__ chk, double chk_tol,
                                                        int* __restrict__ status, const cplx* __restrict__ tw,
                                                        const double* __restrict__ sig, int N, double g, double tau) {
  extern __shared__ cplx lds[];
  __shared__ double red[WW_NT / 64];
  const FftPlan P = make_plan(N);
  lagged_check(chk, chk_tol, status, 32);
  load_twiddles(lds + 3 * N, tw, N);
  base_rhs_map_stage(lds, lds + N, lds + 3 * N, P, red, Ys, Gphi, aux, mesh, nmax, Kout, sig, N, g, tau);
}

// The right-hand side of stage s and the prep of stage s + 1 in one launch (the mapped
// counterpart of k_base_rhs_prep).
__global__ __launch_bounds__(WW_NT) void k_base_rhs_prep_map(
    const double* __restrict__ Gphi, double* __restrict__ aux_cur, double* __restrict__ Kcur,
    unsigned long long* __restrict__ chk, double chk_tol, const double* __restrict__ sig, double g, double tau,
    const double* __restrict__ y, const double* __restrict__ K, double* __restrict__ Ys,
    const double* __restrict__ coef, int stage_next, size_t kstride, double* __restrict__ aux_next,
    double* __restrict__ rhs0, int Np, double hsurf, int nmax, const cplx* __restrict__ tw, int N,
    int* __restrict__ status, const double* __restrict__ mesh) {
  extern __shared__ cplx lds[];
  __shared__ double red[WW_NT / 64];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* S = lds + 2 * N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  lagged_check(chk, chk_tol, status, 32);
  load_twiddles(tws, tw, N);
  base_rhs_map_stage(Z, W, tws, P, red, Ys, Gphi, aux_cur, mesh, nmax, Kcur, sig, N, g, tau);
  __syncthreads();   // K_s (global) and the LDS buffers are complete
  base_prep_stage(Z, W, S, tws, P, y, K, Ys, coef, stage_next, kstride, aux_next, nmax, rhs0, Np, N, hsurf, status);
}

// -------------------------------------------------------------------------------------
// Variational right-hand side on the mapped grid, one workgroup per column (App. B
// (l5a), (l6), (l6a) with d/dx = (1/E) d/dalpha and G psidot = Gpsi / E):
//   etadot_t = G psidot - (1/E) d(etadot u)
//   phidot_t = P[(1/E) d(-etadot u v + tau d_x etadot / (1 + eta_x^2)^{3/2})
//               - u d_x psidot + v G psidot - g etadot]
// P the E-weighted zero-mean projection, then both filtered in alpha.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_col_rhs_map(const double* __restrict__ Ys, const double* __restrict__ Gpsi,
                                                       int Np, const double* __restrict__ aux,
                                                       const double* __restrict__ mesh, int nmax,
                                                       double* __restrict__ Kout, const cplx* __restrict__ tw,
                                                       const double* __restrict__ sig, int N, double g, double tau) {
  extern __shared__ cplx lds[];
  __shared__ double red[WW_NT / 64];
  cplx* Z = lds;
  cplx* W = lds + N;
  cplx* tws = lds + 3 * N;
  const FftPlan P = make_plan(N);
  load_twiddles(tws, tw, N);
  const int c = blockIdx.x + 1;
  const int tid = threadIdx.x;
  const double* ye = Ys + (size_t)c * 2 * N;
  const double* yp = ye + N;
  double ev[NPT], vv[NPT], uv[NPT], gv[NPT], wv[NPT], iv[NPT];
  {
    double pv[NPT];
    gload(ev, ye, N);
    gload(pv, yp, N);
    gload(vv, aux + AUX_V * nmax, N);
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int t = tidx(m);
      if (t < N) Z[t] = cmk(pv[m] - vv[m] * ev[m], ev[m]);   // (psidot, etadot)
    }
  }
  gload(uv, aux + AUX_U * nmax, N);
  gload(gv, Gpsi + (size_t)(c - 1) * Np, N);
  gload(wv, aux + AUX_W3 * nmax, N);
  gload(iv, mesh + MESH_EINV * nmax, N);
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) W[t] = sym_deriv(Z[t], wavenum(t, N), N);
  fft_lds(W, Z, tws, P, +1);
  double dps[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    gv[m] *= iv[m];   // G psidot
    if (t < N) {
      dps[m] = W[t].x * iv[m];
      const double deta = W[t].y * iv[m];
      const double e = ev[m], u = uv[m];
      Z[t] = cmk(e * u, -e * u * vv[m] + tau * deta / wv[m]);
    } else {
      dps[m] = 0.0;
    }
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) W[t] = sym_deriv(Z[t], wavenum(t, N), N);
  fft_lds(W, Z, tws, P, +1);
  double ew[NPT], et[NPT], pre[NPT];
  gload(ew, mesh + MESH_E * nmax, N);
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    et[m] = pre[m] = 0.0;
    if (t < N) {
      const double e = ev[m], u = uv[m], G = gv[m];
      et[m] = G - W[t].x * iv[m];
      pre[m] = W[t].y * iv[m] - u * dps[m] + vv[m] * G - g * e;
      s += ew[m] * pre[m];
    }
  }
  const double mean = block_sum_fixed(s, red) / (double)N;
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int t = tidx(m);
    if (t < N) Z[t] = cmk(et[m], pre[m] - mean);
  }
  fft_lds(Z, W, tws, P, -1);
  for (int t = tid; t < N; t += WW_NT) Z[t] = cscale(Z[t], sig[t]);
  fft_lds(Z, W, tws, P, +1);
  double* ko = Kout + (size_t)c * 2 * N;
  for (int t = tid; t < N; t += WW_NT) {
    ko[t] = Z[t].x;
    ko[N + t] = Z[t].y;
  }
}

// Outputs on the mapped grid: w_i = sqrt(E_i / N), r = w varphi, J = w phidot,
// drdT = w varphi_t / 4 (eq. (f:phi), (Jik), (dfdT) with the mesh spacing).
__global__ void k_outputs_map(const double* __restrict__ y, const double* __restrict__ kT,
                              const double* __restrict__ mesh, int nmax, double* __restrict__ r,
                              double* __restrict__ J, double* __restrict__ drdT, int N, int M) {
  const double invN = 1.0 / (double)N;
  const size_t tot = (size_t)N * (M + 1);
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < tot; idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / N);
    const int i = (int)(idx - (size_t)c * N);
    const double w = sqrt(mesh[MESH_E * nmax + i] * invN);
    const double v = w * y[(size_t)c * 2 * N + N + i];
    if (c == 0) {
      r[i] = v;
      if (drdT && kT) drdT[i] = 0.25 * w * kT[N + i];
    } else if (J) {
      J[(size_t)(c - 1) * N + i] = v;
    }
  }
}

// -------------------------------------------------------------------------------------
// Regridding between segments: values at xi_o(alpha_m) (No points) carried to
// xi_n(alpha_j) (Nn points) by the trigonometric interpolant in alpha evaluated at
// beta_j = xi_o^{-1}(xi_n(alpha_j)).  W_jm = D(beta_j - alpha_m), D(t) = sin(No t/2)
// cos(t/2) / (No sin(t/2)) (even No; D(0) = 1), W row-major (ld No).
// One workgroup per row j; beta_j by Newton's method on xi_o, safeguarded by bisection
// in [x - 1, x + 1] (|xi_o(a) - a| <= 9 A / 16 < 1), at most 100 iterations.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_regrid_w(double* __restrict__ W, int Nn, int No, double An, int sn,
                                                    double Ao, int so) {
  __shared__ double beta_s;
  const int j = blockIdx.x;
  if (j >= Nn) return;   // uniform per workgroup
  if (threadIdx.x == 0) {
    double x;
    mesh_eval(2.0 * M_PI * (double)j / (double)Nn, An, sn, &x, nullptr, nullptr);
    double lo = x - 1.0, hi = x + 1.0, b = x;
    for (int it = 0; it < 100; ++it) {
      double xb, Eb;
      mesh_eval(b, Ao, so, &xb, &Eb, nullptr);
      const double f = xb - x;
      if (f == 0.0) break;
      if (f > 0.0)
        hi = b;
      else
        lo = b;
      double bn = b - f / Eb;
      if (!(bn > lo && bn < hi)) bn = 0.5 * (lo + hi);
      if (bn == b) break;
      b = bn;
    }
    beta_s = b;
  }
  __syncthreads();
  const double b = beta_s;
  const double two_pi = 2.0 * M_PI;
  for (int m = threadIdx.x; m < No; m += WW_NT) {
    double t = b - two_pi * (double)m / (double)No;
    if (t > M_PI) t -= two_pi;
    if (t <= -M_PI) t += two_pi;
    double s, c;
    sincos(0.5 * t, &s, &c);
    W[(size_t)j * No + m] = s == 0.0 ? 1.0 : sin(0.5 * (double)No * t) * c / ((double)No * s);
  }
}

// dst (Nn x ncols, ld Nn) = W (Nn x No, row-major) src (No x ncols, ld No): 64 x 64
// output tiles, 4 x 4 per thread, inner index in chunks of 32 through LDS, summed in
// increasing order.
__global__ __launch_bounds__(WW_NT) void k_regrid_apply(const double* __restrict__ W, const double* __restrict__ src,
                                                        double* __restrict__ dst, int Nn, int No, int ncols) {
  __shared__ double Ws[64][33];
  __shared__ double Ss[32][65];
  const int j0 = blockIdx.x * 64, q0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int m0 = 0; m0 < No; m0 += 32) {
    for (int e = threadIdx.x; e < 64 * 32; e += WW_NT) {
      const int r = e >> 5, k = e & 31;
      const int j = j0 + r, m = m0 + k;
      Ws[r][k] = (j < Nn && m < No) ? W[(size_t)j * No + m] : 0.0;
    }
    for (int e = threadIdx.x; e < 32 * 64; e += WW_NT) {
      const int k = e & 31, cc = e >> 5;
      const int m = m0 + k, q = q0 + cc;
      Ss[k][cc] = (m < No && q < ncols) ? src[(size_t)q * No + m] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) {
      double wv[4], sv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) wv[a] = Ws[ty * 4 + a][k];
#pragma unroll
      for (int b = 0; b < 4; ++b) sv[b] = Ss[k][tx * 4 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(wv[a], sv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int j = j0 + ty * 4 + a;
    if (j >= Nn) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int q = q0 + tx * 4 + b;
      if (q < ncols) dst[(size_t)q * Nn + j] = acc[a][b];
    }
  }
}
