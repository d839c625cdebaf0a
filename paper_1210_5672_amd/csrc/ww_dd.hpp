// Double-double (about 32 significant digits) DtN evaluation on gfx950: the GPU part
// of the quadruple-precision workflow of Wilkening & Yu (Sec. 2.2 on quadruple
// precision, Sec. 3.3): the matrices of eq. (fred) and (G) assembled in double-double,
// residuals of the solve formed in double-double by matrix products, corrections from
// the FP64 factors of the leading part (iterative refinement), and the spectral steps
// (gamma = mu', H gamma) by double-double FFTs.
//
// A double-double value is the unevaluated sum hi + lo of two doubles with
// |lo| <= ulp(hi)/2.  Arithmetic: Knuth's two-sum, the exact product by fma, and the
// accurate addition and multiplication of Hida, Li & Bailey ("Algorithms for
// quad-double precision floating point arithmetic", 2001), relative error about 2^-104;
// division by three quotient digits.  Arrays are stored as separate hi and lo planes.
#pragma once
#include "ww_kernels.hpp"

// No contraction of a product into a later sum inside the primitives: the error-free
// transformations need every product and sum rounded on its own (a product fused into
// the sum of a two-sum loses the low part).
#define CONTRACT_OFF _Pragma("clang fp contract(off)")

struct dd {
  double hi, lo;
};
struct cdd {
  dd re, im;
};

__host__ __device__ inline dd dd_of(double a) { return dd{a, 0.0}; }
__host__ __device__ inline dd dd_two_sum(double a, double b) {
  CONTRACT_OFF
  const double s = a + b;
  const double bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ inline dd dd_quick(double a, double b) {   // |a| >= |b|
  CONTRACT_OFF
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__host__ __device__ inline dd dd_two_prod(double a, double b) {
  CONTRACT_OFF
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__host__ __device__ inline dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
__host__ __device__ inline dd dd_add(dd a, dd b) {
  CONTRACT_OFF
  dd s = dd_two_sum(a.hi, b.hi);
  const dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_quick(s.hi, s.lo);
  s.lo += t.lo;
  return dd_quick(s.hi, s.lo);
}
__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__host__ __device__ inline dd dd_add_d(dd a, double b) {
  CONTRACT_OFF
  dd s = dd_two_sum(a.hi, b);
  s.lo += a.lo;
  return dd_quick(s.hi, s.lo);
}
__host__ __device__ inline dd dd_mul(dd a, dd b) {
  CONTRACT_OFF
  dd p = dd_two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_quick(p.hi, p.lo);
}
__host__ __device__ inline dd dd_mul_d(dd a, double b) {
  CONTRACT_OFF
  dd p = dd_two_prod(a.hi, b);
  p.lo += a.lo * b;
  return dd_quick(p.hi, p.lo);
}
__host__ __device__ inline dd dd_div(dd a, dd b) {
  CONTRACT_OFF
  const double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  const double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  const double q3 = r.hi / b.hi;
  return dd_add_d(dd_quick(q1, q2), q3);
}
__host__ __device__ inline dd dd_div_d(dd a, double b) { return dd_div(a, dd_of(b)); }
__host__ __device__ inline dd dd_sqrt(dd a) {   // one Newton step from the double root
  CONTRACT_OFF
  if (!(a.hi > 0.0)) return dd_of(0.0);
  const double x = sqrt(a.hi);
  const dd r = dd_sub(a, dd_two_prod(x, x));
  return dd_add_d(dd_of(x), r.hi / (2.0 * x));
}
__host__ __device__ inline cdd cdd_add(cdd a, cdd b) { return cdd{dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__host__ __device__ inline cdd cdd_sub(cdd a, cdd b) { return cdd{dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; }
__host__ __device__ inline cdd cdd_mul(cdd a, cdd b) {
  return cdd{dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}

// pi and ln 2 as double-doubles (the standard hi/lo splits)
#define DD_PI_HI 3.141592653589793116e+00
#define DD_PI_LO 1.224646799147353207e-16
#define DD_LN2_HI 6.931471805599452862e-01
#define DD_LN2_LO 2.319046813846299558e-17

// exp in double-double: a = k ln2 + r, |r| <= ln2/2, exp(r) by its Taylor series to
// the term r^27/27! (below 1e-37 for |r| <= 0.35), times 2^k.  No squarings: they would
// multiply the rounding of the series.
__device__ inline dd dd_exp(dd a) {
  const double k = rint(a.hi / DD_LN2_HI);
  const dd ln2 = dd{DD_LN2_HI, DD_LN2_LO};
  const dd r = dd_sub(a, dd_mul_d(ln2, k));
  dd term = r, sum = dd_add_d(r, 1.0);
  for (int n = 2; n <= 27; ++n) {
    term = dd_div_d(dd_mul(term, r), (double)n);
    sum = dd_add(sum, term);
  }
  const int ki = (int)k;
  return dd{ldexp(sum.hi, ki), ldexp(sum.lo, ki)};
}

// cot((x + i y)/2) from cos x, sin x, cosh y, sinh y by the two-branch formula of
// Sec. 2.2 (as the FP64 assembly), in double-double
__device__ inline void dd_cot_half(dd cx, dd sx, dd chy, dd shy, dd& re, dd& im) {
  if (cx.hi >= 0.0) {
    const dd num = dd_add(cx, chy);
    const dd den = dd_add(dd_mul(sx, sx), dd_mul(shy, shy));
    re = dd_div(dd_mul(num, sx), den);
    im = dd_neg(dd_div(dd_mul(num, shy), den));
  } else {
    const dd den = dd_sub(chy, cx);
    re = dd_div(sx, den);
    im = dd_neg(dd_div(shy, den));
  }
}

// -------------------------------------------------------------------------------------
// Radix-2 Stockham FFT of N = 2^a complex double-doubles in LDS (one workgroup);
// a = data, b = scratch, tw[j] = exp(-2 pi i j / N) for j < N/2.  dir -1 forward, +1
// inverse (with the 1/N).  Result in a.  Ends with a barrier.
// -------------------------------------------------------------------------------------
__device__ inline void dd_fft(cdd* a, cdd* b, const cdd* tw, int N, int dir) {
  __syncthreads();
  cdd* src = a;
  cdd* dst = b;
  const int half = N / 2;
  for (int Ns = 1; Ns < N; Ns *= 2) {
    for (int j = threadIdx.x; j < half; j += blockDim.x) {
      const int jm = j % Ns;
      cdd w = tw[jm * (half / Ns)];
      if (dir > 0) w.im = dd_neg(w.im);
      const cdd u = src[j];
      const cdd v = cdd_mul(src[j + half], w);
      const int o = (j / Ns) * Ns * 2 + jm;
      dst[o] = cdd_add(u, v);
      dst[o + Ns] = cdd_sub(u, v);
    }
    __syncthreads();
    cdd* t = src;
    src = dst;
    dst = t;
  }
  const double sc = dir > 0 ? 1.0 / (double)N : 1.0;   // exact: N is a power of two
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    cdd v = src[t];
    if (dir > 0) v = cdd{dd{v.re.hi * sc, v.re.lo * sc}, dd{v.im.hi * sc, v.im.lo * sc}};
    a[t] = v;
  }
  __syncthreads();
}

// i k (with the Nyquist mode set to zero) times X
__device__ inline cdd dd_ik(cdd X, int k, int N) {
  if (2 * k == N || 2 * k == -N) return cdd{dd_of(0.0), dd_of(0.0)};
  const double kk = (double)k;
  return cdd{dd_neg(dd_mul_d(X.im, kk)), dd_mul_d(X.re, kk)};
}

// -------------------------------------------------------------------------------------
// Per-point quantities of a surface (one workgroup): eta' and eta'' (spectral, d/dx
// with the Nyquist mode set to zero, eta'' = d(eta')), exp(s) and exp(-s) of the
// surface height s (h + eta at finite depth, eta otherwise); domain (optional, finite
// depth): status bit 16 where s <= 0.  pt_hi / pt_lo: 4 planes
// of nmax values each: eta', eta'', exp(s), exp(-s).  Dynamic LDS: 3.5 N complex
// double-doubles (data, two scratch buffers, N/2 twiddles).
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_dd_prep(const double* __restrict__ eh, const double* __restrict__ el,
                                                   double hsurf, const cdd* __restrict__ twg, int N, int nmax,
                                                   double* __restrict__ pt_hi, double* __restrict__ pt_lo,
                                                   int* __restrict__ domain) {
  extern __shared__ cdd ldsd[];
  cdd* Z = ldsd;
  cdd* W = ldsd + N;
  cdd* S = ldsd + 2 * N;
  cdd* tw = ldsd + 3 * N;
  for (int t = threadIdx.x; t < N / 2; t += WW_NT) tw[t] = twg[t];
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = cdd{dd{eh[t], el ? el[t] : 0.0}, dd_of(0.0)};
  dd_fft(Z, W, tw, N, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    const int k = t <= N / 2 ? t : t - N;
    const cdd d1 = dd_ik(Z[t], k, N);
    W[t] = d1;
    S[t] = dd_ik(d1, k, N);
  }
  dd_fft(W, Z, tw, N, +1);   // eta'
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    pt_hi[t] = W[t].re.hi;
    pt_lo[t] = W[t].re.lo;
  }
  dd_fft(S, Z, tw, N, +1);   // eta''
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    pt_hi[nmax + t] = S[t].re.hi;
    pt_lo[nmax + t] = S[t].re.lo;
    const dd sh = dd_add_d(dd{eh[t], el ? el[t] : 0.0}, hsurf);
    if (domain && !(sh.hi > 0.0)) atomicOr(domain, 16);   // finite depth: h + eta > 0
    const dd ep = dd_exp(sh), em = dd_exp(dd_neg(sh));
    pt_hi[2 * nmax + t] = ep.hi;
    pt_lo[2 * nmax + t] = ep.lo;
    pt_hi[3 * nmax + t] = em.hi;
    pt_lo[3 * nmax + t] = em.lo;
  }
}

// -------------------------------------------------------------------------------------
// Assembly in double-double (eq. (K1K2), the same formulas as k_assemble): A = I/2 +
// K/N and Gm = G/N, column-major Np x Np, hi and lo planes; Af receives the leading
// part of A for the FP64 factorisation.  cos, sin (of 2 pi d/N) and cot(pi d/N)/2 come
// from double-double circulant tables (d = (i - j) mod N).  N is a power of two, so the
// scaling by 1/N is exact.  One strip of 64 rows x 16 columns per workgroup.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_dd_assemble(const double* __restrict__ pt_hi,
                                                       const double* __restrict__ pt_lo, int nmax,
                                                       const double* __restrict__ tab_hi,
                                                       const double* __restrict__ tab_lo, int N, int Np, int finite,
                                                       double* __restrict__ A_hi, double* __restrict__ A_lo,
                                                       double* __restrict__ G_hi, double* __restrict__ G_lo,
                                                       double* __restrict__ Af) {
  constexpr int CW = 16;
  const int i0 = blockIdx.x * WW_TB, j0 = blockIdx.y * CW;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int i = i0 + tx;
  const double sc = 1.0 / (double)N;
  const bool rin = i < N;
  const int ic = rin ? i : 0;
  const dd exi = dd{pt_hi[ic], pt_lo[ic]}, exxi = dd{pt_hi[nmax + ic], pt_lo[nmax + ic]};
  const dd epi = dd{pt_hi[2 * nmax + ic], pt_lo[2 * nmax + ic]};
  const dd emi = dd{pt_hi[3 * nmax + ic], pt_lo[3 * nmax + ic]};
  for (int jj = ty; jj < CW; jj += 4) {
    const int j = j0 + jj;
    dd a, gm;
    if (!rin || j >= N) {
      a = dd_of(i == j ? 1.0 : 0.0);
      gm = dd_of(0.0);
    } else {
      const dd exj = dd{pt_hi[j], pt_lo[j]};
      const dd epj = dd{pt_hi[2 * nmax + j], pt_lo[2 * nmax + j]};
      const dd emj = dd{pt_hi[3 * nmax + j], pt_lo[3 * nmax + j]};
      int d = (i - j) % N;
      if (d < 0) d += N;
      const dd cx = dd{tab_hi[d], tab_lo[d]}, sx = dd{tab_hi[N + d], tab_lo[N + d]};
      dd Kv, Gv;
      if (i != j) {
        const dd e1 = dd_mul(epi, emj), e2 = dd_mul(emi, epj);
        const dd s = dd_add(e1, e2), t = dd_sub(e1, e2);
        const dd chy = dd{0.5 * s.hi, 0.5 * s.lo}, shy = dd{0.5 * t.hi, 0.5 * t.lo};
        dd cre, cim;
        dd_cot_half(cx, sx, chy, shy, cre, cim);
        const dd k1 = dd_add(cim, dd_mul(exj, cre));
        const dd g1 = dd_sub(cre, dd_mul(exi, cim));
        Kv = dd{0.5 * k1.hi, 0.5 * k1.lo};
        Gv = dd_sub(dd{0.5 * g1.hi, 0.5 * g1.lo}, dd{tab_hi[2 * N + d], tab_lo[2 * N + d]});
      } else {
        const dd den = dd_add_d(dd_mul(exi, exi), 1.0);
        const dd q = dd_div(exxi, den);
        Kv = dd{-0.5 * q.hi, -0.5 * q.lo};
        const dd g = dd_mul(q, exi);
        Gv = dd{0.5 * g.hi, 0.5 * g.lo};
      }
      if (finite) {
        const dd e1 = dd_mul(epi, epj), e2 = dd_mul(emi, emj);
        const dd s = dd_add(e1, e2), t = dd_sub(e1, e2);
        const dd chy = dd{0.5 * s.hi, 0.5 * s.lo}, shy = dd{0.5 * t.hi, 0.5 * t.lo};
        dd dre, dim;
        dd_cot_half(cx, sx, chy, shy, dre, dim);
        const dd k2 = dd_sub(dim, dd_mul(exj, dre));
        const dd g2 = dd_sub(dre, dd_mul(exi, dim));
        Kv = dd_sub(Kv, dd{0.5 * k2.hi, 0.5 * k2.lo});
        Gv = dd_sub(Gv, dd{0.5 * g2.hi, 0.5 * g2.lo});
      }
      a = dd{Kv.hi * sc, Kv.lo * sc};
      if (i == j) a = dd_add_d(a, 0.5);
      gm = dd{Gv.hi * sc, Gv.lo * sc};
    }
    const size_t o = (size_t)j * Np + i;
    A_hi[o] = a.hi;
    A_lo[o] = a.lo;
    G_hi[o] = gm.hi;
    G_lo[o] = gm.lo;
    Af[o] = a.hi;
  }
}

// -------------------------------------------------------------------------------------
// out = add + sgn A B in double-double (the residual and the Gm Gamma products): A
// column-major Np x Np, B, add and out Np x ncols (ld Np), hi and lo planes; add may be
// null.  One workgroup per 64 rows x 4 columns; B in chunks of 64 rows through LDS;
// each output sums its terms in increasing inner index.
// -------------------------------------------------------------------------------------
__global__ __launch_bounds__(WW_NT) void k_dd_gemm(const double* __restrict__ A_hi, const double* __restrict__ A_lo,
                                                   int Np, const double* __restrict__ B_hi,
                                                   const double* __restrict__ B_lo, const double* __restrict__ add_hi,
                                                   const double* __restrict__ add_lo, double sgn,
                                                   double* __restrict__ out_hi, double* __restrict__ out_lo,
                                                   int ncols) {
  __shared__ double bh[64][4], bl[64][4];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int c = blockIdx.y * 4 + (threadIdx.x >> 6);
  dd acc = dd_of(0.0);
  for (int k0 = 0; k0 < Np; k0 += 64) {
    {
      const int kk = threadIdx.x & 63, cc = threadIdx.x >> 6;
      const int cg = blockIdx.y * 4 + cc;
      bh[kk][cc] = cg < ncols ? B_hi[(size_t)cg * Np + k0 + kk] : 0.0;
      bl[kk][cc] = cg < ncols ? B_lo[(size_t)cg * Np + k0 + kk] : 0.0;
    }
    __syncthreads();
    const int cc = threadIdx.x >> 6;
    for (int kk = 0; kk < 64; ++kk) {
      const size_t o = (size_t)(k0 + kk) * Np + i;
      acc = dd_add(acc, dd_mul(dd{A_hi[o], A_lo[o]}, dd{bh[kk][cc], bl[kk][cc]}));
    }
    __syncthreads();
  }
  if (c >= ncols) return;
  const size_t o = (size_t)c * Np + i;
  dd r = dd{sgn * acc.hi, sgn * acc.lo};
  if (add_hi) r = dd_add(dd{add_hi[o], add_lo[o]}, r);
  out_hi[o] = r.hi;
  out_lo[o] = r.lo;
}

// The one-column form of k_dd_gemm (one right-hand side: the double-double march), split
// over the inner index: chunk s = blockIdx.y of Np / gridDim.y indices, 64 rows per
// workgroup; thread (row r, lane q) sums A_ij x_j over j = j0 + q, j0 + q + 4, ... in
// increasing order, then the four lanes' partials in order q = 0..3 give P[s][i]
// (coalesced: the 64 rows of one column are consecutive)
#define DDGV_KS 16
__global__ __launch_bounds__(WW_NT) void k_dd_gemv_part(const double* __restrict__ A_hi,
                                                        const double* __restrict__ A_lo, int Np,
                                                        const double* __restrict__ x_hi,
                                                        const double* __restrict__ x_lo,
                                                        double* __restrict__ P_hi, double* __restrict__ P_lo) {
  __shared__ dd part[4][64];
  const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;
  const int len = Np / gridDim.y, j0 = blockIdx.y * len;
  dd acc = dd_of(0.0);
  for (int j = j0 + q; j < j0 + len; j += 4) {
    const size_t o = (size_t)j * Np + i;
    acc = dd_add(acc, dd_mul(dd{A_hi[o], A_lo[o]}, dd{x_hi[j], x_lo[j]}));
  }
  part[q][r] = acc;
  __syncthreads();
  if (q == 0) {
    dd t = part[0][r];
    for (int u = 1; u < 4; ++u) t = dd_add(t, part[u][r]);
    P_hi[(size_t)blockIdx.y * Np + i] = t.hi;
    P_lo[(size_t)blockIdx.y * Np + i] = t.lo;
  }
}
// out = add + sgn sum_s P[s] (chunks in increasing order); add may be null
__global__ void k_dd_gemv_sum(const double* __restrict__ P_hi, const double* __restrict__ P_lo, int ks, int Np,
                              const double* __restrict__ add_hi, const double* __restrict__ add_lo, double sgn,
                              double* __restrict__ out_hi, double* __restrict__ out_lo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Np) return;
  dd t = dd_of(0.0);
  for (int s = 0; s < ks; ++s) t = dd_add(t, dd{P_hi[(size_t)s * Np + i], P_lo[(size_t)s * Np + i]});
  if (sgn < 0.0) t = dd_neg(t);
  if (add_hi) t = dd_add(dd{add_hi[i], add_lo[i]}, t);
  out_hi[i] = t.hi;
  out_lo[i] = t.lo;
}

// the FP32 copy of the FP64 leading part of A (the mixed form factors it on MFMA)
__global__ void k_dd_a32(const double* __restrict__ A, float* __restrict__ A32, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    A32[e] = (float)A[e];
}

// mu += delta (double-double plus a double), n entries
__global__ void k_dd_correct(double* __restrict__ mu_hi, double* __restrict__ mu_lo, const double* __restrict__ delta,
                             size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const dd v = dd_add_d(dd{mu_hi[t], mu_lo[t]}, delta[t]);
    mu_hi[t] = v.hi;
    mu_lo[t] = v.lo;
  }
}

// gamma = d mu/dalpha and H gamma / 2 (spectrum |k| mu_hat / 2, zero at k = 0 and at
// Nyquist) of one column per workgroup, double-double; rows N..Np-1 zero.  Dynamic
// LDS: 3.5 N complex double-doubles.
__global__ __launch_bounds__(WW_NT) void k_dd_gamma(const double* __restrict__ mu_hi, const double* __restrict__ mu_lo,
                                                    int Np, const cdd* __restrict__ twg, int N,
                                                    double* __restrict__ g_hi, double* __restrict__ g_lo,
                                                    double* __restrict__ h_hi, double* __restrict__ h_lo) {
  extern __shared__ cdd ldsd[];
  cdd* Z = ldsd;
  cdd* W = ldsd + N;
  cdd* S = ldsd + 2 * N;
  cdd* tw = ldsd + 3 * N;
  const size_t off = (size_t)blockIdx.x * Np;
  for (int t = threadIdx.x; t < N / 2; t += WW_NT) tw[t] = twg[t];
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = cdd{dd{mu_hi[off + t], mu_lo[off + t]}, dd_of(0.0)};
  dd_fft(Z, W, tw, N, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    const int k = t <= N / 2 ? t : t - N;
    W[t] = dd_ik(Z[t], k, N);
    const double hk = (k == 0 || 2 * k == N || 2 * k == -N) ? 0.0 : 0.5 * fabs((double)k);
    S[t] = cdd{dd_mul_d(Z[t].re, hk), dd_mul_d(Z[t].im, hk)};
  }
  dd_fft(W, Z, tw, N, +1);
  dd_fft(S, Z, tw, N, +1);
  for (int t = threadIdx.x; t < Np; t += WW_NT) {
    const bool in = t < N;
    g_hi[off + t] = in ? W[t].re.hi : 0.0;
    g_lo[off + t] = in ? W[t].re.lo : 0.0;
    h_hi[off + t] = in ? S[t].re.hi : 0.0;
    h_lo[off + t] = in ? S[t].re.lo : 0.0;
  }
}

// the residual test of a double-double solve: status bit 4 unless max|r| <= tol max|b|
// (mx from k_dd_maxabs); mx is cleared for the next solve
__global__ void k_dd_restest(unsigned long long* __restrict__ mx, double tol, int* __restrict__ status) {
  if (threadIdx.x != 0) return;
  const double mr = __longlong_as_double((long long)mx[0]), mb = __longlong_as_double((long long)mx[1]);
  if (!(mr <= tol * mb)) atomicOr(status, 4);
  mx[0] = 0;
  mx[1] = 0;
}
__global__ void k_dd_mx_reset(unsigned long long* __restrict__ mx) {
  if (threadIdx.x == 0) mx[0] = mx[1] = 0;
}

// max |r| and max |b| over rows < N of ncols columns (ld Np) into mx[0], mx[1] by
// atomic maxima on the bit patterns (non-negative doubles order like their bits; a
// NaN residual counts as infinite)
__global__ void k_dd_maxabs(const double* __restrict__ r, const double* __restrict__ b, int N, int Np, int ncols,
                            unsigned long long* __restrict__ mx) {
  double mr = 0.0, mb = 0.0;
  const size_t tot = (size_t)Np * ncols;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    if ((int)(t % Np) >= N) continue;
    const double v = fabs(r[t]);
    mr = fmax(mr, v != v ? INFINITY : v);
    mb = fmax(mb, fabs(b[t]));
  }
  atomicMax(mx, (unsigned long long)__double_as_longlong(mr));
  atomicMax(mx + 1, (unsigned long long)__double_as_longlong(mb));
}

// =====================================================================================
// The base march in double-double (SDC15, the quadruple-precision workflow of Sec. 2.2):
// the right-hand side of eq. (ww) with the velocities of eq. (uv:from:G), the filter of
// eq. (filter) and the zero-mean projection, stage combinations and the outputs of eq.
// (f:phi) and (dfdT), every quantity a double-double.  States are 2N values [eta | phi]
// in hi and lo planes.
// =====================================================================================

// filter symbol exp(-36 (k / k_max)^36) for k = 0 .. N/2 (k_max = N/2, a power of two:
// k / k_max is exact; its 36th power by squarings in double-double)
__global__ void k_dd_filter_tab(int N, double* __restrict__ f_hi, double* __restrict__ f_lo) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > N / 2) return;
  const dd x = dd_of((double)k / (double)(N / 2));
  const dd x2 = dd_mul(x, x), x4 = dd_mul(x2, x2), x8 = dd_mul(x4, x4);
  const dd x16 = dd_mul(x8, x8), x32 = dd_mul(x16, x16);
  const dd e = dd_exp(dd_mul_d(dd_mul(x32, x4), -36.0));
  f_hi[k] = e.hi;
  f_lo[k] = e.lo;
}

__device__ inline dd dd_ld(const double* __restrict__ h, const double* __restrict__ l, int i) {
  return dd{h[i], l[i]};
}
__device__ inline void dd_st(double* __restrict__ h, double* __restrict__ l, int i, dd v) {
  h[i] = v.hi;
  l[i] = v.lo;
}
// the filter symbol of wavenumber index t (0 .. N-1)
__device__ inline dd dd_filt_at(const double* __restrict__ f_hi, const double* __restrict__ f_lo, int t, int N) {
  const int k = t <= N / 2 ? t : N - t;
  return dd{f_hi[k], f_lo[k]};
}

// out = y0 + sum_t w_t K_{j_t} over n entries (the weights carry dt), double-double, the
// terms added in increasing t
__global__ void k_dd_sdc_combine(const double* __restrict__ y0h, const double* __restrict__ y0l,
                                 const double* __restrict__ Kh, const double* __restrict__ Kl, size_t kstride,
                                 const int* __restrict__ jt, const double* __restrict__ wh,
                                 const double* __restrict__ wl, int cnt, double* __restrict__ oh,
                                 double* __restrict__ ol, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    dd acc = dd{y0h[e], y0l[e]};
    for (int t = 0; t < cnt; ++t) {
      const size_t o = (size_t)jt[t] * kstride + e;
      acc = dd_add(acc, dd_mul(dd{wh[t], wl[t]}, dd{Kh[o], Kl[o]}));
    }
    oh[e] = acc.hi;
    ol[e] = acc.lo;
  }
}

// The base right-hand side at the state y (one workgroup): eta' and phi' by one packed
// transform (both real, the multiplier i k is odd), G phi given (double-double DtN);
//   u = (phi' - eta' G)/(1 + eta'^2),  v = (eta' phi' + G)/(1 + eta'^2),
//   eta_t = G phi,  phi_t = P[v eta_t - u^2/2 - v^2/2 - g eta + tau d/dx(eta'/sqrt(1 + eta'^2))],
// both filtered by one packed transform (the filter is even and real; P zeroes the mean
// of phi_t only: the imaginary part of mode 0).  Dynamic LDS: 3.5 N complex
// double-doubles.
__global__ __launch_bounds__(WW_NT) void k_dd_base_rhs(const double* __restrict__ yh, const double* __restrict__ yl,
                                                       const double* __restrict__ gh, const double* __restrict__ gl,
                                                       const double* __restrict__ f_hi, const double* __restrict__ f_lo,
                                                       const cdd* __restrict__ twg, int N, double g, double tau,
                                                       double* __restrict__ kh, double* __restrict__ kl) {
  extern __shared__ cdd ldsd[];
  cdd* Z = ldsd;
  cdd* W = ldsd + N;
  cdd* S = ldsd + 2 * N;
  cdd* tw = ldsd + 3 * N;
  const dd zero = dd_of(0.0);
  for (int t = threadIdx.x; t < N / 2; t += WW_NT) tw[t] = twg[t];
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = cdd{dd_ld(yh, yl, t), dd_ld(yh, yl, N + t)};
  dd_fft(Z, W, tw, N, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = dd_ik(Z[t], t <= N / 2 ? t : t - N, N);
  dd_fft(Z, W, tw, N, +1);   // Z = eta' + i phi'
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    const dd ex = Z[t].re, ps = Z[t].im, G = dd_ld(gh, gl, t);
    const dd den = dd_add_d(dd_mul(ex, ex), 1.0);
    const dd u = dd_div(dd_sub(ps, dd_mul(ex, G)), den);
    const dd v = dd_div(dd_add(dd_mul(ex, ps), G), den);
    dd s = dd_sub(dd_mul(v, G), dd_mul_d(dd_add(dd_mul(u, u), dd_mul(v, v)), 0.5));
    s = dd_sub(s, dd_mul_d(dd_ld(yh, yl, t), g));
    W[t] = cdd{s, zero};
    S[t] = cdd{dd_div(ex, dd_sqrt(den)), zero};
  }
  dd_fft(S, Z, tw, N, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) S[t] = dd_ik(S[t], t <= N / 2 ? t : t - N, N);
  dd_fft(S, Z, tw, N, +1);   // S.re = d/dx(eta'/sqrt(1 + eta'^2))
  for (int t = threadIdx.x; t < N; t += WW_NT)
    Z[t] = cdd{dd_ld(gh, gl, t), dd_add(W[t].re, dd_mul_d(S[t].re, tau))};
  dd_fft(Z, W, tw, N, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    const dd f = dd_filt_at(f_hi, f_lo, t, N);
    cdd v = cdd{dd_mul(Z[t].re, f), dd_mul(Z[t].im, f)};
    if (t == 0) v.im = zero;   // P: the mean of phi_t
    Z[t] = v;
  }
  dd_fft(Z, W, tw, N, +1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    dd_st(kh, kl, t, Z[t].re);
    dd_st(kh, kl, N + t, Z[t].im);
  }
}

// the filter on the state after a step (eta and phi packed), in place
__global__ __launch_bounds__(WW_NT) void k_dd_filter_state(double* __restrict__ yh, double* __restrict__ yl,
                                                           const double* __restrict__ f_hi,
                                                           const double* __restrict__ f_lo, const cdd* __restrict__ twg,
                                                           int N) {
  extern __shared__ cdd ldsd[];
  cdd* Z = ldsd;
  cdd* W = ldsd + N;
  cdd* tw = ldsd + 3 * N;
  for (int t = threadIdx.x; t < N / 2; t += WW_NT) tw[t] = twg[t];
  for (int t = threadIdx.x; t < N; t += WW_NT) Z[t] = cdd{dd_ld(yh, yl, t), dd_ld(yh, yl, N + t)};
  dd_fft(Z, W, tw, N, -1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    const dd f = dd_filt_at(f_hi, f_lo, t, N);
    Z[t] = cdd{dd_mul(Z[t].re, f), dd_mul(Z[t].im, f)};
  }
  dd_fft(Z, W, tw, N, +1);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    dd_st(yh, yl, t, Z[t].re);
    dd_st(yh, yl, N + t, Z[t].im);
  }
}

// r = w phi, dr/dT = w phi_t / 4 (phi_t: the phi half of a right-hand side at the final
// state), f = r.r / 2 with w = 1/sqrt(N); one workgroup, the sum in a fixed order (each
// thread its strided terms in increasing index, then a tree over the threads)
__global__ __launch_bounds__(WW_NT) void k_dd_outputs(const double* __restrict__ yh, const double* __restrict__ yl,
                                                      const double* __restrict__ kh, const double* __restrict__ kl, int N,
                                                      double* __restrict__ rh, double* __restrict__ rl,
                                                      double* __restrict__ dh, double* __restrict__ dl,
                                                      double* __restrict__ fout) {
  __shared__ dd part[WW_NT];
  const dd w = dd_div(dd_of(1.0), dd_sqrt(dd_of((double)N)));
  dd acc = dd_of(0.0);
  for (int t = threadIdx.x; t < N; t += WW_NT) {
    const dd r = dd_mul(w, dd_ld(yh, yl, N + t));
    dd_st(rh, rl, t, r);
    if (dh) dd_st(dh, dl, t, dd_mul_d(dd_mul(w, dd_ld(kh, kl, N + t)), 0.25));
    acc = dd_add(acc, dd_mul(r, r));
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = WW_NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] = dd_add(part[threadIdx.x], part[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const dd f = dd_mul_d(part[0], 0.5);
    fout[0] = f.hi;
    fout[1] = f.lo;
  }
}
