// LDS-resident complex FP64 FFT for one workgroup, N = 2^a 3^b <= WW_NMAX.
//
// Used for every pseudo-spectral operation of the method (Sec. 2.2: d/dx, Hilbert
// transform, zero-mean projection P and the 36th-order filter are all Fourier
// multipliers).  Real signals are processed in pairs packed as one complex signal.
//
// Algorithm: Stockham autosort with radix 4, 3 and 2 passes, ping-pong between two
// LDS buffers; twiddles are read from an LDS copy of a host-computed table laid out
// pass by pass (load_twiddles, once per kernel).  Forward transform uses exp(-i k x); the inverse
// uses exp(+i k x) and scales by 1/N.
#pragma once
#include <hip/hip_runtime.h>

#ifndef WW_NMAX
#define WW_NMAX 2048
#endif

struct __attribute__((aligned(16))) cplx {
  double x, y;
};

__device__ __forceinline__ cplx cmk(double a, double b) { return cplx{a, b}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.x * s, a.y * s}; }
__device__ __forceinline__ cplx cconj(cplx a) { return cplx{a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse): dir = -1 forward, +1 inverse
__device__ __forceinline__ cplx cmul_i(cplx a, int dir) {
  return dir < 0 ? cplx{a.y, -a.x} : cplx{-a.y, a.x};
}

// Plan: N = 4^n4 3^n3 2^n2; passes run radix 4 first, then 3, then 2.  Stored as
// counts (no per-pass array) so that nothing is indexed dynamically in registers.
struct FftPlan {
  int n, n4, n3, n2;
};

__host__ __device__ inline FftPlan make_plan(int n) {
  FftPlan p;
  p.n = n;
  p.n4 = p.n3 = p.n2 = 0;
  int m = n;
  while (m % 4 == 0) { ++p.n4; m /= 4; }
  while (m % 3 == 0) { ++p.n3; m /= 3; }
  while (m % 2 == 0) { ++p.n2; m /= 2; }
  if (m != 1) p.n4 = -1;
  return p;
}

// One Stockham pass of radix R (fully unrolled butterfly, static register arrays).
// lgNs >= 0: Ns = 2^lgNs, so the index split j -> (j / Ns, j % Ns) is a shift and a
// mask (the radix-4 passes, which run first); lgNs < 0: general Ns (integer division).
// Intermediate buffers between passes use the layout x -> x ^ ((x >> 3) & 7) (a
// permutation inside each aligned group of 8 elements, used when 8 | N): the strided
// writes of the first pass then hit distinct LDS bank groups.  The first pass reads and
// the last pass writes the natural layout.
__device__ __forceinline__ int fft_swz(int x, bool on) { return on ? (x ^ ((x >> 3) & 7)) : x; }

// Butterfly of radix R on v (twiddles already applied); dir = -1 forward, +1 inverse.
template <int R>
__device__ __forceinline__ void fft_bfly(cplx (&v)[R], int dir) {
  if (R == 2) {
    cplx t0 = cadd(v[0], v[1]);
    cplx t1 = csub(v[0], v[1]);
    v[0] = t0;
    v[1] = t1;
  } else if (R == 4) {
    cplx s02 = cadd(v[0], v[2 % R]);
    cplx d02 = csub(v[0], v[2 % R]);
    cplx s13 = cadd(v[1], v[3 % R]);
    cplx d13 = cmul_i(csub(v[1], v[3 % R]), dir);
    v[0] = cadd(s02, s13);
    v[2 % R] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3 % R] = csub(d02, d13);
  } else {  // R == 3
    const double c3 = -0.5;
    const double s3 = 0.86602540378443864676;  // sin(2 pi / 3)
    cplx sm = cadd(v[1], v[2 % R]);
    cplx d = csub(v[1], v[2 % R]);
    cplx m0 = cadd(v[0], cscale(sm, c3));
    // forward: exp(-2 pi i/3) -> multiply d by -i s3 ; inverse: +i s3
    cplx md = cscale(cmul_i(d, dir), s3);
    v[0] = cadd(v[0], sm);
    v[1] = cadd(m0, md);
    v[2 % R] = csub(m0, md);
  }
}

// Inputs of butterfly j of a pass: v[q] = src[j + q nb] times the pass twiddle.
// twp: this pass's twiddles, twp[(q - 1) Ns + jm] = exp(-2 pi i jm q / (Ns R)), so that
// neighbouring lanes read neighbouring entries.
template <int R>
__device__ __forceinline__ void fft_load(const cplx* src, const cplx* twp, int nb, int j, int jm, int Ns, int dir,
                                         bool rsw, cplx (&v)[R]) {
#pragma unroll
  for (int q = 0; q < R; ++q) {
    cplx x = src[fft_swz(j + q * nb, rsw)];
    if (q > 0) {
      cplx w = twp[(q - 1) * Ns + jm];
      if (dir > 0) w = cconj(w);
      x = cmul(x, w);
    }
    v[q] = x;
  }
}

// One Stockham pass src -> dst; outputs scaled by sc (the last pass of an inverse).
template <int R>
__device__ __forceinline__ void fft_pass(const cplx* src, cplx* dst, const cplx* twp, int N, int Ns, int dir,
                                         int lgNs, bool rsw, bool wsw, double sc) {
  const int nb = N / R;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    const int jq = lgNs >= 0 ? (j >> lgNs) : j / Ns;
    const int jm = j - jq * Ns;
    cplx v[R];
    fft_load<R>(src, twp, nb, j, jm, Ns, dir, rsw, v);
    fft_bfly<R>(v, dir);
    const int idxD = jq * Ns * R + jm;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[fft_swz(idxD + q * Ns, wsw)] = cscale(v[q], sc);
  }
}

// The same transform with N a compile-time power of two (the sizes up to WW_NMAX) and
// 256 threads: the passes are unrolled with their span, radix and layout flags as
// constants, so that the index arithmetic folds away; the last pass works in place
// (all of its inputs are read before a barrier, then written), which saves the copy of
// an odd pass count, and carries the 1/N of the inverse.  Same passes, same butterflies
// and the same twiddles as fft_lds, hence the same result.
template <int N, int R, int Ns>
__device__ __forceinline__ void fft_pass_fixed(const cplx* src, cplx* dst, const cplx* twp, int dir, bool rsw,
                                               bool wsw, bool inplace, double sc) {
  constexpr int nb = N / R;
  constexpr int per = (nb + 255) / 256;   // butterflies per thread
  cplx v[per][R];
#pragma unroll
  for (int u = 0; u < per; ++u) {
    const int j = threadIdx.x + 256 * u;
    if (j < nb) fft_load<R>(src, twp, nb, j, j & (Ns - 1), Ns, dir, rsw, v[u]);
  }
  if (inplace) __syncthreads();   // every input of the pass has been read
#pragma unroll
  for (int u = 0; u < per; ++u) {
    const int j = threadIdx.x + 256 * u;
    if (j < nb) {
      fft_bfly<R>(v[u], dir);
      const int jm = j & (Ns - 1);
      const int idxD = (j - jm) * R + jm;
#pragma unroll
      for (int q = 0; q < R; ++q) dst[fft_swz(idxD + q * Ns, wsw)] = sc == 1.0 ? v[u][q] : cscale(v[u][q], sc);
    }
  }
}

template <int N, int Ns>
__device__ __forceinline__ void fft_fixed_from(cplx* a, cplx* b, const cplx* tw, int dir, bool first) {
  if constexpr (Ns < N) {
    constexpr int R = (N / Ns) % 4 == 0 ? 4 : 2;
    constexpr bool last = Ns * R == N;
    constexpr bool sw = (N & 7) == 0;
    const cplx* twp = tw + (Ns - 1);
    // ping-pong a -> b -> a ...; the last pass lands in a (in place when it reads a)
    constexpr int p = __builtin_ctz(Ns) / 2;   // passes before this one (radix 4 first)
    const bool from_a = (p & 1) == 0;
    cplx* src = from_a ? a : b;
    cplx* dst = last ? a : (from_a ? b : a);
    const double sc = (last && dir > 0) ? 1.0 / (double)N : 1.0;
    fft_pass_fixed<N, R, Ns>(src, dst, twp, dir, sw && !first, sw && !last, last && from_a, sc);
    __syncthreads();
    fft_fixed_from<N, Ns * R>(a, b, tw, dir, false);
  }
}

template <int N>
__device__ __forceinline__ void fft_fixed(cplx* a, cplx* b, const cplx* tw, int dir) {
  __syncthreads();
  fft_fixed_from<N, 1>(a, b, tw, dir, true);
}

// Transform `a` (N complex in LDS) in place; `b` is LDS scratch of N complex.
// tw: twiddle table in LDS (load_twiddles) in pass order: the pass with radix R that
// starts at span Ns reads the N_s R - N_s entries from offset Ns - 1 (the offsets
// telescope: the table holds N - 1 entries).
// dir = -1 forward, +1 inverse (inverse also scales by 1/N).
// Must be called by all threads of the workgroup.  Ends with a barrier.
__device__ inline void fft_lds_general(cplx* a, cplx* b, const cplx* tw, const FftPlan& P, int dir) {
  const int N = P.n;
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  cplx* src = a;
  cplx* dst = b;
  int Ns = 1;
  __syncthreads();
  const int npass = P.n4 + P.n3 + P.n2;
  const bool sw = (N & 7) == 0;
  for (int ps = 0; ps < npass; ++ps) {
    const bool rsw = sw && ps > 0, wsw = sw && ps + 1 < npass;
    const cplx* twp = tw + (Ns - 1);
    if (ps < P.n4) {
      fft_pass<4>(src, dst, twp, N, Ns, dir, 2 * ps, rsw, wsw, 1.0);   // Ns = 4^ps
      Ns *= 4;
    } else if (ps < P.n4 + P.n3) {
      fft_pass<3>(src, dst, twp, N, Ns, dir, -1, rsw, wsw, 1.0);
      Ns *= 3;
    } else {
      fft_pass<2>(src, dst, twp, N, Ns, dir, -1, rsw, wsw, 1.0);
      Ns *= 2;
    }
    __syncthreads();
    cplx* t = src;
    src = dst;
    dst = t;
  }
  // result is in src; copy to a if needed and scale for the inverse
  const double sc = dir > 0 ? 1.0 / (double)N : 1.0;
  if (src != a) {
    for (int t = tid; t < N; t += nt) a[t] = cscale(src[t], sc);
  } else if (dir > 0) {
    for (int t = tid; t < N; t += nt) a[t] = cscale(a[t], sc);
  }
  __syncthreads();
}

// Power-of-two sizes with 256 threads take the unrolled passes, the others the general
// ones.
__device__ inline void fft_lds(cplx* a, cplx* b, const cplx* tw, const FftPlan& P, int dir) {
  if (blockDim.x == 256) {
    switch (P.n) {
      case 256: fft_fixed<256>(a, b, tw, dir); return;
      case 512: fft_fixed<512>(a, b, tw, dir); return;
      case 1024: fft_fixed<1024>(a, b, tw, dir); return;
      case 2048: fft_fixed<2048>(a, b, tw, dir); return;
      default: break;
    }
  }
  fft_lds_general(a, b, tw, P, dir);
}

// Copy the global twiddle table into LDS (once per kernel, before the first FFT).
__device__ inline void load_twiddles(cplx* tws, const cplx* __restrict__ twg, int N) {
  // clamped, unconditional loads first (all in flight), then the guarded LDS stores
  cplx v[WW_NMAX / 256];
#pragma unroll
  for (int m = 0; m < WW_NMAX / 256; ++m) {
    const int t = threadIdx.x + 256 * m;
    v[m] = twg[t < N ? t : N - 1];
  }
  // keep the loads here, all in flight, instead of sunk into the guarded stores below
#pragma unroll
  for (int m = 0; m < WW_NMAX / 256; ++m) asm volatile("" ::"v"(v[m].x), "v"(v[m].y));
#pragma unroll
  for (int m = 0; m < WW_NMAX / 256; ++m) {
    const int t = threadIdx.x + 256 * m;
    if (t < N) tws[t] = v[m];
  }
}

// Signed wavenumber of FFT bin t (t = 0..N-1): t for t <= N/2, t - N otherwise.
__device__ __forceinline__ int wavenum(int t, int N) { return t <= N / 2 ? t : t - N; }

// Split the spectrum Z of z = a + i b into the spectra of the real signals a and b:
// A_k = (Z_k + conj Z_{-k}) / 2,  B_k = (Z_k - conj Z_{-k}) / (2 i).
__device__ __forceinline__ void split_pair(const cplx* Z, int t, int N, cplx& A, cplx& B) {
  cplx zk = Z[t];
  cplx zm = cconj(Z[(N - t) % N]);
  A = cscale(cadd(zk, zm), 0.5);
  cplx d = csub(zk, zm);  // = 2 i B
  B = cplx{0.5 * d.y, -0.5 * d.x};
}

// Pack two Hermitian spectra C, D (of real signals c, d) as the spectrum of c + i d.
__device__ __forceinline__ cplx pack_pair(cplx C, cplx D) { return cplx{C.x - D.y, C.y + D.x}; }

// Fourier symbols (Sec. 2.2): derivative ik with the Nyquist mode set to zero, Hilbert
// -i sgn(k) (zero at 0 and Nyquist), and the 36th-order filter exp(-36 (|k|/(N/2))^36).
__device__ __forceinline__ cplx sym_deriv(cplx X, int k, int N) {
  if (2 * k == N || 2 * k == -N) return cplx{0.0, 0.0};
  return cplx{-(double)k * X.y, (double)k * X.x};
}
__device__ __forceinline__ cplx sym_hilbert(cplx X, int k, int N) {
  if (k == 0 || 2 * k == N || 2 * k == -N) return cplx{0.0, 0.0};
  return k > 0 ? cplx{X.y, -X.x} : cplx{-X.y, X.x};
}
