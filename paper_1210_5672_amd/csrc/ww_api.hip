// Host side of the C ABI declared in include/ww.h: context and workspace, the
// per-stage kernel sequence, the march to T/4 and the outputs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ww.h"
#include "ww_kernels.hpp"

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail(WW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));             \
  } while (0)

#define LAUNCHCHK()                                                                      \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess)                                                                \
      return fail(WW_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_));     \
  } while (0)

struct ww_ctx {
  int dev = 0;
  hipStream_t stream = nullptr;
  unsigned flags = 0;
  int n_max = 0, r_max = 0, np_max = 0;
  // current discretisation
  int N = 0, Np = 0;
  int tables_N = 0;
  double h = INFINITY, hsurf = 0.0;
  int finite = 0;
  double tau = 0.0, g = 1.0;
  bool dtn_ready = false;
  // shooting problem (grid kept separately: dtn_setup may use another N)
  int M = -1;
  bool shoot_ready = false;
  int shootN = 0;
  double shootH = INFINITY;
  // tableau
  int nst = 0;
  double ta[16 * 16], tb[16];
  // device buffers
  double *A = nullptr, *Gm = nullptr, *Xi = nullptr, *Zi = nullptr, *Vi = nullptr, *Dinv = nullptr;
  float *A32 = nullptr, *X32 = nullptr, *Z32 = nullptr, *V32 = nullptr, *Dinv32 = nullptr;
  double *Rr = nullptr, *rr0 = nullptr;   // residuals of the refinement sweeps
  int nref = 2;                            // refinement sweeps per solve (mixed mode)
  double *cosT = nullptr, *sinT = nullptr, *c0T = nullptr, *sig = nullptr;
  cplx* tw = nullptr;
  double* aux = nullptr;
  double *rhs0 = nullptr, *y0t = nullptr, *mu0 = nullptr, *gam0 = nullptr, *hg0 = nullptr, *gphi0 = nullptr;
  double *Psi = nullptr, *Ytmp = nullptr, *Mu = nullptr, *Gam = nullptr, *HG = nullptr, *Gpsi = nullptr;
  double* part = nullptr;
  int nsplit_max = 0;
  double *y = nullptr, *Ys = nullptr, *K = nullptr, *Kx = nullptr, *ydtn = nullptr;
  double *basis = nullptr, *qfix = nullptr;
  double* coef = nullptr;
  double* fdev = nullptr;
  int* status = nullptr;
  std::vector<void*> allocs;
  // one RK step captured as a graph, replayed nsteps times
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t step_exec = nullptr;
  int gN = -1, gM = -1, gcols = -1, gnst = -1;
};

static bool valid_n(int N) {
  if (N < 16 || (N & 1)) return false;
  int m = N;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  return m == 1;
}

static int dalloc(ww_ctx* c, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 8);
  if (e != hipSuccess) return fail(WW_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocs.push_back(*p);
  return 0;
}

// circulant and spectral tables for grid size N (host-computed in double)
static int set_tables(ww_ctx* c, int N) {
  if (c->tables_N == N) return 0;
  std::vector<double> co(N), si(N), c0(N), sg(N);
  std::vector<cplx> tw(N);
  const double two_pi = 2.0 * M_PI;
  for (int d = 0; d < N; ++d) {
    const double x = two_pi * d / N;
    co[d] = std::cos(x);
    si[d] = std::sin(x);
    c0[d] = d == 0 ? 0.0 : 0.5 / std::tan(0.5 * x);
    tw[d] = cplx{std::cos(x), -std::sin(x)};
    const int k = d <= N / 2 ? d : N - d;
    sg[d] = std::exp(-36.0 * std::pow((double)k / (N / 2), 36.0));
  }
  HIPCHK(hipMemcpy(c->cosT, co.data(), N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->sinT, si.data(), N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->c0T, c0.data(), N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->sig, sg.data(), N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->tw, tw.data(), N * sizeof(cplx), hipMemcpyHostToDevice));
  c->tables_N = N;
  return 0;
}

static int set_grid(ww_ctx* c, int N, double h) {
  if (!valid_n(N) || N > c->n_max) return fail(WW_EINVAL, "N must be even, 2^a 3^b, 16 <= N <= n_max");
  c->N = N;
  c->Np = (N + WW_TB - 1) / WW_TB * WW_TB;
  c->finite = (std::isfinite(h) && h > 0.0) ? 1 : 0;
  c->h = c->finite ? h : INFINITY;
  c->hsurf = c->finite ? h : 0.0;
  return set_tables(c, N);
}

extern "C" {

const char* ww_last_error(void) { return g_err.c_str(); }

const char* ww_version(void) { return "wwdtn 0.1 gfx950"; }

int ww_create(ww_ctx** out, int n_max, int r_max, unsigned flags, void* hip_stream) {
  if (!out) return fail(WW_EINVAL, "ctx is null");
  *out = nullptr;
  if (!valid_n(n_max) || n_max > WW_NMAX) return fail(WW_EINVAL, "n_max must be even, 2^a 3^b, 16..2048");
  if (r_max < 1 || r_max > 4096) return fail(WW_EINVAL, "r_max out of range");
  if (flags & ~WW_MIXED) return fail(WW_EINVAL, "unknown flags");
  ww_ctx* c = new ww_ctx();
  HIPCHK(hipGetDevice(&c->dev));
  c->stream = (hipStream_t)hip_stream;
  c->flags = flags;
  c->n_max = n_max;
  c->r_max = r_max;
  c->np_max = (n_max + WW_TB - 1) / WW_TB * WW_TB;
  const size_t np = c->np_max, nm = n_max, R = r_max;
  const int nbm = (int)(np / WW_TB);
  c->nsplit_max = nbm;
  int rc = 0;
#define AL(ptr, bytes) \
  if ((rc = dalloc(c, (void**)&(ptr), (bytes))) != 0) { ww_destroy(c); return rc; }
  AL(c->A, np * np * 8);
  AL(c->Gm, np * np * 8);
  AL(c->Xi, np * np * 8);
  AL(c->Zi, np * np * 8);
  AL(c->Vi, np * np * 8);
  AL(c->Dinv, (size_t)nbm * 4096 * 8);
  if (flags & WW_MIXED) {
    AL(c->A32, np * np * 4);
    AL(c->X32, np * np * 4);
    AL(c->Z32, np * np * 4);
    AL(c->V32, np * np * 4);
    AL(c->Dinv32, (size_t)nbm * 4096 * 4);
    AL(c->Rr, np * R * 8);
    AL(c->rr0, np * 8);
  }
  AL(c->cosT, nm * 8);
  AL(c->sinT, nm * 8);
  AL(c->c0T, nm * 8);
  AL(c->sig, nm * 8);
  AL(c->tw, nm * sizeof(cplx));
  AL(c->aux, (size_t)AUX_COUNT * nm * 8);
  AL(c->rhs0, np * 8);
  AL(c->y0t, np * 8);
  AL(c->mu0, np * 8);
  AL(c->gam0, np * 8);
  AL(c->hg0, np * 8);
  AL(c->gphi0, np * 8);
  AL(c->Psi, np * R * 8);
  AL(c->Ytmp, np * R * 8);
  AL(c->Mu, np * R * 8);
  AL(c->Gam, np * R * 8);
  AL(c->HG, np * R * 8);
  AL(c->Gpsi, np * R * 8);
  AL(c->part, (size_t)c->nsplit_max * np * R * 8);
  AL(c->y, 2 * nm * R * 8);
  AL(c->Ys, 2 * nm * R * 8);
  AL(c->K, 16 * 2 * nm * R * 8);
  AL(c->Kx, 2 * nm * 8);
  AL(c->ydtn, 2 * nm * 8);
  AL(c->basis, 2 * nm * (R > 1 ? R - 1 : 1) * 8);
  AL(c->qfix, 2 * nm * 8);
  AL(c->coef, COEF_SIZE * 8);
  AL(c->fdev, 64);
  AL(c->status, 64);
#undef AL
  HIPCHK(hipMemset(c->status, 0, 64));
  HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  {
    const char* ng = std::getenv("WW_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    const char* nr = std::getenv("WW_NREF");
    if (nr) c->nref = std::max(0, std::min(8, std::atoi(nr)));
  }
  // kernels whose dynamic LDS can exceed the default 64 KiB
  const int big = 160 * 1024;
  HIPCHK(hipFuncSetAttribute((const void*)k_blu_init<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_blu_step<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_blu_final<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_gemm_part<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_blu_init<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_blu_step<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_blu_final<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_gemm_part<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_base_prep, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_gamma, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_base_rhs, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_col_rhs, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_step_end, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  *out = c;
  return 0;
}

void ww_destroy(ww_ctx* c) {
  if (!c) return;
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}

int ww_set_stream(ww_ctx* c, void* s) {
  if (!c) return fail(WW_EINVAL, "ctx is null");
  c->stream = (hipStream_t)s;
  return 0;
}

int ww_set_tableau(ww_ctx* c, int s, const double* a, const double* b, const double* cn) {
  (void)cn;
  if (!c || !a || !b) return fail(WW_EINVAL, "null argument");
  if (s < 1 || s > 16) return fail(WW_EINVAL, "1 <= s <= 16 stages");
  for (int i = 0; i < s; ++i)
    for (int j = i; j < s; ++j)
      if (a[i * s + j] != 0.0) return fail(WW_EINVAL, "tableau is not explicit (a not strictly lower)");
  c->nst = s;
  c->gnst = -1;   // re-capture the step graph
  std::memset(c->ta, 0, sizeof(c->ta));
  std::memset(c->tb, 0, sizeof(c->tb));
  for (int i = 0; i < s; ++i) {
    for (int j = 0; j < i; ++j) c->ta[i * 16 + j] = a[i * s + j];
    c->tb[i] = b[i];
  }
  return 0;
}

}  // extern "C"

// ------------------------------------------------------------------------------------
// kernel sequences
// ------------------------------------------------------------------------------------
static size_t fft_lds_bytes(int N, int nbuf) { return (size_t)nbuf * N * sizeof(cplx); }
static const size_t TILE_BYTES = (size_t)TILE_DBL * 8;

template <typename T>
static BluBufs<T> blu_bufs(ww_ctx* c, T* A, T* X, T* Z, T* V, T* D) {
  BluBufs<T> b;
  b.A = A;
  b.X = X;
  b.Z = Z;
  b.V = V;
  b.Dinv = D;
  b.status = c->status;
  b.Np = c->Np;
  b.pivguard = 1e-8;
  return b;
}

template <typename T>
static int enqueue_blu(ww_ctx* c, const BluBufs<T>& b) {
  const int nb = c->Np / WW_TB;
  const size_t es = sizeof(T);
  hipLaunchKernelGGL(k_blu_init<T>, dim3(1), dim3(WW_NT), (TILE_DBL + 256) * es, c->stream, b);
  LAUNCHCHK();
  for (int k = 0; k + 1 < nb; ++k) {
    const int nt = nb - k - 1;
    const int nblk = nt * nt + 2 * nt * (k + 1);
    hipLaunchKernelGGL(k_blu_step<T>, dim3(nblk), dim3(WW_NT), (4 * TILE_DBL + 256) * es, c->stream, b, k);
    LAUNCHCHK();
  }
  if (nb > 1) {
    hipLaunchKernelGGL(k_blu_final<T>, dim3(nb - 1), dim3(WW_NT), 2 * TILE_DBL * es, c->stream, b);
    LAUNCHCHK();
  }
  return 0;
}

static bool mixed(const ww_ctx* c) { return (c->flags & WW_MIXED) != 0; }

// assembly of A, Gm and the block LU of A (FP64, or of the FP32 copy in mixed mode)
// with the block-triangular inverses
static int enqueue_assemble_lu(ww_ctx* c) {
  const int nb = c->Np / WW_TB;
  hipLaunchKernelGGL(k_assemble, dim3(nb, nb), dim3(WW_NT), 0, c->stream, c->aux, c->n_max, c->cosT, c->sinT,
                     c->c0T, c->A, c->Gm, mixed(c) ? c->A32 : nullptr, c->N, c->Np, c->finite);
  LAUNCHCHK();
  if (mixed(c)) return enqueue_blu<float>(c, blu_bufs<float>(c, c->A32, c->X32, c->Z32, c->V32, c->Dinv32));
  return enqueue_blu<double>(c, blu_bufs<double>(c, c->A, c->Xi, c->Zi, c->Vi, c->Dinv));
}

// out = add + sgn * M B for R columns (ld Np), M taken as full (mode 0), strictly lower
// (mode 1) or upper (mode 2) in 64-blocks.  Split-K partials, then a reduction.
template <typename T>
static int enqueue_gemm(ww_ctx* c, const T* M, int mode, const double* B, const double* add, double sgn,
                        double* out, int R) {
  const int nkt = c->Np / WW_TB;
  const int tiles = nkt * ((R + 63) / 64);
  int nsplit = (512 + tiles - 1) / tiles;
  if (nsplit > nkt) nsplit = nkt;
  if (nsplit < 1) nsplit = 1;
  const int kchunk = (nkt + nsplit - 1) / nsplit;
  nsplit = (nkt + kchunk - 1) / kchunk;
  hipLaunchKernelGGL(k_gemm_part<T>, dim3(nkt, (R + 63) / 64, nsplit), dim3(WW_NT), 2 * TILE_DBL * sizeof(T),
                     c->stream, M, c->Np, mode, B, R, c->part, kchunk);
  LAUNCHCHK();
  const size_t n = (size_t)c->Np * R;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_gemm_reduce, dim3(blocks), dim3(256), 0, c->stream, c->part, nsplit, add, sgn, out, c->Np, R);
  LAUNCHCHK();
  return 0;
}

// X = A^{-1} B for R columns (ld Np); Y and Rs are scratch; B is kept.
// FP64:  X = Z (B + Xs B).
// mixed: X = Z32 (B + X32 B), then nref sweeps of  r = B - A X (FP64 residual with the
//        FP64 matrix),  X += Z32 (r + X32 r)  (FP32 factors, FP64 accumulation).
static int enqueue_solve(ww_ctx* c, double* B, double* Y, double* X, double* Rs, int R) {
  int rc;
  if (!mixed(c)) {
    if ((rc = enqueue_gemm<double>(c, c->Xi, 1, B, B, 1.0, Y, R))) return rc;
    return enqueue_gemm<double>(c, c->Zi, 2, Y, nullptr, 1.0, X, R);
  }
  if ((rc = enqueue_gemm<float>(c, c->X32, 1, B, B, 1.0, Y, R))) return rc;
  if ((rc = enqueue_gemm<float>(c, c->Z32, 2, Y, nullptr, 1.0, X, R))) return rc;
  for (int it = 0; it < c->nref; ++it) {
    if ((rc = enqueue_gemm<double>(c, c->A, 0, X, B, -1.0, Rs, R))) return rc;
    if ((rc = enqueue_gemm<float>(c, c->X32, 1, Rs, Rs, 1.0, Y, R))) return rc;
    if ((rc = enqueue_gemm<float>(c, c->Z32, 2, Y, X, 1.0, X, R))) return rc;
  }
  return 0;
}

// DtN of R columns in B (ld Np): out = G psi (ld Np); mu in Mu; Rs residual scratch
static int enqueue_dtn_cols(ww_ctx* c, double* B, double* Yt, double* Mu, double* Gam, double* HGm, double* out,
                            double* Rs, int R) {
  int rc;
  if ((rc = enqueue_solve(c, B, Yt, Mu, Rs, R))) return rc;
  hipLaunchKernelGGL(k_gamma, dim3((R + 1) / 2), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, Mu, c->Np, R, Gam,
                     HGm, c->tw, c->N);
  LAUNCHCHK();
  return enqueue_gemm<double>(c, c->Gm, 0, Gam, HGm, 1.0, out, R);
}

static size_t kstride(const ww_ctx* c) { return (size_t)2 * c->N * (c->M + 1); }

// base chain of stage s: prep, assembly, LU, base DtN, base right-hand side -> kout
static int enqueue_base_chain(ww_ctx* c, const double* ysrc, int s, double* kout) {
  int rc;
  hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, ysrc, c->K, c->Ys, c->coef,
                     s, kstride(c), c->aux, c->n_max, c->rhs0, c->Np, c->tw, c->N, c->hsurf);
  LAUNCHCHK();
  if ((rc = enqueue_assemble_lu(c))) return rc;
  if ((rc = enqueue_dtn_cols(c, c->rhs0, c->y0t, c->mu0, c->gam0, c->hg0, c->gphi0, c->rr0, 1))) return rc;
  hipLaunchKernelGGL(k_base_rhs, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->gphi0, c->aux,
                     c->n_max, kout, c->tw, c->sig, c->N, c->g, c->tau);
  LAUNCHCHK();
  return 0;
}

static int enqueue_col_chain(ww_ctx* c, int s) {
  int rc;
  const int M = c->M;
  const size_t tot = (size_t)c->Np * M;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_col_pre, dim3(blocks), dim3(256), 0, c->stream, c->y, c->K, c->Ys, c->coef, s, kstride(c),
                     c->aux, c->n_max, c->Psi, c->Np, c->N, M);
  LAUNCHCHK();
  if ((rc = enqueue_dtn_cols(c, c->Psi, c->Ytmp, c->Mu, c->Gam, c->HG, c->Gpsi, c->Rr, M))) return rc;
  hipLaunchKernelGGL(k_col_rhs, dim3(M), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->Gpsi, c->Np,
                     c->aux, c->n_max, c->K + (size_t)s * kstride(c), c->tw, c->sig, c->N, c->g, c->tau);
  LAUNCHCHK();
  return 0;
}

static int enqueue_step(ww_ctx* c, bool cols) {
  int rc;
  for (int s = 0; s < c->nst; ++s) {
    if ((rc = enqueue_base_chain(c, c->y, s, c->K + (size_t)s * kstride(c)))) return rc;
    if (cols && c->M > 0)
      if ((rc = enqueue_col_chain(c, s))) return rc;
  }
  const int ncol = cols ? c->M + 1 : 1;
  hipLaunchKernelGGL(k_step_end, dim3(ncol), dim3(WW_NT), fft_lds_bytes(c->N, 3), c->stream, c->y, c->K, kstride(c),
                     c->nst, c->coef, c->tw, c->sig, c->N, 0);
  LAUNCHCHK();
  return 0;
}

// Capture one step (all stages + end of step) into a graph on the private capture
// stream; the graph is reused while (N, M, columns, stages) are unchanged.  Step
// coefficients live in device memory, so T and the parameters may change freely.
static int ensure_step_graph(ww_ctx* c, bool cols) {
  if (c->step_exec && c->gN == c->N && c->gM == c->M && c->gcols == (int)cols && c->gnst == c->nst) return 0;
  if (c->step_exec) {
    HIPCHK(hipGraphExecDestroy(c->step_exec));
    c->step_exec = nullptr;
  }
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_step(c, cols);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  c->stream = user;
  if (rc) {
    if (e == hipSuccess && g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIPCHK(e);
  const hipError_t ei = hipGraphInstantiate(&c->step_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(ei);
  c->gN = c->N;
  c->gM = c->M;
  c->gcols = (int)cols;
  c->gnst = c->nst;
  return 0;
}

static int read_status(ww_ctx* c, int* st) {
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(st, c->status, sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(c->status, 0, sizeof(int)));
  return 0;
}

static int check_domain(ww_ctx* c, const double* surface) {
  if (!c->finite) return 0;
  std::vector<double> hs(c->N);
  HIPCHK(hipMemcpyAsync(hs.data(), surface, c->N * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < c->N; ++i)
    if (!(c->h + hs[i] > 0.0)) return fail(WW_EDOMAIN, "finite depth: surface height h + eta <= 0");
  return 0;
}

extern "C" {

int dtn_setup(ww_ctx* c, const double* surface, double h, double tau, int N) {
  if (!c || !surface) return fail(WW_EINVAL, "null argument");
  int rc;
  if ((rc = set_grid(c, N, h))) return rc;
  c->tau = tau;
  if ((rc = check_domain(c, surface))) return rc;
  HIPCHK(hipMemcpyAsync(c->ydtn, surface, N * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemsetAsync(c->ydtn + N, 0, N * 8, c->stream));
  hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 4), c->stream, c->ydtn, c->K, c->Ys,
                     c->coef, 0, (size_t)0, c->aux, c->n_max, c->rhs0, c->Np, c->tw, N, c->hsurf);
  LAUNCHCHK();
  if ((rc = enqueue_assemble_lu(c))) return rc;
  int st = 0;
  if ((rc = read_status(c, &st))) return rc;
  c->dtn_ready = true;
  if (st & 1) return fail(WW_EPIVOT, "unpivoted LU: pivot below guard");
  return 0;
}

int dtn_solve_multi(ww_ctx* c, const double* rhs, int nrhs, double* dtn_out, double* mu_out) {
  if (!c || !rhs || !dtn_out) return fail(WW_EINVAL, "null argument");
  if (!c->dtn_ready) return fail(WW_ENOSETUP, "dtn_solve_multi before dtn_setup");
  if (nrhs < 1 || nrhs > c->r_max) return fail(WW_EINVAL, "nrhs out of range");
  const int N = c->N, Np = c->Np;
  const size_t tot = (size_t)Np * nrhs;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, rhs, N, c->Psi, Np, N, Np, nrhs);
  LAUNCHCHK();
  int rc;
  if ((rc = enqueue_dtn_cols(c, c->Psi, c->Ytmp, c->Mu, c->Gam, c->HG, c->Gpsi, c->Rr, nrhs))) return rc;
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, c->Gpsi, Np, dtn_out, N, Np, N, nrhs);
  LAUNCHCHK();
  if (mu_out) {
    hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, c->Mu, Np, mu_out, N, Np, N, nrhs);
    LAUNCHCHK();
  }
  return 0;
}

int shoot_setup(ww_ctx* c, int N, double h, double tau, double g, const double* basis, const double* q_fixed,
                int M) {
  if (!c || (!basis && M > 0)) return fail(WW_EINVAL, "null argument");
  if (M < 0 || M + 1 > c->r_max) return fail(WW_EINVAL, "M + 1 must be <= r_max");
  int rc;
  if ((rc = set_grid(c, N, h))) return rc;
  c->tau = tau;
  c->g = g;
  c->M = M;
  c->shootN = N;
  c->shootH = h;
  if (M > 0) HIPCHK(hipMemcpyAsync(c->basis, basis, (size_t)2 * N * M * 8, hipMemcpyDeviceToDevice, c->stream));
  if (q_fixed)
    HIPCHK(hipMemcpyAsync(c->qfix, q_fixed, (size_t)2 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  else
    HIPCHK(hipMemsetAsync(c->qfix, 0, (size_t)2 * N * 8, c->stream));
  c->shoot_ready = true;
  return 0;
}

int shoot_eval(ww_ctx* c, const double* params, double T, int nsteps, double* r, double* J, double* drdT,
               double* f) {
  if (!c || !r || (!params && c->M > 0)) return fail(WW_EINVAL, "null argument");
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "shoot_eval before shoot_setup");
  if (c->nst < 1) return fail(WW_EINVAL, "no tableau set");
  if (nsteps < 1 || !std::isfinite(T)) return fail(WW_EINVAL, "nsteps >= 1 and finite T required");
  int rc;
  if ((rc = set_grid(c, c->shootN, c->shootH))) return rc;
  c->dtn_ready = false;   // the factor arrays are reused by the march
  const int N = c->N, M = c->M;
  const bool cols = (J != nullptr) && M > 0;
  // step coefficients: a_sj dt, b_s dt
  double coef[COEF_SIZE];
  std::memset(coef, 0, sizeof(coef));
  const double dt = T / (4.0 * nsteps);
  for (int s = 0; s < c->nst; ++s) {
    for (int j = 0; j < s; ++j) coef[s * 16 + j] = c->ta[s * 16 + j] * dt;
    coef[COEF_B + s] = c->tb[s] * dt;
  }
  coef[COEF_DT] = dt;
  HIPCHK(hipMemcpyAsync(c->coef, coef, sizeof(coef), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemsetAsync(c->status, 0, sizeof(int), c->stream));
  {
    const size_t tot = (size_t)2 * N * (M + 1);
    const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, c->stream, c->y, c->basis, c->qfix, params, N, M);
    LAUNCHCHK();
  }
  // the march works on R = M + 1 columns when J is requested, on the base otherwise;
  // K and state strides always use M + 1 columns
  if (c->use_graph) {
    if ((rc = ensure_step_graph(c, cols))) return rc;
    for (int n = 0; n < nsteps; ++n) HIPCHK(hipGraphLaunch(c->step_exec, c->stream));
  } else {
    for (int n = 0; n < nsteps; ++n)
      if ((rc = enqueue_step(c, cols))) return rc;
  }
  {
    const size_t n = (size_t)2 * N * (cols ? M + 1 : 1);
    hipLaunchKernelGGL(k_check_finite, dim3(64), dim3(256), 0, c->stream, c->y, n, c->status);
    LAUNCHCHK();
  }
  if (drdT)
    if ((rc = enqueue_base_chain(c, c->y, 0, c->Kx))) return rc;
  {
    const size_t tot = (size_t)N * (M + 1);
    const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_outputs, dim3(blocks), dim3(256), 0, c->stream, c->y, c->Kx, r, cols ? J : nullptr, drdT, N,
                       cols ? M : 0);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(WW_NT), 0, c->stream, r, N, c->fdev);
  LAUNCHCHK();
  if (f) HIPCHK(hipMemcpyAsync(f, c->fdev, 8, hipMemcpyDeviceToHost, c->stream));
  int st = 0;
  if ((rc = read_status(c, &st))) return rc;
  if (st & 2) return fail(WW_ENONFINITE, "non-finite value in the marched state");
  if (st & 1) return fail(WW_EPIVOT, "unpivoted LU: pivot below guard");
  return 0;
}

int shoot_adjoint(ww_ctx* c, const double* params, double T, int nsteps, int ckpt_every, double* grad,
                  double* dfdT, double* f) {
  (void)params; (void)T; (void)nsteps; (void)ckpt_every; (void)grad; (void)dfdT; (void)f;
  if (!c) return fail(WW_EINVAL, "null argument");
  return fail(WW_EINVAL, "shoot_adjoint: not available in this build");
}

}  // extern "C"
