// Host side of the C ABI declared in include/ww.h: context and workspace, the
// per-stage kernel sequence, the march to T/4 and the outputs.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "ww.h"
#include "ww_kernels.hpp"
#include "ww_mesh.hpp"
#include "ww_dd.hpp"
#include "ww_sdc.hpp"
#include "ww_svd.hpp"
#include "ww_gmres.hpp"

#include <algorithm>
#include <chrono>
#include <mutex>
#include <numeric>

// Fixed device workspace of the allocation-free solve (dtn_solve_multi_noalloc): one
// array per GPU, held until the process ends.  Host code never uses its name as an
// address: ww_create resolves the address on each device once (hipGetSymbolAddress,
// with that device current) and every use goes through that pointer.
#define WW_SCRATCH_DOUBLES ((size_t)WW_SCRATCH_BYTES / 8)
static __device__ __align__(256) double scratch[WW_SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static const int SCRATCH_MAX_DEV = 64;
static double* g_scratch_dev[SCRATCH_MAX_DEV] = {};

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

// One stage's factor set of the lagged-factor pipeline (all Np x Np unless noted)
struct RingSet {
  double *A = nullptr, *Gm = nullptr, *X = nullptr, *Z = nullptr, *V = nullptr, *Dinv = nullptr;
  double *Mi = nullptr, *Gmr = nullptr, *Ar = nullptr, *aux = nullptr;
  float *A32 = nullptr, *X32 = nullptr, *Z32 = nullptr, *V32 = nullptr, *Dinv32 = nullptr;
  float* Mi32 = nullptr;
};
#define PIPE_MAXLAG 11
#define PIPE_MAXLUS 6

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
  // second factor set and per-point arrays: stages alternate between the two sets so
  // that the column chain of stage s overlaps the base chain of stage s + 1
  double *A_1 = nullptr, *Gm_1 = nullptr, *Xi_1 = nullptr, *Zi_1 = nullptr, *Vi_1 = nullptr, *Dinv_1 = nullptr;
  float *A32_1 = nullptr, *X32_1 = nullptr, *Z32_1 = nullptr, *V32_1 = nullptr, *Dinv32_1 = nullptr;
  double* aux_1 = nullptr;
  // row-major explicit inverses A^{-1} (per parity; FP32 in the mixed form) and
  // row-major Gm, read by the one-vector products of the base chain and (the inverse)
  // by the column solves
  double *Mi = nullptr, *Gmr = nullptr, *Mi_1 = nullptr, *Gmr_1 = nullptr;
  float *Mi32 = nullptr, *Mi32_1 = nullptr;
  double *Ar = nullptr, *Ar_1 = nullptr;   // mixed mode: FP64 A for the residuals
  hipStream_t side = nullptr;  // column-chain stream
  hipEvent_t evB[16] = {}, evC[16] = {};
  float *A32 = nullptr, *X32 = nullptr, *Z32 = nullptr, *V32 = nullptr, *Dinv32 = nullptr;
  double *Rr = nullptr, *rr0 = nullptr;   // residuals of the refinement sweeps
  int nref = 2;                            // refinement sweeps per solve (mixed mode)
  int nref_lag = -1;                       // sweeps of a lagged-factor solve (-1: nref)
  double *cosT = nullptr, *sinT = nullptr, *c0T = nullptr, *sig = nullptr;
  cplx* tw = nullptr;
  double* aux = nullptr;
  double *rhs0 = nullptr, *y0t = nullptr, *mu0 = nullptr, *gam0 = nullptr, *hg0 = nullptr, *gphi0 = nullptr;
  double *Psi = nullptr, *Ytmp = nullptr, *Mu = nullptr, *Gam = nullptr, *HG = nullptr, *Gpsi = nullptr;
  double *y = nullptr, *Ys = nullptr, *K = nullptr, *Kx = nullptr, *ydtn = nullptr;
  double *basis = nullptr, *qfix = nullptr;
  double* coef = nullptr;
  double* fdev = nullptr;
  // non-uniform mesh of the segmented march (shoot_eval_segments only): while `mapped`,
  // the assembly, right-hand sides and outputs take the mapped-grid kernels and read
  // the per-point tables of the current segment (MESH_COUNT x n_max doubles)
  bool mapped = false;
  double* mesh = nullptr;
  // double-double DtN (dtn_setup_dd, dtn_solve_multi_dd), allocated at first use:
  // circulant tables (cos, sin of 2 pi d/N, cot(pi d/N)/2; 3 planes of n_max) and FFT
  // twiddles for grid dd_N, per-point surface quantities (4 planes), A and Gm (Np x Np,
  // hi and lo planes), and the solve's work planes (DD_WORK planes of np_max x r_max)
  int dd_N = 0;
  bool dd_ready = false;
  double *dd_tab_hi = nullptr, *dd_tab_lo = nullptr;
  cdd* dd_tw = nullptr;
  double *dd_pt_hi = nullptr, *dd_pt_lo = nullptr;
  double *dd_Ah = nullptr, *dd_Al = nullptr, *dd_Gh = nullptr, *dd_Gl = nullptr;
  double* dd_w = nullptr;
  double* dd_part = nullptr;   // chunk partials of the one-column double-double product
  // SDC15 (shoot_eval_sdc), allocated at first use: the stage slopes of one step
  // (SDC_STAGES slots of 2 n_max r_max), the stage state, and the sparse stage rows
  // (SDC_STAGES + 1 rows of SDC_MAXNZ slot indices and weights; the last row is the
  // step's final combination)
  double *sdc_K = nullptr, *sdc_y = nullptr, *sdc_w = nullptr;
  int* sdc_j = nullptr;
  int sdc_cnt[SDC_STAGES + 1] = {};
  // the nodes of a correction sweep, evaluated together: per node the stage state, its
  // stage-state copy and the base Dirichlet data (SDC_NODES each); the LU stream's event
  double *sdc_yn = nullptr, *sdc_ysn = nullptr, *sdc_rhsn = nullptr;
  hipEvent_t sdc_ev = nullptr;
  // per lane (SDC_NODES lanes: a factor set of the ring and the per-node buffers above):
  // the base chain that last used it (main stream), its column chain (column stream)
  hipEvent_t sdc_evB[SDC_NODES] = {}, sdc_evC[SDC_NODES] = {};
  // the base-chain scratch of the sweep nodes whose chains run on the LU stream (6 Np_max)
  double* sdc_b2 = nullptr;
  // lagged factors for the predictor's base solves (environment WW_SDC_LAG=0: off); the
  // LU stream's event per lane (the lagged stages' own LUs, read by their column chains)
  bool sdc_lag = true;
  int sdc_lag_sweeps = LAG_SWEEPS;   // environment WW_SDC_LAG_SWEEPS (0..8)
  hipEvent_t sdc_evL[SDC_NODES] = {};
  // the base march in double-double (shoot_eval_sdc_dd), allocated at first use: state
  // and stage state (2 n_max, hi and lo), the slopes (SDC_STAGES + 1 slots: the last
  // for the right-hand side at the final state), G phi, the filter symbol, the sparse
  // stage rows with double-double weights, f
  double *sdd_yh = nullptr, *sdd_yl = nullptr, *sdd_Yh = nullptr, *sdd_Yl = nullptr;
  double *sdd_Kh = nullptr, *sdd_Kl = nullptr, *sdd_Gh = nullptr, *sdd_Gl = nullptr;
  double *sdd_fh = nullptr, *sdd_fl = nullptr, *sdd_wh = nullptr, *sdd_wl = nullptr, *sdd_fo = nullptr;
  int* sdd_j = nullptr;
  int sdd_cnt[SDC_STAGES + 1] = {};
  double* sdd_lane = nullptr;   // the grouped sweeps' lanes (SDC_NODES of them)
  // the second group's solve workspace, partials and G phi (hi, lo) of the grouped sweeps
  double *sdd_w2 = nullptr, *sdd_part2 = nullptr, *sdd_G2 = nullptr;
  int gmap = -1;   // `mapped` of the captured step graph
  int* status = nullptr;
  std::vector<void*> allocs;
  // adjoint: checkpoints, per-stage factor storage of one segment, work vectors
  double* ckpt = nullptr;
  size_t ckpt_cap = 0;
  double* seg = nullptr;
  size_t seg_cap = 0;
  double* adj = nullptr;   // lam, mu, ups[16], gt, hd, e1, q, g2, zeta, y1, y2, rv, dv
  // optional HIP events around phases of every stage of the captured step
  // (0: block LU, 1: whole base chain, 2: column chain); the values of the last
  // replayed step are read back by ww_profile_read
  bool prof = false;
  int prof_stage = -1;   // stage being enqueued (marks are taken only inside a step)
  bool prof_kev = false;   // time every directly launched block-LU step with HIP events
  std::vector<hipEvent_t> kev_a, kev_b;
  size_t kev_n = 0;
  unsigned long long* stamps = nullptr;   // [phase][stage] x {start, sum, count}
  // host time spent enqueueing the steps of profiled marches (phase 3), and their count
  double host_enq_ms = 0.0;
  long long host_enq_steps = 0;
  // one RK step captured as a graph, replayed nsteps times
  bool use_graph = true;
  bool overlap = true;   // column chain on the side stream (environment WW_NO_OVERLAP=1: one stream)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t step_exec = nullptr;
  int gN = -1, gM = -1, gcols = -1, gnst = -1, gtwo = -1;
  unsigned gfb = ~0u;
  int ggm = -1;   // GMRES step budget captured in the graph (0: no GMRES)
  // fallbacks: fb is the mode the factor sets are built in (WW_FB_* bits), fb_last what
  // the results of the last call came from; guard is the unpivoted LU's pivot bound
  unsigned fb = 0, fb_last = 0;
  // a march on lagged factors failed its refinement test: the context's later marches
  // (until the next shoot_setup) start on each stage's own factors (WW_FB_DIRECT); not
  // for WW_STRICT contexts, which report every failure instead
  bool lag_off = false;
  double guard = 1e-8;
  double* scratch = nullptr;   // this device's fixed workspace (address resolved at create)
  // partial-pivoting buffers, allocated on the first fallback: row order, elimination
  // workspace (Np x Np), gathered right-hand sides (Np x r_max); the adjoint keeps one
  // row order per stored stage
  int* perm = nullptr;
  double *pw = nullptr, *pb = nullptr;
  int* seg_perm = nullptr;
  size_t seg_perm_cap = 0;
  // lagged-factor pipeline of single-instance marches: the base solve of stage s uses
  // the factors of stage s - lag (refined against its own matrix) while the LU of
  // stage s runs on one of `lag` streams; the column chain of stage s waits for it
  int lag = 8;   // environment WW_PIPE_LAG, 0..PIPE_MAXLAG (0: every solve uses its own factors)
  // stages factored together by one LU launch sequence (environment WW_LU_GROUP,
  // 1..BLU_GMAX; at most the lag)
  int lu_group = 2;
  int minv_wgs = 1 << 20;                  // workgroup cap of the explicit-inverse launch
  int graph_parts = 10;                    // parts of a march stage replayed from graphs (bit per part)
  int blu_strip = 4;                       // tiles per strip task of a block-LU step
  int dtn_rows = 8;                        // rows per workgroup of the base DtN launch
  int gemm_split = 4;                      // wave groups splitting the inner dimension of a product
  int gemm_rows = 32;                      // rows of a column product's output tile (16 or 32)
  int lag32 = 0;                           // FP64 form: lagged solves read an FP32 copy of the inverse
  int asm_cw = 16;                         // columns per assembly workgroup
  int tune_gen = 0;                        // bumped by ww_set_tuning (graphs are re-captured)
  int gtune = -1;                          // tune_gen of the captured step graph
  // LU streams (stage s on stream s mod nlus), at most lag; environment WW_LU_STREAMS,
  // by default 3 with the column chains on them, 2 beside the column stream
  int nlus = 3;
  // the column chain of stage s runs on the LU stream of stage s, after its LU, instead
  // of on the column stream (environment WW_COLS_ON_LU=0 turns it off)
  bool cols_on_lu = true;
  int ring_n = 0;          // factor sets allocated (one per stage)
  RingSet ring[16];
  hipStream_t lus[PIPE_MAXLUS] = {};
  hipEvent_t evA[16] = {}, evL[16] = {};
  // one graph per branch and stage of the lagged-factor march (prep, LU, base, columns)
  // and the two halves of the step end (base column: main stream; Jacobian columns:
  // column stream), replayed on their own streams; pkey: what they were captured for.
  // evE: the column stream's step end; pjoin: the main stream has not yet waited for it
  hipGraphExec_t pgx[16][4] = {};
  hipGraphExec_t pgend = nullptr, pgendc = nullptr;
  hipEvent_t evE = nullptr;
  bool pjoin = false;
  bool pcols = true;   // the current lagged march has Jacobian columns (column chains)
  long long pkey = -1;
  // thin SVD / Levenberg-Marquardt workspace (first use): W (n_max x r_max), residuals,
  // parameters, V (r_max^2), column norms and dots, convergence flag, column order
  double *lmW = nullptr, *lmr = nullptr, *lmrn = nullptr, *lmp = nullptr, *lmV = nullptr;
  double *lmsig = nullptr, *lmdot = nullptr;
  int *lmflag = nullptr, *lmperm = nullptr;
  // GMRES base solves of marches without columns (flag WW_GMRES): at most gm_m Arnoldi
  // steps per solve (environment WW_GMRES_ITERS); buffers on first use
  int gm_m = 24;
  bool gm_fixed = false;   // WW_GMRES_ITERS given: no calibration
  bool gm_active = false;
  double *gmV = nullptr, *gmw = nullptr, *gmH = nullptr, *gmcs = nullptr, *gmsn = nullptr, *gmg = nullptr;
  double* gmbeta = nullptr;
  int* gmstate = nullptr;
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
  // queued work of the previous grid may still read the tables
  HIPCHK(hipStreamSynchronize(c->stream));
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
  // FFT twiddles in pass order (radix 4, then 3, then 2): the pass of radix R starting
  // at span Ns takes exp(-2 pi i jm q / (Ns R)) = tw[jm q N / (Ns R)] at offset
  // Ns - 1 + (q - 1) Ns + jm
  std::vector<cplx> twp(N, cplx{0.0, 0.0});
  {
    int m = N, Ns = 1;
    auto add_pass = [&](int R) {
      const int tstride = N / (Ns * R);
      for (int q = 1; q < R; ++q)
        for (int jm = 0; jm < Ns; ++jm) twp[Ns - 1 + (q - 1) * Ns + jm] = tw[(size_t)jm * q * tstride];
      Ns *= R;
      m /= R;
    };
    while (m % 4 == 0) add_pass(4);
    while (m % 3 == 0) add_pass(3);
    while (m % 2 == 0) add_pass(2);
  }
  HIPCHK(hipMemcpy(c->tw, twp.data(), N * sizeof(cplx), hipMemcpyHostToDevice));
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
  if (flags & ~(WW_MIXED | WW_STRICT | WW_GMRES)) return fail(WW_EINVAL, "unknown flags");
  ww_ctx* c = new ww_ctx();
  // a failure after this point releases what was created so far
#define CCHK(x)                                                                        \
  do {                                                                                 \
    const hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                            \
      ww_destroy(c);                                                                   \
      return fail(WW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));             \
    }                                                                                  \
  } while (0)
  CCHK(hipGetDevice(&c->dev));
  {
    // the fixed workspace of the allocation-free solve: its address on this device,
    // resolved once per device with the device current
    if (c->dev < 0 || c->dev >= SCRATCH_MAX_DEV) {
      ww_destroy(c);
      return fail(WW_EINVAL, "device index out of range");
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[c->dev]) {
      void* sp = nullptr;
      const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !sp) {
        ww_destroy(c);
        return fail(WW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      }
      g_scratch_dev[c->dev] = (double*)sp;
    }
    c->scratch = g_scratch_dev[c->dev];
  }
  c->stream = (hipStream_t)hip_stream;
  c->flags = flags;
  c->n_max = n_max;
  c->r_max = r_max;
  c->np_max = (n_max + WW_TB - 1) / WW_TB * WW_TB;
  const size_t np = c->np_max, nm = n_max, R = r_max;
  const int nbm = (int)(np / WW_TB);
  int rc = 0;
#define AL(ptr, bytes) \
  if ((rc = dalloc(c, (void**)&(ptr), (bytes))) != 0) { ww_destroy(c); return rc; }
  AL(c->A, np * np * 8);
  AL(c->Gm, np * np * 8);
  AL(c->Xi, np * np * 8);
  AL(c->Zi, np * np * 8);
  AL(c->Vi, np * np * 8);
  AL(c->Dinv, (size_t)nbm * 4096 * 8);
  AL(c->A_1, np * np * 8);
  AL(c->Gm_1, np * np * 8);
  AL(c->Xi_1, np * np * 8);
  AL(c->Zi_1, np * np * 8);
  AL(c->Vi_1, np * np * 8);
  AL(c->Dinv_1, (size_t)nbm * 4096 * 8);
  AL(c->Mi, np * np * 8);
  AL(c->Gmr, np * np * 8);
  AL(c->Mi_1, np * np * 8);
  AL(c->Gmr_1, np * np * 8);
  if (flags & WW_MIXED) {
    AL(c->Mi32, np * np * 4);
    AL(c->Mi32_1, np * np * 4);
    AL(c->Ar, np * np * 8);
    AL(c->Ar_1, np * np * 8);
    AL(c->A32, np * np * 4);
    AL(c->X32, np * np * 4);
    AL(c->Z32, np * np * 4);
    AL(c->V32, np * np * 4);
    AL(c->Dinv32, (size_t)nbm * 4096 * 4);
    AL(c->A32_1, np * np * 4);
    AL(c->X32_1, np * np * 4);
    AL(c->Z32_1, np * np * 4);
    AL(c->V32_1, np * np * 4);
    AL(c->Dinv32_1, (size_t)nbm * 4096 * 4);
    AL(c->Rr, np * R * 8);
  }
  AL(c->rr0, np * 8);   // residual of the one-vector solves (mixed form, lagged factors)
  AL(c->cosT, nm * 8);
  AL(c->sinT, nm * 8);
  AL(c->c0T, nm * 8);
  AL(c->sig, nm * 8);
  AL(c->tw, nm * sizeof(cplx));
  AL(c->aux, (size_t)AUX_COUNT * nm * 8);
  AL(c->aux_1, (size_t)AUX_COUNT * nm * 8);
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
  CCHK(hipMemset(c->status, 0, 64));
  for (int i = 0; i < 16; ++i) {
    CCHK(hipEventCreateWithFlags(&c->evB[i], hipEventDisableTiming));
    CCHK(hipEventCreateWithFlags(&c->evC[i], hipEventDisableTiming));
  }
  {
    const char* ng = std::getenv("WW_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    const char* no = std::getenv("WW_NO_OVERLAP");
    c->overlap = !(no && no[0] == '1');
    const char* sl = std::getenv("WW_SDC_LAG");
    c->sdc_lag = !(sl && sl[0] == '0');
    const char* ss = std::getenv("WW_SDC_LAG_SWEEPS");
    if (ss) c->sdc_lag_sweeps = std::max(0, std::min(8, std::atoi(ss)));
    const char* nr = std::getenv("WW_NREF");
    if (nr) c->nref = std::max(0, std::min(8, std::atoi(nr)));
    const char* nl = std::getenv("WW_NREF_LAG");
    if (nl) c->nref_lag = std::max(1, std::min(8, std::atoi(nl)));
    const char* gi = std::getenv("WW_GMRES_ITERS");
    if (gi) {
      c->gm_m = std::max(2, std::min(GM_MAXM, std::atoi(gi)));
      c->gm_fixed = true;
    }
    const char* pl = std::getenv("WW_PIPE_LAG");
    if (pl) c->lag = std::max(0, std::min(PIPE_MAXLAG, std::atoi(pl)));
    const char* cl = std::getenv("WW_COLS_ON_LU");
    c->cols_on_lu = !(cl && cl[0] == '0');
    if (!c->cols_on_lu) c->nlus = 2;
    const char* ns = std::getenv("WW_LU_STREAMS");
    if (ns) c->nlus = std::max(1, std::min(PIPE_MAXLUS, std::atoi(ns)));
    const char* lg = std::getenv("WW_LU_GROUP");
    if (lg) c->lu_group = std::max(1, std::min(BLU_GMAX, std::atoi(lg)));
    const char* gp = std::getenv("WW_GRAPH_PARTS");
    if (gp) c->graph_parts = std::atoi(gp) & 15;
    const char* mw = std::getenv("WW_MINV_WGS");
    if (mw) c->minv_wgs = std::max(1, std::atoi(mw));
    // streams: the working ones first, the capture stream (which never executes) last.
    // HIP shares its few hardware queues among a process's streams, each new stream
    // taking the least-used queue: created in this order, the caller's stream and the
    // three LU streams of a march (or the column stream and two LU streams) each get a
    // queue of their own (with four), and no LU waits in the base chain's in-order queue.
    const int nls = c->lag > 0 ? std::min(c->nlus, c->lag) : 0;
    // the column stream only where it is used (created on first need otherwise: every
    // stream a context holds shifts the queues of the streams created after it)
    if (!c->cols_on_lu) CCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    for (int i = 0; i < nls; ++i) CCHK(hipStreamCreateWithFlags(&c->lus[i], hipStreamNonBlocking));
    CCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const char* pg = std::getenv("WW_PIVOT_GUARD");
    if (pg) {
      const double v = std::atof(pg);
      if (std::isfinite(v) && v >= 0.0) c->guard = v;
    }
  }
  // kernels whose dynamic LDS can exceed the default 64 KiB
  const int big = 160 * 1024;
  CCHK(hipFuncSetAttribute((const void*)k_blu_init<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_blu_step<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_blu_final<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_minv<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_minv<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_blu_init<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_blu_step<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_blu_final<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_base_prep, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  {
    // k_gamma holds static LDS too (the folded refinement test): dynamic + static <= big
    hipFuncAttributes fa;
    CCHK(hipFuncGetAttributes(&fa, (const void*)k_gamma));
    CCHK(hipFuncSetAttribute((const void*)k_gamma, hipFuncAttributeMaxDynamicSharedMemorySize,
                             big - (int)fa.sharedSizeBytes));
  }
  for (const void* fn : {(const void*)k_base_rhs_map, (const void*)k_col_rhs_map, (const void*)k_base_rhs_prep_map}) {
    // static LDS (a reduction buffer) besides the dynamic transform buffers
    hipFuncAttributes fa;
    CCHK(hipFuncGetAttributes(&fa, fn));
    CCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, big - (int)fa.sharedSizeBytes));
  }
  CCHK(hipFuncSetAttribute((const void*)k_base_rhs, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_dd_prep, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_dd_gamma, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_dd_base_rhs, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_dd_filter_state, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_base_rhs_prep, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_base_dtn<16>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_base_dtn<WW_NMAX / 64>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_col_rhs, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_step_end, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_adj_pre, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_adj_mid, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  CCHK(hipFuncSetAttribute((const void*)k_adj_step, hipFuncAttributeMaxDynamicSharedMemorySize, big));
#undef CCHK
  *out = c;
  return 0;
}

void ww_destroy(ww_ctx* c) {
  if (!c) return;
  // no work of this context (stream-ordered calls, graph branches) may still run
  (void)hipDeviceSynchronize();
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  for (int s = 0; s < 16; ++s)
    for (int q = 0; q < 4; ++q)
      if (c->pgx[s][q]) (void)hipGraphExecDestroy(c->pgx[s][q]);
  if (c->pgend) (void)hipGraphExecDestroy(c->pgend);
  if (c->pgendc) (void)hipGraphExecDestroy(c->pgendc);
  if (c->evE) (void)hipEventDestroy(c->evE);
  if (c->sdc_ev) (void)hipEventDestroy(c->sdc_ev);
  for (int i = 0; i < SDC_NODES; ++i) {
    if (c->sdc_evB[i]) (void)hipEventDestroy(c->sdc_evB[i]);
    if (c->sdc_evC[i]) (void)hipEventDestroy(c->sdc_evC[i]);
    if (c->sdc_evL[i]) (void)hipEventDestroy(c->sdc_evL[i]);
  }
  for (hipEvent_t e : c->kev_a) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->kev_b) (void)hipEventDestroy(e);
  if (c->stamps) (void)hipFree(c->stamps);
  if (c->ckpt) (void)hipFree(c->ckpt);
  if (c->seg) (void)hipFree(c->seg);
  if (c->adj) (void)hipFree(c->adj);
  if (c->seg_perm) (void)hipFree(c->seg_perm);
  for (int i = 0; i < PIPE_MAXLUS; ++i)
    if (c->lus[i]) (void)hipStreamDestroy(c->lus[i]);
  for (int i = 0; i < 16; ++i) {
    if (c->evA[i]) (void)hipEventDestroy(c->evA[i]);
    if (c->evL[i]) (void)hipEventDestroy(c->evL[i]);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->side) (void)hipStreamDestroy(c->side);
  for (int i = 0; i < 16; ++i) {
    if (c->evB[i]) (void)hipEventDestroy(c->evB[i]);
    if (c->evC[i]) (void)hipEventDestroy(c->evC[i]);
  }
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}

int ww_get_tuning(ww_ctx* c, ww_tuning* t) {
  if (!c || !t) return fail(WW_EINVAL, "null argument");
  t->lag = c->lag;
  t->lu_group = c->lu_group;
  t->lu_streams = c->nlus;
  t->graph_parts = c->graph_parts;
  t->minv_wgs = c->minv_wgs;
  t->blu_strip = c->blu_strip;
  t->dtn_rows = c->dtn_rows;
  t->gemm_split = c->gemm_split;
  t->gemm_rows = c->gemm_rows;
  t->lag_fp32 = c->lag32;
  t->asm_cw = c->asm_cw;
  t->lag_sweeps = c->nref_lag >= 0 ? c->nref_lag : c->nref;
  return 0;
}

int ww_set_tuning(ww_ctx* c, const ww_tuning* t) {
  if (!c || !t) return fail(WW_EINVAL, "null argument");
  if (t->lag < 0 || t->lag > PIPE_MAXLAG) return fail(WW_EINVAL, "tuning: lag out of range");
  if (t->lu_group < 1 || t->lu_group > BLU_GMAX) return fail(WW_EINVAL, "tuning: lu_group out of range");
  if (t->lu_streams < 1 || t->lu_streams > PIPE_MAXLUS) return fail(WW_EINVAL, "tuning: lu_streams out of range");
  if (t->graph_parts < 0 || t->graph_parts > 15) return fail(WW_EINVAL, "tuning: graph_parts out of range");
  if (t->minv_wgs < 1) return fail(WW_EINVAL, "tuning: minv_wgs out of range");
  if (t->blu_strip < 1 || t->blu_strip > BLU_STRIP_MAX) return fail(WW_EINVAL, "tuning: blu_strip out of range");
  if (t->dtn_rows < 4 || t->dtn_rows > 32 || t->dtn_rows % 4) return fail(WW_EINVAL, "tuning: dtn_rows out of range");
  if (t->gemm_split != 2 && t->gemm_split != 4) return fail(WW_EINVAL, "tuning: gemm_split must be 2 or 4");
  if (t->asm_cw != 16 && t->asm_cw != 32) return fail(WW_EINVAL, "tuning: asm_cw must be 16 or 32");
  if (t->gemm_rows != 16 && t->gemm_rows != 32) return fail(WW_EINVAL, "tuning: gemm_rows must be 16 or 32");
  if (t->lag_fp32 != 0 && t->lag_fp32 != 1) return fail(WW_EINVAL, "tuning: lag_fp32 must be 0 or 1");
  if (t->lag_sweeps < 1 || t->lag_sweeps > 8) return fail(WW_EINVAL, "tuning: lag_sweeps out of range");
  c->lag = t->lag;
  c->lu_group = t->lu_group;
  c->nlus = t->lu_streams;
  c->graph_parts = t->graph_parts;
  c->minv_wgs = t->minv_wgs;
  c->blu_strip = t->blu_strip;
  c->dtn_rows = t->dtn_rows;
  c->gemm_split = t->gemm_split;
  c->gemm_rows = t->gemm_rows;
  c->lag32 = t->lag_fp32;
  c->asm_cw = t->asm_cw;
  c->nref_lag = t->lag_sweeps;
  ++c->tune_gen;
  return 0;
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
static BluBufs<T> blu_bufs(ww_ctx* c, T* A, T* X, T* Z, T* V, T* D, double guard) {
  BluBufs<T> b;
  b.A = A;
  b.X = X;
  b.Z = Z;
  b.V = V;
  b.Dinv = D;
  b.Xr = nullptr;   // the solves use the explicit inverse (k_minv), not row-major factors
  b.Zr = nullptr;
  b.status = c->status;
  b.Np = c->Np;
  b.pivguard = guard;
  return b;
}

// measurement hook: a pair of HIP events attached to one kernel dispatch on the current
// stream (hipExtLaunchKernel: the events take the dispatch's own start and end times),
// only inside a march step, where the phase marks are taken too, outside stream capture,
// and at most KEV_MAX pairs per profiled interval; *a = *b = null when off
static const size_t KEV_MAX = 1u << 14;
static int kev_pair(ww_ctx* c, hipEvent_t* a, hipEvent_t* b) {
  *a = *b = nullptr;
  if (!c->prof_kev || c->prof_stage < 0 || c->kev_n >= KEV_MAX) return 0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(c->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return 0;
  if (c->kev_n == c->kev_a.size()) {
    hipEvent_t ea = nullptr, eb = nullptr;
    HIPCHK(hipEventCreate(&ea));
    const hipError_t e = hipEventCreate(&eb);
    if (e != hipSuccess) {
      (void)hipEventDestroy(ea);
      HIPCHK(e);
    }
    c->kev_a.push_back(ea);
    c->kev_b.push_back(eb);
  }
  *a = c->kev_a[c->kev_n];
  *b = c->kev_b[c->kev_n];
  return 0;
}

template <typename T>
static int enqueue_blu(ww_ctx* c, const BluGroup<T>& g) {
  const int nb = c->Np / WW_TB;
  const size_t es = sizeof(T);
  int rc;
  hipLaunchKernelGGL(k_blu_init<T>, dim3(g.count), dim3(WW_NT), (TILE_DBL + GJ_SCR) * es, c->stream, g);
  LAUNCHCHK();
  for (int k = 0; k + 1 < nb; ++k) {
    const int nblk = blu_step_tasks(nb, k, g.strip);
    hipEvent_t ea, eb;
    if ((rc = kev_pair(c, &ea, &eb))) return rc;
    if (ea) {
      BluGroup<T> ga = g;
      int ka = k;
      void* args[] = {&ga, &ka};
      HIPCHK(hipExtLaunchKernel(reinterpret_cast<const void*>(&k_blu_step<T>), dim3(nblk * g.count), dim3(WW_NT),
                                args, 2 * TILE_DBL * es, c->stream, ea, eb, 0));
      ++c->kev_n;
    } else {
      hipLaunchKernelGGL(k_blu_step<T>, dim3(nblk * g.count), dim3(WW_NT), 2 * TILE_DBL * es, c->stream, g, k);
    }
    LAUNCHCHK();
  }
  if (nb > 1) {
    hipLaunchKernelGGL(k_blu_final<T>, dim3((nb - 1) * g.count), dim3(WW_NT), 2 * TILE_DBL * es, c->stream, g);
    LAUNCHCHK();
  }
  return 0;
}

// profiling mark (only while a profiled step is being enqueued)
static int prof_mark(ww_ctx* c, int phase, int which) {
  if (!c->prof || c->prof_stage < 0) return 0;
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, c->stream, c->stamps, phase * 16 + c->prof_stage, which);
  LAUNCHCHK();
  return 0;
}

static bool mixed(const ww_ctx* c) { return (c->flags & WW_MIXED) != 0; }
static bool strict(const ww_ctx* c) { return (c->flags & WW_STRICT) != 0; }
// FP32 factors in the mixed form, except after the FP64 or the pivoting fallback (the
// fallback to each stage's own factors keeps the precision form)
static bool use32(const ww_ctx* c) { return mixed(c) && !(c->fb & (WW_FB_FP64 | WW_FB_PIVOTED)); }
static bool pivoted(const ww_ctx* c) { return (c->fb & WW_FB_PIVOTED) != 0; }
// pivot bound of the pivoted factorisation (near singularity)
static const double PIVOTED_GUARD = 1e-8;

// The FP64 factor set of one stage: A (overwritten by the Schur complements), Gm, the
// block-triangular inverses X, Z, and the scratch V, Dinv.  The adjoint keeps one set
// per stage of a segment; everything else uses the context's set.
struct Fac {
  double *A, *Gm, *X, *Z, *V, *Dinv;
  bool use32;   // mixed precision: factor the FP32 copy and refine the solves
  float *A32, *X32, *Z32, *V32, *Dinv32;
  double* aux;    // per-point base arrays of the stage
  // row-major arrays: Mi = A^{-1} from the FP64 factors, Mi32 from the FP32 factors
  // (every solve is one product with it), Gm, and the FP64 A of the residuals
  double *Mi, *Gmr, *Ar;
  float* Mi32;
  int* perm;   // partial-pivoting row order of this set, or null (no interchanges)
  bool lag32 = false;   // FP64 factors whose lagged solves read the FP32 copy Mi32 of Mi
};
// factor set of parity `p`; `cols` selects the column chain's GEMM partials
static Fac fac_set(ww_ctx* c, int p, bool cols) {
  Fac F;
  if (p == 0) {
    F = Fac{c->A, c->Gm, c->Xi, c->Zi, c->Vi, c->Dinv, use32(c), c->A32, c->X32, c->Z32, c->V32, c->Dinv32, c->aux,
            nullptr};
  } else {
    F = Fac{c->A_1, c->Gm_1, c->Xi_1, c->Zi_1, c->Vi_1, c->Dinv_1, use32(c), c->A32_1, c->X32_1, c->Z32_1, c->V32_1,
            c->Dinv32_1, c->aux_1, nullptr};
  }
  F.Mi = p ? c->Mi_1 : c->Mi;
  F.Gmr = p ? c->Gmr_1 : c->Gmr;
  F.Ar = p ? c->Ar_1 : c->Ar;
  F.Mi32 = p ? c->Mi32_1 : c->Mi32;
  F.perm = pivoted(c) ? c->perm : nullptr;
  return F;
}

// buffers of the pivoting fallback (first use)
static int ensure_pivot_buffers(ww_ctx* c) {
  if (c->perm) return 0;
  int rc;
  const size_t np = c->np_max;
  if ((rc = dalloc(c, (void**)&c->perm, np * sizeof(int)))) return rc;
  if ((rc = dalloc(c, (void**)&c->pw, np * np * 8))) return rc;
  return dalloc(c, (void**)&c->pb, np * (size_t)c->r_max * 8);
}

// Row order of partial pivoting for the assembled A of F (column-major, ld Np), then
// A := P A.  Elimination runs on a copy in the workspace; the padding rows keep their
// place (the padding of A is the identity).
static int enqueue_pivot_order(ww_ctx* c, const Fac& F) {
  const int N = c->N, Np = c->Np;
  const int cblk = (int)std::min<size_t>(((size_t)Np * Np + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_copy, dim3(cblk), dim3(256), 0, c->stream, F.A, Np, c->pw, Np, Np, Np, Np);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_iota, dim3((Np + 255) / 256), dim3(256), 0, c->stream, F.perm, Np);
  LAUNCHCHK();
  for (int k = 0; k < N; ++k) {
    hipLaunchKernelGGL(k_plu_pivot, dim3(1), dim3(PLU_NT), 0, c->stream, c->pw, Np, N, k, F.perm, PIVOTED_GUARD,
                       c->status);
    LAUNCHCHK();
    const int n = N - k - 1;
    if (n > 0) {
      hipLaunchKernelGGL(k_plu_update, dim3((n + 63) / 64, (n + 15) / 16), dim3(256), 0, c->stream, c->pw, Np, N, k);
      LAUNCHCHK();
    }
  }
  hipLaunchKernelGGL(k_permute_rows, dim3(cblk), dim3(256), 0, c->stream, F.A, c->pw, F.perm, Np, Np, 0);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_pad_copy, dim3(cblk), dim3(256), 0, c->stream, c->pw, Np, F.A, Np, Np, Np, Np);
  LAUNCHCHK();
  return 0;
}
static Fac fac_default(ww_ctx* c) { return fac_set(c, 0, false); }

// assembly of A, Gm (and the row-major FP64 copy Ar when the solves refine: mixed
// mode, or lagged factors)
// The lagged inverse Fo (optional): the same launch forms x0 = Fo.Mi psi (the first
// solve of a lagged-factor base chain) in 16 more rows of workgroups.
static int enqueue_assemble(ww_ctx* c, const Fac& F, bool want_ar, const Fac* Fo = nullptr,
                            const double* psi = nullptr, double* x0 = nullptr) {
  const int nb = c->Np / WW_TB;
  const bool f32 = Fo && (Fo->use32 || Fo->lag32);
  const double* mx64 = (Fo && !f32) ? Fo->Mi : nullptr;
  const float* mx32 = f32 ? Fo->Mi32 : nullptr;
  if (Fo && !(mx64 || mx32)) return fail(WW_EHIP, "internal: lagged first solve without its inverse");
  if (c->mapped) {
    hipLaunchKernelGGL(k_assemble_map, dim3(nb, c->Np / 16 + (Fo ? 16 : 0)), dim3(WW_NT), 0, c->stream, F.aux,
                       c->mesh, c->n_max, c->c0T, F.A, F.Gm, F.use32 ? F.A32 : nullptr, F.Gmr,
                       (F.use32 || want_ar) ? F.Ar : nullptr, c->N, c->Np, c->finite, mx64, mx32, psi, x0);
    LAUNCHCHK();
    return 0;
  }
  const int cw = c->asm_cw == 32 ? 32 : 16;
  const int gy = c->Np / cw + (Fo ? 16 : 0);
  hipLaunchKernelGGL(cw == 32 ? k_assemble<32> : k_assemble<16>, dim3(nb, gy), dim3(WW_NT), 0, c->stream, F.aux,
                     c->n_max, c->cosT, c->sinT, c->c0T, F.A, F.Gm, F.use32 ? F.A32 : nullptr, F.Gmr,
                     (F.use32 || want_ar) ? F.Ar : nullptr, c->N, c->Np, c->finite, mx64, mx32, psi, x0);
  LAUNCHCHK();
  return 0;
}

// block LU of A (FP64, or of the FP32 copy in mixed mode) with the block-triangular
// inverses and the explicit inverse Mi = Z (I + X); with a row order, first the
// partial-pivoting order and A := P A.  A group (count > 1: consecutive stages of a
// lagged-factor march, never pivoted) shares every launch of the sequence.
static int minv_grid(const ww_ctx* c, int ntask) { return std::max(1, std::min(ntask, c->minv_wgs)); }

static int enqueue_lu_group(ww_ctx* c, const Fac* F, int count) {
  int rc;
  if (count < 1 || count > BLU_GMAX) return fail(WW_EHIP, "internal: LU group size");
  if ((rc = prof_mark(c, 0, 0))) return rc;
  if (count == 1 && F[0].perm && (rc = enqueue_pivot_order(c, F[0]))) return rc;
  const int nb = c->Np / WW_TB;
  if (F[0].use32) {
    BluGroup<float> g{};
    MinvGroup<float> mg{};
    for (int q = 0; q < count; ++q) {
      if (!F[q].Mi32) return fail(WW_EHIP, "internal: LU without its inverse buffer");
      g.m[q] = blu_bufs<float>(c, F[q].A32, F[q].X32, F[q].Z32, F[q].V32, F[q].Dinv32, c->guard);
      mg.Z[q] = F[q].Z32;
      mg.X[q] = F[q].X32;
      mg.Mr[q] = F[q].Mi32;
    }
    g.count = count;
    g.strip = c->blu_strip;
    if ((rc = enqueue_blu<float>(c, g))) return rc;
    mg.count = count;
    hipLaunchKernelGGL(k_minv<float>, dim3(minv_grid(c, nb * nb * count)), dim3(WW_NT), 2 * TILE_DBL * sizeof(float),
                       c->stream, mg, c->Np);
  } else {
    BluGroup<double> g{};
    MinvGroup<double> mg{};
    for (int q = 0; q < count; ++q) {
      if (!F[q].Mi) return fail(WW_EHIP, "internal: LU without its inverse buffer");
      g.m[q] = blu_bufs<double>(c, F[q].A, F[q].X, F[q].Z, F[q].V, F[q].Dinv, F[q].perm ? PIVOTED_GUARD : c->guard);
      mg.Z[q] = F[q].Z;
      mg.X[q] = F[q].X;
      mg.Mr[q] = F[q].Mi;
      mg.Mr32[q] = F[q].lag32 ? F[q].Mi32 : nullptr;
    }
    g.count = count;
    g.strip = c->blu_strip;
    if ((rc = enqueue_blu<double>(c, g))) return rc;
    mg.count = count;
    hipLaunchKernelGGL(k_minv<double>, dim3(minv_grid(c, nb * nb * count)), dim3(WW_NT), 2 * TILE_DBL * sizeof(double),
                       c->stream, mg, c->Np);
  }
  LAUNCHCHK();
  return prof_mark(c, 0, 1);
}
static int enqueue_lu(ww_ctx* c, const Fac& F) { return enqueue_lu_group(c, &F, 1); }

static int enqueue_assemble_lu(ww_ctx* c, const Fac& F) {
  int rc;
  if ((rc = enqueue_assemble(c, F, false))) return rc;
  return enqueue_lu(c, F);
}

// out = add + sgn * M B for R columns (ld Np) with the row-major M (element type T).
// One column: one wave per row (mode: the 64-block range, 0 all, 1 strictly lower, 2
// upper with the diagonal); several: 32 x 32 output tiles over the whole inner
// dimension (the full matrix).
template <typename T>
static int enqueue_gemm(ww_ctx* c, const T* Mr, int mode, const double* B, const double* add, double sgn,
                        double* out, int R) {
  if (!Mr) return fail(WW_EHIP, "internal: product without its matrix");
  if (R == 1) {
    hipLaunchKernelGGL(k_gemv_row<T>, dim3(c->Np * 64 / WW_NT), dim3(WW_NT), 0, c->stream, Mr, c->Np, mode, B, add,
                       sgn, out);
    LAUNCHCHK();
    return 0;
  }
  if (mode & 3) return fail(WW_EHIP, "internal: triangular product of several columns");
  const dim3 g32(c->Np / GT, (R + GT - 1) / GT), g16(c->Np / 16, (R + GT - 1) / GT);
  if (c->gemm_rows == 16) {
    if (c->gemm_split == 2)
      hipLaunchKernelGGL((k_gemm_rm<T, 2, 16>), g16, dim3(256), 0, c->stream, Mr, c->Np, B, R, add, sgn, out);
    else
      hipLaunchKernelGGL((k_gemm_rm<T, 4, 16>), g16, dim3(512), 0, c->stream, Mr, c->Np, B, R, add, sgn, out);
  } else {
    if (c->gemm_split == 2)
      hipLaunchKernelGGL((k_gemm_rm<T, 2, 32>), g32, dim3(512), 0, c->stream, Mr, c->Np, B, R, add, sgn, out);
    else
      hipLaunchKernelGGL((k_gemm_rm<T, 4, 32>), g32, dim3(1024), 0, c->stream, Mr, c->Np, B, R, add, sgn, out);
  }
  LAUNCHCHK();
  return 0;
}

// Convergence test of the mixed-precision refinement: per column, the FP64 residual
// of the final solution must be at most 2^-43 of the right-hand side (max norm); the
// solution's relative error is then at most about cond(A) * 2^-43.
static const double REFINE_TOL = 1.1368683772161603e-13;

// X = A^{-1} B for R columns (ld Np); Rs is scratch; B is kept.  Mi is the explicit
// inverse Z (I + X) of the block LU (row-major).
// FP64:  X = Mi B.
// mixed: X = Mi32 B, then nref sweeps of  r = B - A X (FP64 residual with the FP64
//        matrix),  X += Mi32 r  (FP32 inverse, FP64 accumulation).
static int enqueue_solve(ww_ctx* c, const Fac& F, double* B, double* Y, double* X, double* Rs, int R) {
  (void)Y;
  int rc;
  if (F.perm) {   // P A = Lt Ut: solve with P B
    const size_t n = (size_t)c->Np * R;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_permute_rows, dim3(blocks), dim3(256), 0, c->stream, B, c->pb, F.perm, c->Np, R, 0);
    LAUNCHCHK();
    B = c->pb;
  }
  if (!F.use32) return enqueue_gemm<double>(c, F.Mi, 0, B, nullptr, 1.0, X, R);
  if ((rc = enqueue_gemm<float>(c, F.Mi32, 0, B, nullptr, 1.0, X, R))) return rc;
  for (int it = 0; it < c->nref; ++it) {
    if ((rc = enqueue_gemm<double>(c, F.Ar, 0, X, B, -1.0, Rs, R))) return rc;
    if ((rc = enqueue_gemm<float>(c, F.Mi32, 0, Rs, X, 1.0, X, R))) return rc;
  }
  {
    // convergence test on the FP64 residual of the final solution (also with no sweep)
    if ((rc = enqueue_gemm<double>(c, F.Ar, 0, X, B, -1.0, Rs, R))) return rc;
    hipLaunchKernelGGL(k_refine_check, dim3(R), dim3(WW_NT), 0, c->stream, Rs, B, c->Np, c->N, REFINE_TOL,
                       c->status, 4);
    LAUNCHCHK();
  }
  return 0;
}

// DtN of R columns in B (ld Np): out = G psi (ld Np); mu in Mu; Rs residual scratch
static int enqueue_dtn_cols(ww_ctx* c, const Fac& F, double* B, double* Yt, double* Mu, double* Gam, double* HGm,
                            double* out, double* Rs, int R) {
  int rc;
  if ((rc = enqueue_solve(c, F, B, Yt, Mu, Rs, R))) return rc;
  hipLaunchKernelGGL(k_gamma, dim3((R + 1) / 2), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, Mu, c->Np, R, Gam,
                     HGm, c->tw, c->N, nullptr, nullptr, 0.0, nullptr, 0);
  LAUNCHCHK();
  return enqueue_gemm<double>(c, F.Gmr, 0, Gam, HGm, 1.0, out, R);
}

static size_t kstride(const ww_ctx* c) { return (size_t)2 * c->N * (c->M + 1); }



static int ensure_gmres(ww_ctx* c) {
  int rc;
  const size_t np = c->np_max, m = GM_MAXM;
  // the row-major FP64 A that GMRES multiplies by (allocated with the mixed form only)
  if (!c->Ar && (rc = dalloc(c, (void**)&c->Ar, np * np * 8))) return rc;
  if (!c->Ar_1 && (rc = dalloc(c, (void**)&c->Ar_1, np * np * 8))) return rc;
  if (c->gmV) return 0;
  if ((rc = dalloc(c, (void**)&c->gmV, np * (m + 1) * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->gmw, np * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->gmH, (m + 1) * m * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->gmcs, m * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->gmsn, m * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->gmg, (m + 1) * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->gmbeta, 8))) return rc;
  return dalloc(c, (void**)&c->gmstate, 64);
}

// Convergence bound of the GMRES residual estimate (relative to ||psi||)
static const double GMRES_TOL = 1e-15;

// mu = A^{-1} psi by GMRES with the row-major Ar of F (one cycle of gm_m steps, see
// ww_gmres.hpp), then the FP64 residual test of the mixed form (status bit 64)
static int enqueue_gmres(ww_ctx* c, const Fac& F, double* psi, double* mu, double* rs) {
  if (!F.Ar || !c->gmV || !c->gmstate) return fail(WW_EHIP, "internal: GMRES buffers missing");
  GmBufs b;
  b.Ar = F.Ar;
  b.Np = c->Np;
  b.N = c->N;
  b.m = c->gm_m;
  b.V = c->gmV;
  b.w = c->gmw;
  b.H = c->gmH;
  b.cs = c->gmcs;
  b.sn = c->gmsn;
  b.g = c->gmg;
  b.beta = c->gmbeta;
  b.state = c->gmstate;
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(GM_NT), 0, c->stream, b, (const double*)psi);
  LAUNCHCHK();
  const int rows_per = GM_NT / 64;
  for (int k = 0; k < b.m; ++k) {
    hipLaunchKernelGGL(k_gm_matvec, dim3((c->N + rows_per - 1) / rows_per), dim3(GM_NT), 0, c->stream, b, k);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_gm_arnoldi, dim3(1), dim3(GM_NT), 0, c->stream, b, k, GMRES_TOL);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_gm_finish, dim3(1), dim3(GM_NT), 0, c->stream, b, mu);
  LAUNCHCHK();
  int rc;
  if ((rc = enqueue_gemm<double>(c, F.Ar, 0, mu, psi, -1.0, rs, 1))) return rc;
  hipLaunchKernelGGL(k_refine_check, dim3(1), dim3(WW_NT), 0, c->stream, rs, psi, c->Np, c->N, REFINE_TOL, c->status,
                     64);
  LAUNCHCHK();
  return 0;
}

static int read_status(ww_ctx* c, int* st, int* where = nullptr);

// Step budget of a GMRES march: one solve of a rough right-hand side with the largest
// budget on the surface at the start of the march, then the steps it took plus 4 (the operator changes slowly along
// the march; a stage that needs more fails the residual test and the march falls back
// to LU factors).
static int gmres_calibrate(ww_ctx* c) {
  const Fac F = fac_default(c);
  hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->y, c->K, c->Ys, c->coef,
                     0, kstride(c), F.aux, c->n_max, c->rhs0, c->Np, c->tw, c->N, c->hsurf, c->status);
  LAUNCHCHK();
  int rc;
  if ((rc = enqueue_assemble(c, F, true))) return rc;
  // a rough right-hand side (the initial potential is often zero, which GMRES solves in
  // no step)
  hipLaunchKernelGGL(k_gm_probe_rhs, dim3((c->Np + 255) / 256), dim3(256), 0, c->stream, c->y0t, c->N, c->Np);
  LAUNCHCHK();
  c->gm_m = GM_MAXM;
  if ((rc = enqueue_gmres(c, F, c->y0t, c->mu0, c->rr0))) return rc;
  int used[2] = {0, 0}, st = 0;
  HIPCHK(hipMemcpyAsync(used, c->gmstate, sizeof(used), hipMemcpyDeviceToHost, c->stream));
  if ((rc = read_status(c, &st))) return rc;   // (synchronises; the march checks again)
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  c->gm_m = std::max(4, std::min(GM_MAXM, used[1] + 4));
  return 0;
}

// base chain of stage s: prep, assembly, LU, base DtN, base right-hand side -> kout
// (GMRES marches: assembly and a GMRES solve in place of the LU and its solve)
static int enqueue_base_chain(ww_ctx* c, const double* ysrc, int s, double* kout, const Fac& F) {
  int rc;
  if ((rc = prof_mark(c, 1, 0))) return rc;
  hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, ysrc, c->K, c->Ys, c->coef,
                     s, kstride(c), F.aux, c->n_max, c->rhs0, c->Np, c->tw, c->N, c->hsurf, c->status);
  LAUNCHCHK();
  if (c->gm_active) {
    if ((rc = enqueue_assemble(c, F, true))) return rc;
    if ((rc = enqueue_gmres(c, F, c->rhs0, c->mu0, c->rr0))) return rc;
    hipLaunchKernelGGL(k_gamma, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->mu0, c->Np, 1, c->gam0,
                       c->hg0, c->tw, c->N, nullptr, nullptr, 0.0, nullptr, 0);
    LAUNCHCHK();
    if ((rc = enqueue_gemm<double>(c, F.Gmr, 0, c->gam0, c->hg0, 1.0, c->gphi0, 1))) return rc;
  } else {
    if ((rc = enqueue_assemble_lu(c, F))) return rc;
    if ((rc = enqueue_dtn_cols(c, F, c->rhs0, c->y0t, c->mu0, c->gam0, c->hg0, c->gphi0, c->rr0, 1))) return rc;
  }
  if (c->mapped)
    hipLaunchKernelGGL(k_base_rhs_map, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->gphi0,
                       F.aux, c->mesh, c->n_max, kout, (unsigned long long*)nullptr, 0.0, (int*)nullptr, c->tw,
                       c->sig, c->N, c->g, c->tau);
  else
    hipLaunchKernelGGL(k_base_rhs, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->gphi0, F.aux,
                       c->n_max, kout, (unsigned long long*)nullptr, 0.0, (int*)nullptr, c->tw, c->sig, c->N, c->g,
                       c->tau);
  LAUNCHCHK();
  return prof_mark(c, 1, 1);
}

static int enqueue_col_chain(ww_ctx* c, int s, const Fac& F) {
  int rc;
  if ((rc = prof_mark(c, 2, 0))) return rc;
  const int M = c->M;
  const size_t tot = (size_t)c->Np * M;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_col_pre, dim3(blocks), dim3(256), 0, c->stream, c->y, c->K, c->Ys, c->coef, s, kstride(c),
                     F.aux, c->n_max, c->Psi, c->Np, c->N, M);
  LAUNCHCHK();
  if ((rc = enqueue_dtn_cols(c, F, c->Psi, c->Ytmp, c->Mu, c->Gam, c->HG, c->Gpsi, c->Rr, M))) return rc;
  if (c->mapped)
    hipLaunchKernelGGL(k_col_rhs_map, dim3(M), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->Gpsi,
                       c->Np, F.aux, c->mesh, c->n_max, c->K + (size_t)s * kstride(c), c->tw, c->sig, c->N, c->g,
                       c->tau);
  else
    hipLaunchKernelGGL(k_col_rhs, dim3(M), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->Gpsi, c->Np,
                       F.aux, c->n_max, c->K + (size_t)s * kstride(c), c->tw, c->sig, c->N, c->g, c->tau);
  LAUNCHCHK();
  return prof_mark(c, 2, 1);
}

// ----- lagged-factor pipeline -----
// A changes little between nearby stages (a second-kind operator of a surface that
// moves by O(dt)): with the factors of stage s - lag, one refinement sweep with the
// FP64 residual of stage s's own matrix already reaches the rounding level.  The base
// chain (the march's critical path) therefore solves with lagged factors while the
// LU of its own matrix runs concurrently; the column chain, which lags behind anyway,
// uses the exact factors of its stage.
static bool pipelined(const ww_ctx* c, bool cols, bool two_streams) {
  (void)cols;   // with or without Jacobian columns (c->pcols)
  return c->lag > 0 && two_streams && c->fb == 0 && c->nst > c->lag && !c->gm_active;
}

// a march without columns keeps to two LU streams: they carry its LUs, and a third
// concurrent LU only slows its base chain
static int lu_count(const ww_ctx* c) { return std::min(c->pcols ? c->nlus : std::min(c->nlus, 2), c->lag); }
// LU groups: consecutive stages g G .. g G + G - 1 (the last group of a step may be
// shorter) are factored by one launch sequence, on LU stream g mod (LU streams); the
// group is at most the lag, so that a base solve never waits for its own group
static int lu_group(const ww_ctx* c) { return std::max(1, std::min(c->lu_group, c->lag)); }
static int grp_first(const ww_ctx* c, int s) { return s / lu_group(c) * lu_group(c); }
static int grp_last(const ww_ctx* c, int s) { return std::min(c->nst, grp_first(c, s) + lu_group(c)) - 1; }
static hipStream_t lu_stream(const ww_ctx* c, int s) { return c->lus[(s / lu_group(c)) % lu_count(c)]; }

// the first n factor sets of the ring (each for n_max)
static int ensure_ring(ww_ctx* c, int n) {
  int rc;
  const size_t np = c->np_max, nn = np * np;
  const size_t nbm = np / WW_TB;
  while (c->ring_n < n) {
    RingSet& r = c->ring[c->ring_n];
    double** d[] = {&r.A, &r.Gm, &r.X, &r.Z, &r.V, &r.Mi, &r.Gmr, &r.Ar};
    for (double** q : d)
      if ((rc = dalloc(c, (void**)q, nn * 8))) return rc;
    if ((rc = dalloc(c, (void**)&r.Dinv, nbm * 4096 * 8))) return rc;
    if ((rc = dalloc(c, (void**)&r.aux, (size_t)AUX_COUNT * c->n_max * 8))) return rc;
    if ((rc = dalloc(c, (void**)&r.Mi32, nn * 4))) return rc;   // also the FP64 form's FP32 copy
    if (mixed(c)) {
      float** f[] = {&r.A32, &r.X32, &r.Z32, &r.V32};
      for (float** q : f)
        if ((rc = dalloc(c, (void**)q, nn * 4))) return rc;
      if ((rc = dalloc(c, (void**)&r.Dinv32, nbm * 4096 * 4))) return rc;
    }
    ++c->ring_n;
  }
  return 0;
}

static int ensure_pipe(ww_ctx* c) {
  for (int i = 0; i < lu_count(c); ++i)
    if (!c->lus[i]) HIPCHK(hipStreamCreateWithFlags(&c->lus[i], hipStreamNonBlocking));
  for (int i = 0; i < 16; ++i) {
    if (!c->evA[i]) HIPCHK(hipEventCreateWithFlags(&c->evA[i], hipEventDisableTiming));
    if (!c->evL[i]) HIPCHK(hipEventCreateWithFlags(&c->evL[i], hipEventDisableTiming));
  }
  if (!c->evE) HIPCHK(hipEventCreateWithFlags(&c->evE, hipEventDisableTiming));
  return ensure_ring(c, c->nst);
}

static Fac pipe_set(ww_ctx* c, int s, bool cols) {
  const RingSet& r = c->ring[s];
  Fac F = Fac{r.A, r.Gm, r.X, r.Z, r.V, r.Dinv, use32(c), r.A32, r.X32, r.Z32, r.V32, r.Dinv32, r.aux, nullptr};
  F.Mi = r.Mi;
  F.Gmr = r.Gmr;
  F.Ar = r.Ar;
  F.Mi32 = r.Mi32;
  F.perm = nullptr;
  F.lag32 = c->lag32 && !F.use32 && r.Mi32;
  return F;
}

// Before the first step: the factors of the initial surface in the sets that the first
// `lag` stages read (those of the last stages of a previous step).
static int pipe_prologue(ww_ctx* c) {
  int rc;
  const int nst = c->nst, L = c->lag;
  const Fac P0 = pipe_set(c, nst - L, false);
  hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->y, c->K, c->Ys, c->coef,
                     0, kstride(c), P0.aux, c->n_max, c->rhs0, c->Np, c->tw, c->N, c->hsurf, c->status);
  LAUNCHCHK();
  if ((rc = enqueue_assemble(c, P0, true))) return rc;
  if ((rc = enqueue_lu(c, P0))) return rc;
  const size_t nn = (size_t)c->Np * c->Np;
  for (int q = nst - L + 1; q < nst; ++q) {
    const RingSet &a = c->ring[nst - L], &b = c->ring[q];
    if (use32(c) || P0.lag32)
      HIPCHK(hipMemcpyAsync(b.Mi32, a.Mi32, nn * 4, hipMemcpyDeviceToDevice, c->stream));
    if (!use32(c))
      HIPCHK(hipMemcpyAsync(b.Mi, a.Mi, nn * 8, hipMemcpyDeviceToDevice, c->stream));
  }
  // the first step of the per-branch graphs waits, at stage s, for the column chain of
  // stage s and the LU of stage s - lag of the step before: here, for this prologue
  for (int q = 0; q < nst; ++q) {
    HIPCHK(hipEventRecord(c->evC[q], c->stream));
    HIPCHK(hipEventRecord(c->evL[q], c->stream));
  }
  HIPCHK(hipEventRecord(c->evE, c->stream));
  return 0;
}

// The parts of stage s of the lagged-factor march, each captured alone: 0 spectral prep
// and assembly (main stream), 1 the LU of the stage (LU stream s % lag), 2 the lagged
// base solve to the base right-hand side (main), 3 the column chain (side stream).
enum { PP_PREP = 0, PP_LU = 1, PP_BASE = 2, PP_COL = 3 };

static int enqueue_pipe_part(ww_ctx* c, int s, int part) {
  const int nst = c->nst, L = c->lag;
  const Fac F = pipe_set(c, s, false);
  int rc = 0;
  const Fac Fo = pipe_set(c, (s - L + nst) % nst, false);   // the lagged factor set
  if (part == PP_PREP) {
    // spectral prep; assembly, and in the same launch the first lagged solve
    // x0 = Mi_old psi, which does not need this stage's matrix
    if ((rc = prof_mark(c, 1, 0))) return rc;
    if (s == 0) {   // later stages are prepared by the base chain of the stage before
      hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->y, c->K, c->Ys,
                         c->coef, s, kstride(c), F.aux, c->n_max, c->rhs0, c->Np, c->tw, c->N, c->hsurf, c->status);
      LAUNCHCHK();
    }
    // the march reads Gm only row-major (base and column chains): no column-major copy
    Fac Fa = F;
    Fa.Gm = nullptr;
    return enqueue_assemble(c, Fa, true, &Fo, c->rhs0, c->mu0);
  }
  if (part == PP_LU) {
    // the group that ends at this stage (stages of a group are never pivoted)
    if (s != grp_last(c, s)) return 0;
    const int f = grp_first(c, s);
    Fac Fs[BLU_GMAX];
    for (int q = f; q <= s; ++q) Fs[q - f] = pipe_set(c, q, false);
    return enqueue_lu_group(c, Fs, s - f + 1);
  }
  if (part == PP_BASE) {
    // refinement sweeps against this stage's matrix: r = psi - A x, x += Mi_old r
    const int nref = c->nref_lag >= 0 ? c->nref_lag : c->nref;
    for (int it = 0; it < nref; ++it) {
      if ((rc = enqueue_gemm<double>(c, F.Ar, 0, c->mu0, c->rhs0, -1.0, c->rr0, 1))) return rc;
      rc = (Fo.use32 || Fo.lag32) ? enqueue_gemm<float>(c, Fo.Mi32, 0, c->rr0, c->mu0, 1.0, c->mu0, 1)
                    : enqueue_gemm<double>(c, Fo.Mi, 0, c->rr0, c->mu0, 1.0, c->mu0, 1);
      if (rc) return rc;
    }
    // gamma, (1/2) H gamma, G phi and the residual of the convergence test in one
    // launch; the test's decision is taken at the start of k_base_rhs
    unsigned long long* chk = (unsigned long long*)(c->status + 4);
    hipLaunchKernelGGL(c->N <= 1024 ? k_base_dtn<16> : k_base_dtn<WW_NMAX / 64>,
                       dim3((c->Np + c->dtn_rows - 1) / c->dtn_rows), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream,
                       c->mu0, c->rhs0, F.Gmr, F.Ar, c->Np, c->tw, c->N, c->gphi0, chk, c->dtn_rows);
    LAUNCHCHK();
    if (s + 1 < nst && c->mapped) {
      const Fac Fn = pipe_set(c, s + 1, false);
      hipLaunchKernelGGL(k_base_rhs_prep_map, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->gphi0,
                         F.aux, c->K + (size_t)s * kstride(c), chk, REFINE_TOL, c->sig, c->g, c->tau, c->y, c->K,
                         c->Ys, c->coef, s + 1, kstride(c), Fn.aux, c->rhs0, c->Np, c->hsurf, c->n_max, c->tw, c->N,
                         c->status, c->mesh);
    } else if (c->mapped) {
      hipLaunchKernelGGL(k_base_rhs_map, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->gphi0,
                         F.aux, c->mesh, c->n_max, c->K + (size_t)s * kstride(c), chk, REFINE_TOL, c->status, c->tw,
                         c->sig, c->N, c->g, c->tau);
    } else if (s + 1 < nst) {
      // this stage's right-hand side and the next stage's prep in one launch
      const Fac Fn = pipe_set(c, s + 1, false);
      hipLaunchKernelGGL(k_base_rhs_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->gphi0, F.aux,
                         c->K + (size_t)s * kstride(c), chk, REFINE_TOL, c->sig, c->g, c->tau, c->y, c->K, c->Ys,
                         c->coef, s + 1, kstride(c), Fn.aux, c->rhs0, c->Np, c->hsurf, c->n_max, c->tw, c->N,
                         c->status);
    } else {
      hipLaunchKernelGGL(k_base_rhs, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, c->Ys, c->gphi0, F.aux,
                         c->n_max, c->K + (size_t)s * kstride(c), chk, REFINE_TOL, c->status, c->tw, c->sig, c->N,
                         c->g, c->tau);
    }
    LAUNCHCHK();
    return prof_mark(c, 1, 1);
  }
  return enqueue_col_chain(c, s, pipe_set(c, s, true));
}

// the step end of the base column (cols false; it counts the step) or of the Jacobian
// columns 1..M (cols true)
static int enqueue_pipe_end(ww_ctx* c, bool cols) {
  hipLaunchKernelGGL(k_step_end, dim3(cols ? c->M : 1), dim3(WW_NT), fft_lds_bytes(c->N, 3), c->stream, c->y, c->K,
                     kstride(c), c->nst, c->coef, c->tw, c->sig, c->N, cols ? 1 : 0, cols ? nullptr : c->status);
  LAUNCHCHK();
  return 0;
}

// capture one part on the capture stream, alone (part -1: the step end of the base
// column, -2: that of the Jacobian columns)
static int capture_part(ww_ctx* c, int s, int part, hipGraphExec_t* out) {
  hipStream_t user = c->stream;
  const hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) return fail(WW_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(eb));
  c->stream = c->cap_stream;
  c->prof_stage = part < 0 ? -1 : s;
  const int rc = part < 0 ? enqueue_pipe_end(c, part == -2) : enqueue_pipe_part(c, s, part);
  c->prof_stage = -1;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  c->stream = user;
  if (rc) {
    if (e == hipSuccess && g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIPCHK(e);
  const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(ei);
  return 0;
}

static long long pipe_key(const ww_ctx* c) {
  return ((((((((long long)c->N * 4096 + c->M) * 32 + c->nst) * 16 + c->lag) * 8 + lu_group(c)) * 2 + (c->prof ? 1 : 0)) *
              16 + c->fb) * 1024 + (c->tune_gen & 1023)) * 2 + (c->mapped ? 1 : 0);
}

static int ensure_pipe_graphs(ww_ctx* c) {
  int rc;
  if (c->pkey == pipe_key(c) && c->pgend) {
    if (!c->pcols || c->pgendc) return 0;
    // the column branches (first march with columns on these graphs; an exec left by a
    // capture that failed part-way has never been replayed)
    for (int s = 0; s < c->nst; ++s) {
      if (c->pgx[s][PP_COL]) {
        HIPCHK(hipGraphExecDestroy(c->pgx[s][PP_COL]));
        c->pgx[s][PP_COL] = nullptr;
      }
      if ((rc = capture_part(c, s, PP_COL, &c->pgx[s][PP_COL]))) return rc;
    }
    return capture_part(c, 0, -2, &c->pgendc);
  }
  HIPCHK(hipDeviceSynchronize());   // no replay of the old graphs may still run
  for (int s = 0; s < 16; ++s)
    for (int q = 0; q < 4; ++q)
      if (c->pgx[s][q]) {
        HIPCHK(hipGraphExecDestroy(c->pgx[s][q]));
        c->pgx[s][q] = nullptr;
      }
  for (hipGraphExec_t* g : {&c->pgend, &c->pgendc})
    if (*g) {
      HIPCHK(hipGraphExecDestroy(*g));
      *g = nullptr;
    }
  c->pkey = -1;
  for (int s = 0; s < c->nst; ++s)
    for (int q = 0; q < 4; ++q) {
      if (q == PP_COL && !c->pcols) continue;
      if (q == PP_LU && s != grp_last(c, s)) continue;   // one LU graph per group
      if ((rc = capture_part(c, s, q, &c->pgx[s][q]))) return rc;
    }
  if ((rc = capture_part(c, 0, -1, &c->pgend))) return rc;
  if (c->pcols && (rc = capture_part(c, 0, -2, &c->pgendc))) return rc;
  c->pkey = pipe_key(c);
  return 0;
}

// One step of the lagged-factor march from the per-branch graphs: each branch on its
// own stream (so on its own queue), the dependencies as events.  The step ends in two
// halves: the base column's on the main stream, right after the last base chain, and
// the Jacobian columns' on the column stream, so that the next step's base chain does
// not wait for the last LU and column chain of this one.  What crosses the step
// boundary is explicit: stage s rewrites its factor set only after the step before has
// finished with it (its column chain of stage s; without columns, its LU of stage s),
// and the base solve of stage s < lag reads the factors of the LU of stage
// s - lag + nst of the step before.  The main stream joins the other streams
// (pipe_join) before the march's outputs are read.
static int pipe_launch(ww_ctx* c, int s, int part, hipStream_t st, bool graphed) {
  if (graphed && (part < 0 || ((c->graph_parts >> part) & 1))) {
    HIPCHK(hipGraphLaunch(part < 0 ? (part == -1 ? c->pgend : c->pgendc) : c->pgx[s][part], st));
    return 0;
  }
  hipStream_t user = c->stream;
  c->stream = st;
  c->prof_stage = part < 0 ? -1 : s;
  const int rc = part < 0 ? enqueue_pipe_end(c, part == -2) : enqueue_pipe_part(c, s, part);
  c->prof_stage = -1;
  c->stream = user;
  return rc;
}

static int pipe_step(ww_ctx* c, bool graphed) {
  const int nst = c->nst, L = c->lag;
  hipStream_t s0 = c->stream;
  int rc;
  for (int s = 0; s < nst; ++s) {
    hipStream_t ls = lu_stream(c, s);
    const bool last = s == grp_last(c, s);
    // Each wait is a barrier packet that the command processor takes microseconds to
    // clear even when its event has long completed, and these sit on the critical path:
    // a group's sets are released together (its column chains run in stage order, and
    // its LU records the events of all its stages at once), so the first stage of a
    // group waits for the whole group and the others wait for nothing.
    const int q = (s - L + nst) % nst;   // the stage whose factors the lagged solve reads
    if (s == grp_first(c, s)) HIPCHK(hipStreamWaitEvent(s0, c->pcols ? c->evC[grp_last(c, s)] : c->evL[grp_last(c, s)], 0));
    // the prep part already applies the lagged inverse (the first solve)
    if (s == 0 || q == grp_first(c, q)) HIPCHK(hipStreamWaitEvent(s0, c->evL[grp_last(c, q)], 0));
    if ((rc = pipe_launch(c, s, PP_PREP, s0, graphed))) return rc;
    if (last) {
      // the LU group of stages grp_first .. s, once the last of them is assembled
      HIPCHK(hipEventRecord(c->evA[s], s0));
      HIPCHK(hipStreamWaitEvent(ls, c->evA[s], 0));
      if ((rc = pipe_launch(c, s, PP_LU, ls, graphed))) return rc;
      for (int q = grp_first(c, s); q <= s; ++q) HIPCHK(hipEventRecord(c->evL[q], ls));
    }
    if ((rc = pipe_launch(c, s, PP_BASE, s0, graphed))) return rc;
    if (!c->pcols) continue;
    HIPCHK(hipEventRecord(c->evB[s], s0));
    if (!last) continue;
    // the column chains of the group, after its LU, each after the base chain of its
    // stage and the column chain before it (stage order; the first of a step waits
    // for the last step's Jacobian step end)
    for (int q = grp_first(c, s); q <= s; ++q) {
      hipStream_t cs = c->cols_on_lu ? ls : c->side;
      if (!c->cols_on_lu) HIPCHK(hipStreamWaitEvent(cs, c->evL[q], 0));
      HIPCHK(hipStreamWaitEvent(cs, c->evB[q], 0));
      HIPCHK(hipStreamWaitEvent(cs, q == 0 ? c->evE : c->evC[q - 1], 0));
      if ((rc = pipe_launch(c, q, PP_COL, cs, graphed))) return rc;
      HIPCHK(hipEventRecord(c->evC[q], cs));
    }
  }
  if ((rc = pipe_launch(c, 0, -1, s0, graphed))) return rc;
  if (c->pcols) {
    hipStream_t cs = c->cols_on_lu ? lu_stream(c, nst - 1) : c->side;   // after the last column chain
    if ((rc = pipe_launch(c, 0, -2, cs, graphed))) return rc;
    HIPCHK(hipEventRecord(c->evE, cs));
  }
  c->pjoin = true;
  return 0;
}

// the main stream waits for the column stream's last step end (and through it for
// every LU and column chain of the march); without columns, for the LUs of the last
// step (each LU stream's last LU ends after its earlier ones)
static int pipe_join(ww_ctx* c) {
  if (!c->pjoin) return 0;
  if (c->pcols) {
    HIPCHK(hipStreamWaitEvent(c->stream, c->evE, 0));
  } else {
    for (int s = 0; s < c->nst; ++s) HIPCHK(hipStreamWaitEvent(c->stream, c->evL[s], 0));
  }
  c->pjoin = false;
  return 0;
}

// two_streams: the column chain of stage s runs on the side stream while stage s + 1
// refactors (single instances); otherwise it follows the base chain on one stream
// (batches, where the instances overlap each other instead).
static int enqueue_step(ww_ctx* c, bool cols, bool two_streams) {
  if (pipelined(c, cols, two_streams)) return pipe_step(c, false);
  int rc;
  const bool two = cols && c->M > 0 && two_streams;
  hipStream_t s0 = c->stream;
  for (int s = 0; s < c->nst; ++s) {
    const int par = s & 1;
    c->prof_stage = s;
    // the factor set of this parity was last read by the column chain of stage s - 2
    if (two && s >= 2) HIPCHK(hipStreamWaitEvent(s0, c->evC[s - 2], 0));
    rc = enqueue_base_chain(c, c->y, s, c->K + (size_t)s * kstride(c), fac_set(c, par, false));
    if (!rc && two) {
      // column chain of stage s on the side stream, overlapping the next base chain
      HIPCHK(hipEventRecord(c->evB[s], s0));
      HIPCHK(hipStreamWaitEvent(c->side, c->evB[s], 0));
      c->stream = c->side;
      rc = enqueue_col_chain(c, s, fac_set(c, par, true));
      c->stream = s0;
      if (!rc) HIPCHK(hipEventRecord(c->evC[s], c->side));
    } else if (!rc && cols && c->M > 0) {
      rc = enqueue_col_chain(c, s, fac_set(c, par, true));   // one stream: after the base chain
    }
    c->prof_stage = -1;
    if (rc) return rc;
  }
  if (two) HIPCHK(hipStreamWaitEvent(s0, c->evC[c->nst - 1], 0));
  const int ncol = cols ? c->M + 1 : 1;
  hipLaunchKernelGGL(k_step_end, dim3(ncol), dim3(WW_NT), fft_lds_bytes(c->N, 3), c->stream, c->y, c->K, kstride(c),
                     c->nst, c->coef, c->tw, c->sig, c->N, 0, c->status);
  LAUNCHCHK();
  return 0;
}

// Capture one step (all stages + end of step) into a graph on the private capture
// stream; the graph is reused while (N, M, columns, stages) are unchanged.  Step
// coefficients live in device memory, so T and the parameters may change freely.
static int ensure_step_graph(ww_ctx* c, bool cols, bool two_streams) {
  if (c->step_exec && c->gN == c->N && c->gM == c->M && c->gcols == (int)cols && c->gnst == c->nst &&
      c->gtwo == (int)two_streams && c->gfb == c->fb && c->ggm == (c->gm_active ? c->gm_m : 0) &&
      c->gtune == c->tune_gen && c->gmap == (int)c->mapped)
    return 0;
  if (c->step_exec) {
    HIPCHK(hipDeviceSynchronize());   // every branch of its last replay has ended
    HIPCHK(hipGraphExecDestroy(c->step_exec));
    c->step_exec = nullptr;
  }
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_step(c, cols, two_streams);
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
  c->gtwo = (int)two_streams;
  c->gnst = c->nst;
  c->gfb = c->fb;
  c->ggm = c->gm_active ? c->gm_m : 0;
  c->gtune = c->tune_gen;
  c->gmap = (int)c->mapped;
  return 0;
}

// status bits (clears them); *where (optional) receives 16 step + stage of the first
// non-finite or bed-crossing stage state of a march (INT_MAX if none)
static int read_status(ww_ctx* c, int* st, int* where) {
  int h[3] = {0, 0, 0};
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(h, c->status, sizeof(h), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(c->status, 0, sizeof(int)));
  *st = h[0];
  if (where) *where = h[2];
  return 0;
}

static const char* const MSG_PIVOT = "pivot below the guard (unpivoted LU, WW_STRICT)";
static const char* const MSG_PIVOT2 = "pivot below the guard also with partial pivoting (A numerically singular)";
static const char* const MSG_REFINE = "mixed precision: relative residual of the refined solution above 2^-43";

// Assemble and factor the DtN matrices of the surface prepared in aux, with the
// pivoting fallback when a pivot falls below the guard.
static int dtn_factor(ww_ctx* c) {
  for (;;) {
    int rc;
    if (pivoted(c) && (rc = ensure_pivot_buffers(c))) return rc;
    if ((rc = enqueue_assemble_lu(c, fac_default(c)))) return rc;
    int st = 0;
    if ((rc = read_status(c, &st))) return rc;
    if (st & 2) return fail(WW_ENONFINITE, "non-finite surface");
    if (!(st & (1 | 8))) return 0;
    if (pivoted(c)) return fail(WW_EPIVOT, MSG_PIVOT2);
    if (strict(c)) return fail(WW_EPIVOT, MSG_PIVOT);
    c->fb |= WW_FB_PIVOTED | WW_FB_FP64;
  }
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
  c->dtn_ready = false;   // until this surface is factored
  c->fb = 0;
  c->gm_active = false;
  int rc;
  if ((rc = set_grid(c, N, h))) return rc;
  c->tau = tau;
  if ((rc = check_domain(c, surface))) return rc;
  HIPCHK(hipMemcpyAsync(c->ydtn, surface, N * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemsetAsync(c->ydtn + N, 0, N * 8, c->stream));
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 4), c->stream, c->ydtn, c->K, c->Ys,
                     c->coef, 0, (size_t)0, c->aux, c->n_max, c->rhs0, c->Np, c->tw, N, c->hsurf, c->status);
  LAUNCHCHK();
  if ((rc = dtn_factor(c))) return rc;
  c->dtn_ready = true;
  c->fb_last = c->fb;
  return 0;
}

}  // extern "C"

// work arrays of one dtn_solve_multi call (each Np x nrhs, ld Np; Rr only in the mixed
// form) and the split-K partials of its products
struct SolveWork {
  double *Psi, *Ytmp, *Mu, *Gam, *HG, *Gpsi, *Rr;
};

static int dtn_solve_impl(ww_ctx* c, const double* rhs, int nrhs, double* dtn_out, double* mu_out,
                          const SolveWork& w) {
  const int N = c->N, Np = c->Np;
  const size_t tot = (size_t)Np * nrhs;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, rhs, N, w.Psi, Np, N, Np, nrhs);
  LAUNCHCHK();
  int rc;
  for (;;) {
    const Fac F = fac_default(c);
    if ((rc = enqueue_dtn_cols(c, F, w.Psi, w.Ytmp, w.Mu, w.Gam, w.HG, w.Gpsi, w.Rr, nrhs))) return rc;
    if (!use32(c)) break;
    int st = 0;   // the refinement test of the mixed path
    if ((rc = read_status(c, &st))) return rc;
    if (!(st & 4)) break;
    if (strict(c)) return fail(WW_EREFINE, MSG_REFINE);
    c->fb |= WW_FB_FP64;   // refactor in FP64 (kept for the later calls) and solve again
    c->dtn_ready = false;
    if ((rc = dtn_factor(c))) return rc;
    c->dtn_ready = true;
  }
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, w.Gpsi, Np, dtn_out, N, Np, N, nrhs);
  LAUNCHCHK();
  if (mu_out) {
    hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, w.Mu, Np, mu_out, N, Np, N, nrhs);
    LAUNCHCHK();
  }
  c->fb_last = c->fb;
  return 0;
}

static int dtn_solve_check(ww_ctx* c, const double* rhs, int nrhs, double* dtn_out) {
  if (!c || !rhs || !dtn_out) return fail(WW_EINVAL, "null argument");
  if (!c->dtn_ready) return fail(WW_ENOSETUP, "dtn_solve_multi before dtn_setup");
  if (nrhs < 1 || nrhs > c->r_max) return fail(WW_EINVAL, "nrhs out of range");
  return 0;
}

extern "C" {

int dtn_solve_multi(ww_ctx* c, const double* rhs, int nrhs, double* dtn_out, double* mu_out) {
  int rc;
  if ((rc = dtn_solve_check(c, rhs, nrhs, dtn_out))) return rc;
  const SolveWork w{c->Psi, c->Ytmp, c->Mu, c->Gam, c->HG, c->Gpsi, c->Rr};
  return dtn_solve_impl(c, rhs, nrhs, dtn_out, mu_out, w);
}

int dtn_solve_multi_noalloc(ww_ctx* c, const double* rhs, int nrhs, double* dtn_out, double* mu_out) {
  int rc;
  if ((rc = dtn_solve_check(c, rhs, nrhs, dtn_out))) return rc;
  if (!c->scratch) return fail(WW_EHIP, "internal: fixed workspace address not resolved");
  // layout: Psi, Ytmp, Mu, Gam, HG, Gpsi, Rr, Np x nrhs each
  const size_t blk = (size_t)c->Np * nrhs;
  const size_t nbuf = 7;
  if (nbuf * blk > WW_SCRATCH_DOUBLES)
    return fail(WW_EINVAL, "dtn_solve_multi_noalloc: 7 Np nrhs doubles exceed the fixed workspace (" +
                               std::to_string(WW_SCRATCH_BYTES >> 20) + " MiB); use dtn_solve_multi");
  double* s = c->scratch;
  const SolveWork w{s, s + blk, s + 2 * blk, s + 3 * blk, s + 4 * blk, s + 5 * blk, s + 6 * blk};
  return dtn_solve_impl(c, rhs, nrhs, dtn_out, mu_out, w);
}

}  // extern "C"

// ----- double-double DtN -----
// sin and cos of 2 pi d / n in double-double (host, for the tables): the angle is
// reduced exactly to [0, pi/4] with integer arithmetic (quadrant, then the complement),
// and both Taylor series are summed until a term falls below 1e-34.
static void dd_sincos_2pi(long d, long n, dd* s_out, dd* c_out) {
  d %= n;
  if (d < 0) d += n;
  const long q = (4 * d) / n;               // quadrant
  const long r4 = 4 * d - q * n;            // 4 d - q n in [0, n): angle 2 pi r4 / (4 n)
  const bool comp = 2 * r4 > n;             // beyond pi/4: use the complement
  const long num = comp ? n - r4 : r4;      // angle 2 pi num / (4 n) = pi num / (2 n)
  const dd pi = dd{DD_PI_HI, DD_PI_LO};
  const dd x = dd_div_d(dd_mul_d(pi, (double)num), 2.0 * (double)n);
  const dd x2 = dd_mul(x, x);
  dd sn = x, term = x;
  for (int k = 1; k < 40; ++k) {
    term = dd_div_d(dd_mul(term, x2), -(double)((2 * k) * (2 * k + 1)));
    sn = dd_add(sn, term);
    if (std::fabs(term.hi) < 1e-34) break;
  }
  dd cs = dd_of(1.0);
  term = dd_of(1.0);
  for (int k = 1; k < 40; ++k) {
    term = dd_div_d(dd_mul(term, x2), -(double)((2 * k - 1) * (2 * k)));
    cs = dd_add(cs, term);
    if (std::fabs(term.hi) < 1e-34) break;
  }
  if (comp) std::swap(sn, cs);
  dd so, co;
  switch (q) {
    case 0: so = sn; co = cs; break;
    case 1: so = cs; co = dd_neg(sn); break;
    case 2: so = dd_neg(sn); co = dd_neg(cs); break;
    default: so = dd_neg(cs); co = sn; break;
  }
  *s_out = so;
  *c_out = co;
}

#define DD_WORK 13
#define DD_SWEEPS 3
#define DD_SWEEPS_32 6   // with FP32 factors: each sweep gains about 2^-24 cond(A)
static const double DD_TOL = 1.2621774483536189e-29;   // 2^-96
static int ensure_dd(ww_ctx* c) {
  if (c->dd_w) return 0;
  int rc;
  const size_t nm = c->n_max, np = c->np_max;
  double** planes[] = {&c->dd_tab_hi, &c->dd_tab_lo};
  for (double** q : planes)
    if ((rc = dalloc(c, (void**)q, 3 * nm * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->dd_tw, nm / 2 * sizeof(cdd)))) return rc;
  if ((rc = dalloc(c, (void**)&c->dd_pt_hi, 4 * nm * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->dd_pt_lo, 4 * nm * 8))) return rc;
  double** mats[] = {&c->dd_Ah, &c->dd_Al, &c->dd_Gh, &c->dd_Gl};
  for (double** q : mats)
    if ((rc = dalloc(c, (void**)q, np * np * 8))) return rc;
  if (!c->dd_part && (rc = dalloc(c, (void**)&c->dd_part, (size_t)2 * DDGV_KS * np * 8))) return rc;
  return dalloc(c, (void**)&c->dd_w, (size_t)DD_WORK * np * c->r_max * 8);
}

// out = add + sgn A B in double-double for nrhs columns (ld Np): one column by the
// inner-index split of k_dd_gemv_part / k_dd_gemv_sum, several by k_dd_gemm
static int dd_gemm(ww_ctx* c, double* part, const double* Ah, const double* Al, const double* Bh, const double* Bl,
                   const double* addh, const double* addl, double sgn, double* outh, double* outl, int nrhs) {
  const int Np = c->Np;
  if (nrhs == 1) {
    double *Ph = part, *Pl = part + (size_t)DDGV_KS * c->np_max;
    hipLaunchKernelGGL(k_dd_gemv_part, dim3(Np / 64, DDGV_KS), dim3(WW_NT), 0, c->stream, Ah, Al, Np, Bh, Bl, Ph, Pl);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_dd_gemv_sum, dim3((Np + 255) / 256), dim3(256), 0, c->stream, Ph, Pl, DDGV_KS, Np, addh,
                       addl, sgn, outh, outl);
    LAUNCHCHK();
    return 0;
  }
  hipLaunchKernelGGL(k_dd_gemm, dim3(Np / 64, (nrhs + 3) / 4), dim3(WW_NT), 0, c->stream, Ah, Al, Np, Bh, Bl, addh,
                     addl, sgn, outh, outl, nrhs);
  LAUNCHCHK();
  return 0;
}

static int dd_tables(ww_ctx* c, int N) {
  if (c->dd_N == N) return 0;
  HIPCHK(hipStreamSynchronize(c->stream));   // queued work may still read the old tables
  std::vector<double> th(3 * N), tl(3 * N);
  std::vector<cdd> tw(N / 2);
  for (int d = 0; d < N; ++d) {
    dd sn, cs;
    dd_sincos_2pi(d, N, &sn, &cs);
    th[d] = cs.hi;
    tl[d] = cs.lo;
    th[N + d] = sn.hi;
    tl[N + d] = sn.lo;
    if (d < N / 2) tw[d] = cdd{cs, dd_neg(sn)};
    dd c0 = dd_of(0.0);
    if (d > 0) {   // cot(pi d / N) / 2 = cos / (2 sin) of 2 pi d / (2 N)
      dd sh, ch;
      dd_sincos_2pi(d, 2L * N, &sh, &ch);
      c0 = dd_div(ch, dd_mul_d(sh, 2.0));
    }
    th[2 * N + d] = c0.hi;
    tl[2 * N + d] = c0.lo;
  }
  HIPCHK(hipMemcpy(c->dd_tab_hi, th.data(), 3 * N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->dd_tab_lo, tl.data(), 3 * N * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->dd_tw, tw.data(), (N / 2) * sizeof(cdd), hipMemcpyHostToDevice));
  c->dd_N = N;
  return 0;
}

static size_t dd_lds_bytes(int N) { return (size_t)(3 * N + N / 2) * sizeof(cdd); }

// The buffers of one double-double DtN: per-point quantities, A and Gm (hi and lo
// planes), and the FP64 factor set whose A receives A's leading part and whose Mi the
// explicit inverse.  The context's own (dd_lane) serves dtn_setup_dd / dtn_solve_multi_dd
// and the double-double march's predictor; the nodes of its correction sweeps take one
// lane each (with the ring's factor sets).
struct DdLane {
  double *pt_hi, *pt_lo, *Ah, *Al, *Gh, *Gl;
  Fac F;
  double *w, *part;   // the solve's workspace: DD_WORK planes, the one-column product's partials
};
// the factors of the corrections: FP64, or FP32 on MFMA in a WW_MIXED context
static Fac dd_fac(const ww_ctx* c, Fac F) {
  F.use32 = mixed(c);
  F.lag32 = false;
  F.perm = nullptr;
  F.Gm = nullptr;
  return F;
}
static DdLane dd_lane(ww_ctx* c) {
  return DdLane{c->dd_pt_hi, c->dd_pt_lo, c->dd_Ah, c->dd_Al, c->dd_Gh,
                c->dd_Gl,    dd_fac(c, fac_default(c)), c->dd_w, c->dd_part};
}

// per-point quantities and the double-double assembly of the surface (sh, sl) into lane
// L; domain (optional): status word for the finite-depth test h + eta > 0
static int dd_prep_assemble(ww_ctx* c, const DdLane& L, const double* sh, const double* sl, int* domain) {
  const int N = c->N, Np = c->Np;
  hipLaunchKernelGGL(k_dd_prep, dim3(1), dim3(WW_NT), dd_lds_bytes(N), c->stream, sh, sl, c->hsurf, c->dd_tw, N,
                     c->n_max, L.pt_hi, L.pt_lo, c->finite ? domain : nullptr);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dd_assemble, dim3(Np / WW_TB, Np / 16), dim3(WW_NT), 0, c->stream, L.pt_hi, L.pt_lo, c->n_max,
                     c->dd_tab_hi, c->dd_tab_lo, N, Np, c->finite, L.Ah, L.Al, L.Gh, L.Gl, L.F.A);
  LAUNCHCHK();
  if (L.F.use32) {
    if (!L.F.A32) return fail(WW_EHIP, "internal: FP32 factors without their buffer");
    const size_t nn = (size_t)Np * Np;
    hipLaunchKernelGGL(k_dd_a32, dim3((int)std::min<size_t>((nn + 255) / 256, 4096)), dim3(256), 0, c->stream, L.F.A,
                       L.F.A32, nn);
    LAUNCHCHK();
  }
  return 0;
}

// The double-double set-up of the grid's surface in the context's lane: per-point
// quantities, the double-double assembly, the FP64 factors (block LU and explicit
// inverse) of A's leading part
static int dd_setup_enqueue(ww_ctx* c, const double* sh, const double* sl, int* domain) {
  const DdLane L = dd_lane(c);
  int rc;
  if ((rc = dd_prep_assemble(c, L, sh, sl, domain))) return rc;
  return enqueue_lu(c, L.F);
}

// The double-double solve and DtN of nrhs columns with the set-up's factors: mu = Mi psi,
// DD_SWEEPS sweeps r = psi - A mu (double-double), mu += Mi r_hi, the final residual's
// and the right-hand side's largest entries into mx[0], mx[1] (zero on entry), then
// gamma = mu', H gamma / 2 and G psi = H gamma / 2 + Gm gamma
static int dd_solve_enqueue(ww_ctx* c, const DdLane& L, const double* rhs_hi, const double* rhs_lo, int nrhs,
                            double* out_hi, double* out_lo, double* mu_hi, double* mu_lo, unsigned long long* mx) {
  const int N = c->N, Np = c->Np;
  const size_t blk = (size_t)Np * nrhs, pl = (size_t)c->np_max * c->r_max;
  double* w = L.w;
  double *psh = w, *psl = w + pl, *muh = w + 2 * pl, *mul = w + 3 * pl, *rh = w + 4 * pl, *rl = w + 5 * pl;
  double *del = w + 6 * pl, *gh = w + 7 * pl, *gl = w + 8 * pl, *hh = w + 9 * pl, *hl = w + 10 * pl;
  double *oh = w + 11 * pl, *ol = w + 12 * pl;
  const int blocks = (int)std::min<size_t>((blk + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, rhs_hi, N, psh, Np, N, Np, nrhs);
  LAUNCHCHK();
  if (rhs_lo)
    hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, rhs_lo, N, psl, Np, N, Np, nrhs);
  else
    hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, psh, Np, psl, Np, 0, Np, nrhs);
  LAUNCHCHK();
  int rc;
  // corrections from the FP64 inverse, or from the FP32 one (a mixed context: more sweeps)
  auto corr = [&](const double* B, double* X) -> int {
    return L.F.use32 ? enqueue_gemm<float>(c, L.F.Mi32, 0, B, nullptr, 1.0, X, nrhs)
                     : enqueue_gemm<double>(c, L.F.Mi, 0, B, nullptr, 1.0, X, nrhs);
  };
  const int sweeps = L.F.use32 ? DD_SWEEPS_32 : DD_SWEEPS;
  if ((rc = corr(psh, muh))) return rc;
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, c->stream, psh, Np, mul, Np, 0, Np, nrhs);
  LAUNCHCHK();
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    if ((rc = dd_gemm(c, L.part, L.Ah, L.Al, muh, mul, psh, psl, -1.0, rh, rl, nrhs))) return rc;
    if ((rc = corr(rh, del))) return rc;
    hipLaunchKernelGGL(k_dd_correct, dim3(blocks), dim3(256), 0, c->stream, muh, mul, del, blk);
    LAUNCHCHK();
  }
  if ((rc = dd_gemm(c, L.part, L.Ah, L.Al, muh, mul, psh, psl, -1.0, rh, rl, nrhs))) return rc;
  hipLaunchKernelGGL(k_dd_maxabs, dim3(std::min(blocks, 256)), dim3(256), 0, c->stream, rh, psh, N, Np, nrhs, mx);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dd_gamma, dim3(nrhs), dim3(WW_NT), dd_lds_bytes(N), c->stream, muh, mul, Np, c->dd_tw, N, gh,
                     gl, hh, hl);
  LAUNCHCHK();
  if ((rc = dd_gemm(c, L.part, L.Gh, L.Gl, gh, gl, hh, hl, 1.0, oh, ol, nrhs))) return rc;
  const size_t tot = (size_t)N * nrhs;
  const int ob = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_copy, dim3(ob), dim3(256), 0, c->stream, oh, Np, out_hi, N, Np, N, nrhs);
  hipLaunchKernelGGL(k_pad_copy, dim3(ob), dim3(256), 0, c->stream, ol, Np, out_lo, N, Np, N, nrhs);
  if (mu_hi) {
    hipLaunchKernelGGL(k_pad_copy, dim3(ob), dim3(256), 0, c->stream, muh, Np, mu_hi, N, Np, N, nrhs);
    hipLaunchKernelGGL(k_pad_copy, dim3(ob), dim3(256), 0, c->stream, mul, Np, mu_lo, N, Np, N, nrhs);
  }
  LAUNCHCHK();
  return 0;
}

extern "C" {

int dtn_setup_dd(ww_ctx* c, const double* surface_hi, const double* surface_lo, double h, int N) {
  if (!c || !surface_hi) return fail(WW_EINVAL, "null argument");
  c->dd_ready = false;
  c->dtn_ready = false;   // the FP64 factor buffers are reused
  if (N < 16 || (N & (N - 1)) || N > c->n_max || N > 1024)
    return fail(WW_EINVAL, "double-double DtN: N must be a power of two, 16 <= N <= min(n_max, 1024)");
  int rc;
  if ((rc = set_grid(c, N, h))) return rc;
  if ((rc = check_domain(c, surface_hi))) return rc;
  if ((rc = ensure_dd(c))) return rc;
  if ((rc = dd_tables(c, N))) return rc;
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  if ((rc = dd_setup_enqueue(c, surface_hi, surface_lo, nullptr))) return rc;
  int st = 0;
  if ((rc = read_status(c, &st))) return rc;
  if (st & 2) return fail(WW_ENONFINITE, "non-finite surface");
  if (st & (1 | 8)) return fail(WW_EPIVOT, "double-double DtN: pivot below the guard (no pivoted form)");
  c->dd_ready = true;
  return 0;
}

int dtn_solve_multi_dd(ww_ctx* c, const double* rhs_hi, const double* rhs_lo, int nrhs, double* out_hi,
                       double* out_lo, double* mu_hi, double* mu_lo) {
  if (!c || !rhs_hi || !out_hi || !out_lo || (!mu_hi != !mu_lo)) return fail(WW_EINVAL, "null argument");
  if (!c->dd_ready) return fail(WW_ENOSETUP, "dtn_solve_multi_dd before dtn_setup_dd");
  if (nrhs < 1 || nrhs > c->r_max) return fail(WW_EINVAL, "1 <= nrhs <= r_max required");
  unsigned long long* mx = (unsigned long long*)(c->status + 4);
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  int rc;
  if ((rc = dd_solve_enqueue(c, dd_lane(c), rhs_hi, rhs_lo, nrhs, out_hi, out_lo, mu_hi, mu_lo, mx))) return rc;
  unsigned long long m[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(m, mx, sizeof(m), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double mr, mb;
  std::memcpy(&mr, &m[0], 8);
  std::memcpy(&mb, &m[1], 8);
  if (!(mr <= DD_TOL * mb)) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "double-double DtN: residual %.3e of the right-hand side after the sweeps (above 2^-96)",
                  mb > 0.0 ? mr / mb : mr);
    return fail(WW_EREFINE, msg);
  }
  return 0;
}

int ww_profile(ww_ctx* c, int enable) {
  if (!c) return fail(WW_EINVAL, "null argument");
  c->prof_kev = (enable & 2) != 0;
  c->kev_n = 0;
  if (enable && !c->stamps) HIPCHK(hipMalloc(&c->stamps, 3 * 16 * 3 * sizeof(unsigned long long)));
  if (enable) HIPCHK(hipMemsetAsync(c->stamps, 0, 3 * 16 * 3 * sizeof(unsigned long long), c->stream));
  if (enable) {
    c->host_enq_ms = 0.0;
    c->host_enq_steps = 0;
  }
  if ((bool)enable != c->prof) {
    c->prof = enable != 0;
    c->gnst = -1;   // re-capture the step graph with or without the stamp nodes
  }
  return 0;
}

int ww_profile_read(ww_ctx* c, int phase, double* avg_ms, int* count) {
  if (!c || !avg_ms || phase < 0 || phase > 4) return fail(WW_EINVAL, "bad argument");
  if (!c->prof || !c->stamps) return fail(WW_EINVAL, "profiling is off");
  if (phase == 4) {
    if (c->kev_n == 0) return fail(WW_EINVAL, "no block-LU step launched outside graphs since ww_profile");
    double sum = 0.0;
    for (size_t i = 0; i < c->kev_n; ++i) {
      HIPCHK(hipEventSynchronize(c->kev_b[i]));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, c->kev_a[i], c->kev_b[i]));
      sum += ms;
    }
    *avg_ms = sum / (double)c->kev_n;
    if (count) *count = (int)c->kev_n;
    return 0;
  }
  if (phase == 3) {
    if (c->host_enq_steps == 0) return fail(WW_EINVAL, "no profiled step");
    *avg_ms = c->host_enq_ms / (double)c->host_enq_steps;
    if (count) *count = (int)c->host_enq_steps;
    return 0;
  }
  unsigned long long h[16 * 3];
  HIPCHK(hipMemcpyAsync(h, c->stamps + (size_t)phase * 16 * 3, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(WW_EHIP, "wall clock rate unavailable");
  unsigned long long ticks = 0, n = 0;
  for (int s = 0; s < 16; ++s) {
    ticks += h[3 * s + 1];
    n += h[3 * s + 2];
  }
  if (n == 0) return fail(WW_EINVAL, "no profiled stage (run shoot_eval with profiling on first)");
  *avg_ms = (double)ticks / (double)n / (double)khz;
  if (count) *count = (int)n;
  return 0;
}

int shoot_setup(ww_ctx* c, int N, double h, double tau, double g, const double* basis, const double* q_fixed,
                int M) {
  if (!c || (!basis && M > 0)) return fail(WW_EINVAL, "null argument");
  if (M < 0 || M + 1 > c->r_max) return fail(WW_EINVAL, "M + 1 must be <= r_max");
  int rc;
  if ((rc = set_grid(c, N, h))) return rc;
  c->dtn_ready = false;   // the grid of a previous dtn_setup is gone
  // the step graphs hold depth, tension and gravity as kernel arguments: capture again
  c->gnst = -1;
  c->pkey = -1;
  c->lag_off = false;
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

}  // extern "C"

// the pivoting fallback launches two kernels per column of A and runs without a graph
static bool graphed(const ww_ctx* c) { return c->use_graph && !pivoted(c); }

// step coefficients a_sj dt, b_s dt and dt of nsteps steps over T/4
static void coef_fill(const ww_ctx* c, double T, int nsteps, double* coef) {
  std::memset(coef, 0, COEF_SIZE * sizeof(double));
  const double dt = T / (4.0 * nsteps);
  for (int s = 0; s < c->nst; ++s) {
    for (int j = 0; j < s; ++j) coef[s * 16 + j] = c->ta[s * 16 + j] * dt;
    coef[COEF_B + s] = c->tb[s] * dt;
  }
  coef[COEF_DT] = dt;
}

// shoot_eval in three parts so that shoot_eval_batch can interleave instances:
// prepare (coefficients, initial state, step graph), one step, finish (outputs).
static int shoot_prepare(ww_ctx* c, const double* params, double T, int nsteps, bool cols, bool two_streams) {
  if (int rj = pipe_join(c)) return rj;   // a march that ended early (an error) left its streams unjoined
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "shoot_eval before shoot_setup");
  if (c->nst < 1) return fail(WW_EINVAL, "no tableau set");
  if (nsteps < 1 || !std::isfinite(T)) return fail(WW_EINVAL, "nsteps >= 1 and finite T required");
  int rc;
  if ((rc = set_grid(c, c->shootN, c->shootH))) return rc;
  c->dtn_ready = false;   // the factor arrays are reused by the march
  const int N = c->N, M = c->M;
  double coef[COEF_SIZE];
  coef_fill(c, T, nsteps, coef);
  HIPCHK(hipMemcpyAsync(c->coef, coef, sizeof(coef), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  const size_t tot = (size_t)2 * N * (M + 1);
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, c->stream, c->y, c->basis, c->qfix, params, N, M);
  LAUNCHCHK();
  c->gm_active = (c->flags & WW_GMRES) && !cols && c->fb == 0 && !c->mapped;
  if (c->gm_active) {
    if ((rc = ensure_gmres(c))) return rc;
    if (!c->gm_fixed && (rc = gmres_calibrate(c))) return rc;
  }
  {
    // the column stream: two-stream step graphs, and lagged marches whose column chains
    // do not run on the LU streams
    const bool pipe = pipelined(c, cols, two_streams);
    if (cols && c->M > 0 && two_streams && !(pipe && graphed(c) && c->cols_on_lu) && !c->side)
      HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  }
  if (pipelined(c, cols, two_streams)) {
    c->pcols = cols && c->M > 0;
    if ((rc = ensure_pipe(c))) return rc;
    if ((rc = pipe_prologue(c))) return rc;
    if (graphed(c)) return ensure_pipe_graphs(c);
    return 0;
  }
  if (graphed(c)) return ensure_step_graph(c, cols, two_streams);
  return 0;
}

static int shoot_one_step(ww_ctx* c, bool cols, bool two_streams) {
  if (graphed(c) && pipelined(c, cols, two_streams)) return pipe_step(c, true);
  if (graphed(c)) {
    HIPCHK(hipGraphLaunch(c->step_exec, c->stream));
    return 0;
  }
  return enqueue_step(c, cols, two_streams);
}

static int shoot_finish(ww_ctx* c, bool cols, double* r, double* J, double* drdT, double* fhost) {
  const int N = c->N, M = c->M;
  int rc;
  if ((rc = pipe_join(c))) return rc;
  {
    const size_t n = (size_t)2 * N * (cols ? M + 1 : 1);
    hipLaunchKernelGGL(k_check_finite, dim3(64), dim3(256), 0, c->stream, c->y, n, c->status);
    LAUNCHCHK();
  }
  if (drdT)
    if ((rc = enqueue_base_chain(c, c->y, 0, c->Kx, fac_default(c)))) return rc;
  {
    const size_t tot = (size_t)N * (M + 1);
    const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
    if (c->mapped)
      hipLaunchKernelGGL(k_outputs_map, dim3(blocks), dim3(256), 0, c->stream, c->y, c->Kx, c->mesh, c->n_max, r,
                         cols ? J : nullptr, drdT, N, cols ? M : 0);
    else
      hipLaunchKernelGGL(k_outputs, dim3(blocks), dim3(256), 0, c->stream, c->y, c->Kx, r, cols ? J : nullptr, drdT,
                         N, cols ? M : 0);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(WW_NT), 0, c->stream, r, N, c->fdev, (const double*)nullptr);
  LAUNCHCHK();
  if (fhost) HIPCHK(hipMemcpyAsync(fhost, c->fdev, 8, hipMemcpyDeviceToHost, c->stream));
  return 0;
}

// Status bits of a march: 1 pivot below the guard (unpivoted LU), 8 pivot below the
// guard (pivoted LU), 2 non-finite state, 4 failed refinement test (mixed form), 16
// surface through the bottom, 32 failed refinement test of a lagged-factor solve, 64
// failed residual test of a GMRES solve.  The fallback that a redo of the call takes,
// or 0.  A small pivot redoes the march with pivoted factors first (which also ends
// the lagged and GMRES solves: every stage then solves with its own factors).
// Unconverged lagged or GMRES solves are redone on each stage's own factors: the state
// they produced, a bed crossing included, is not the method's.  A crossing on a march
// without such solves is reported, not redone (small pivots there come from the
// crossing).
static unsigned fallback_decision(unsigned flags, unsigned fb, int st) {
  if (flags & WW_STRICT) return 0;
  const bool unconverged = (st & (32 | 64)) && !(fb & WW_FB_DIRECT);
  if ((st & (1 | 8)) && !(fb & WW_FB_PIVOTED) && (!(st & 16) || unconverged)) return WW_FB_PIVOTED | WW_FB_FP64;
  if (unconverged) return WW_FB_DIRECT;
  if (st & 16) return 0;   // a surface through the bottom is no factorisation issue
  if ((st & 4) && !(fb & WW_FB_FP64)) return WW_FB_FP64;
  return 0;
}

static unsigned next_fallback(const ww_ctx* c, int st) { return fallback_decision(c->flags, c->fb, st); }

extern "C" unsigned ww_next_fallback(unsigned flags, unsigned fb, int status) {
  return fallback_decision(flags, fb, status);
}

static int status_error(const ww_ctx* c, int st, int where) {
  std::string at;
  if (where != 0x7fffffff) at = " at step " + std::to_string(where / 16) + ", stage " + std::to_string(where % 16);
  if (st & 16) return fail(WW_EDOMAIN, "finite depth: surface height h + eta <= 0 in the march" + at);
  if (st & 2)
    return fail(WW_ENONFINITE, "non-finite value in the marched state" + (at.empty() ? std::string(" (at T/4)") : at));
  if (st & (1 | 8)) return fail(WW_EPIVOT, pivoted(c) ? MSG_PIVOT2 : MSG_PIVOT);
  if (st & 4) return fail(WW_EREFINE, MSG_REFINE);
  if (st & 32) return fail(WW_EREFINE, "lagged-factor solves: relative residual above 2^-43 (WW_STRICT)");
  if (st & 64) return fail(WW_EREFINE, "GMRES base solves: relative residual above 2^-43 (WW_STRICT)");
  return 0;
}

// one march in the current fallback mode; *st receives the status bits
static int shoot_run(ww_ctx* c, const double* params, double T, int nsteps, double* r, double* J, double* drdT,
                     double* f, int* st, int* where) {
  const bool cols = (J != nullptr) && c->M > 0;
  const bool two = c->overlap && !pivoted(c);
  int rc;
  if (pivoted(c) && (rc = ensure_pivot_buffers(c))) return rc;
  if ((rc = shoot_prepare(c, params, T, nsteps, cols, two))) return rc;
  const bool pipe = pipelined(c, cols, two);   // after the set-up, which decides on GMRES
  for (int n = 0; n < nsteps; ++n) {
    const auto h0 = std::chrono::steady_clock::now();
    if ((rc = shoot_one_step(c, cols, two))) return rc;
    if (c->prof) {
      c->host_enq_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
      ++c->host_enq_steps;
    }
    if (pipe && n == 0 && nsteps > 1) {
      // lagged factors that do not converge show in the first step: stop there (the
      // caller redoes the march in its fallback mode or reports the status)
      int peek = 0;
      if ((rc = pipe_join(c))) return rc;
      HIPCHK(hipStreamSynchronize(c->stream));
      HIPCHK(hipMemcpy(&peek, c->status, sizeof(int), hipMemcpyDeviceToHost));
      if (peek) return read_status(c, st, where);
    }
  }
  if ((rc = shoot_finish(c, cols, r, J, drdT, f))) {
    // work already enqueued may still write the caller's outputs (and f on the host)
    const std::string msg = g_err;
    (void)pipe_join(c);
    (void)hipStreamSynchronize(c->stream);
    g_err = msg;
    return rc;
  }
  return read_status(c, st, where);
}

// marches from fallback mode fb0 until the status needs no further fallback
static int shoot_eval_fb(ww_ctx* c, const double* params, double T, int nsteps, double* r, double* J, double* drdT,
                         double* f, unsigned fb0) {
  c->fb = fb0;
  for (;;) {
    int st = 0, where = 0, rc;
    if ((rc = shoot_run(c, params, T, nsteps, r, J, drdT, f, &st, &where))) return rc;
    const unsigned nf = next_fallback(c, st);
    if ((st & 32) && !strict(c)) c->lag_off = true;
    if (!nf) {
      if ((rc = status_error(c, st, where))) return rc;
      c->fb_last = c->fb;
      return 0;
    }
    c->fb |= nf;
  }
}

// ----- segmented march on non-uniform meshes (Sec. 2.2 eq. (xi), (rho:def)) -----
#define WW_MAX_SEGMENTS 64
static double mesh_coef(double rho) { return 8.0 * (1.0 - rho) / (5.0 + 3.0 * rho); }

static int seg_check(const ww_ctx* c, int nseg, const ww_segment* sg) {
  if (nseg < 1 || nseg > WW_MAX_SEGMENTS || !sg) return fail(WW_EINVAL, "1 <= nseg <= 64 segments required");
  double tsum = 0.0;
  for (int l = 0; l < nseg; ++l) {
    const ww_segment& q = sg[l];
    if (!valid_n(q.N) || q.N > c->n_max) return fail(WW_EINVAL, "segment N must be even, 2^a 3^b, 16 <= N <= n_max");
    if (q.nsteps < 1) return fail(WW_EINVAL, "segment nsteps >= 1 required");
    if (!(q.theta > 0.0) || !std::isfinite(q.theta)) return fail(WW_EINVAL, "segment theta must be positive");
    if (!(q.rho > 0.0 && q.rho <= 1.0)) return fail(WW_EINVAL, "segment rho must lie in (0, 1]");
    if (q.refine_at != WW_REFINE_PI && q.refine_at != WW_REFINE_ZERO) return fail(WW_EINVAL, "bad refine_at");
    tsum += q.theta;
    if (l > 0) {
      const ww_segment& p = sg[l - 1];
      if (q.rho < p.rho && q.N * (5.0 + 3.0 * q.rho) < p.N * (5.0 + 3.0 * p.rho) * (1.0 - 1e-15))
        return fail(WW_EINVAL, "refining the mesh needs N_l+1 / N_l >= (5 + 3 rho_l) / (5 + 3 rho_l+1)");
    }
  }
  if (std::fabs(tsum - 1.0) > 1e-12) return fail(WW_EINVAL, "the segment fractions theta must sum to 1");
  if (sg[0].N != c->shootN) return fail(WW_EINVAL, "the first segment's N must be shoot_setup's N (the basis grid)");
  return 0;
}

// SDC15 (defined with the stepper below): work arrays, the two-stream form's set-up, and
// nsteps steps of dt (two streams, or stage by stage)
static int ensure_sdc(ww_ctx* c);
static int ensure_sdc_groups(ww_ctx* c);
static int sdc_steps(ww_ctx* c, bool cols, double dt, int nsteps, bool two);

// one segmented march in the current fallback mode: segment 0 starts from the initial
// state on its mesh; at each later segment the state (and the Jacobian columns) is
// regridded to the new mesh, then the segment marches its steps of theta_l T / (4
// nsteps_l) each; the outputs are taken on the last mesh
// (sdc: every segment's steps by SDC15 instead of DOP853)
static int seg_run(ww_ctx* c, const double* params, double T, int nseg, const ww_segment* sg, double* r, double* J,
                   double* drdT, double* f, int* st, int* where, bool sdc) {
  const bool cols = (J != nullptr) && c->M > 0;
  const bool two = c->overlap && !pivoted(c);
  const bool sdc_two = sdc && two && !c->gm_active;
  int rc;
  if (pivoted(c) && (rc = ensure_pivot_buffers(c))) return rc;
  if (sdc && (rc = ensure_sdc(c))) return rc;
  if (sdc_two && (rc = ensure_sdc_groups(c))) return rc;
  if (!c->mesh && (rc = dalloc(c, (void**)&c->mesh, (size_t)MESH_COUNT * c->n_max * 8))) return rc;
  for (int l = 0; l < nseg; ++l) {
    const double Tl = sg[l].theta * T;
    const double Al = mesh_coef(sg[l].rho);
    // this segment's mesh tables, before anything of the segment is enqueued (the
    // lagged march's prologue assembles the segment's first surface)
    auto tables = [&]() -> int {
      hipLaunchKernelGGL(k_mesh_tables, dim3((sg[l].N + 255) / 256), dim3(256), 0, c->stream, c->mesh, c->n_max,
                         sg[l].N, Al, sg[l].refine_at);
      LAUNCHCHK();
      return 0;
    };
    if (l == 0) {
      if ((rc = pipe_join(c))) return rc;   // a previous march's streams
      if ((rc = tables())) return rc;
      if (sdc) {   // the state only: no Runge-Kutta step graph
        const bool ug = c->use_graph;
        c->use_graph = false;
        rc = shoot_prepare(c, params, Tl, sg[0].nsteps, cols, false);
        c->use_graph = ug;
        if (rc) return rc;
      } else if ((rc = shoot_prepare(c, params, Tl, sg[0].nsteps, cols, two))) {
        return rc;
      }
    } else {
      if ((rc = pipe_join(c))) return rc;   // the lagged march's LU and column streams
      const int No = c->N, Nn = sg[l].N;
      const int ncols = 2 * (cols ? c->M + 1 : 1);
      // interpolation weights (row-major Nn x No, in the A buffer of the default factor
      // set, free between segments), then the old state to the stage buffer
      hipLaunchKernelGGL(k_regrid_w, dim3(Nn), dim3(WW_NT), 0, c->stream, c->A, Nn, No, Al, sg[l].refine_at,
                         mesh_coef(sg[l - 1].rho), sg[l - 1].refine_at);
      LAUNCHCHK();
      HIPCHK(hipMemcpyAsync(c->Ys, c->y, (size_t)ncols * No * 8, hipMemcpyDeviceToDevice, c->stream));
      if ((rc = set_grid(c, Nn, c->shootH))) return rc;
      hipLaunchKernelGGL(k_regrid_apply, dim3((Nn + 63) / 64, (ncols + 63) / 64), dim3(WW_NT), 0, c->stream, c->A,
                         c->Ys, c->y, Nn, No, ncols);
      LAUNCHCHK();
      if (sdc) {
        if ((rc = tables())) return rc;
      } else {
      double coef[COEF_SIZE];
      coef_fill(c, Tl, sg[l].nsteps, coef);
      HIPCHK(hipStreamSynchronize(c->stream));
      HIPCHK(hipMemcpy(c->coef, coef, sizeof(coef), hipMemcpyHostToDevice));
      if ((rc = tables())) return rc;
      if (pipelined(c, cols, two)) {
        // lagged factors restart on the new mesh: the prologue factors the segment's
        // first surface into the sets its first stages read
        if ((rc = ensure_pipe(c))) return rc;
        if ((rc = pipe_prologue(c))) return rc;
        if (graphed(c) && (rc = ensure_pipe_graphs(c))) return rc;
      } else if (graphed(c) && (rc = ensure_step_graph(c, cols, two))) {
        return rc;
      }
      }
    }
    if (sdc) {
      if ((rc = sdc_steps(c, cols, Tl / (4.0 * sg[l].nsteps), sg[l].nsteps, sdc_two))) return rc;
    } else {
      for (int n = 0; n < sg[l].nsteps; ++n)
        if ((rc = shoot_one_step(c, cols, two))) return rc;
    }
  }
  if ((rc = shoot_finish(c, cols, r, J, drdT, f))) {
    const std::string msg = g_err;
    (void)pipe_join(c);
    (void)hipStreamSynchronize(c->stream);
    g_err = msg;
    return rc;
  }
  return read_status(c, st, where);
}

// ----- SDC15 time stepping (Sec. 2.2) -----
// Legendre polynomial P_n(x) and its derivative by the three-term recurrence
static void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// Radau IIa nodes on (0, 1]: zeros of P_8(x) - P_7(x), x = 2c - 1, found by a sign scan
// and bisection to the last bit; the last node is c = 1
static void radau_nodes(double* c) {
  auto f = [](double x) {
    double a, b, da, db;
    legendre(SDC_NODES, x, &a, &da);
    legendre(SDC_NODES - 1, x, &b, &db);
    return a - b;
  };
  int n = 0;
  const int grid = 4096;
  double xl = -1.0, fl = f(xl);
  for (int g = 1; g < grid && n < SDC_NODES - 1; ++g) {
    const double xr = -1.0 + 2.0 * g / grid, fr = f(xr);
    if ((fl < 0) != (fr < 0)) {
      double a = xl, b = xr, fa = fl;
      for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (m == a || m == b) break;
        const double fm = f(m);
        if ((fm < 0) == (fa < 0)) {
          a = m;
          fa = fm;
        } else {
          b = m;
        }
      }
      c[n++] = 0.5 * (0.5 * (a + b) + 1.0);
    }
    xl = xr;
    fl = fr;
  }
  c[SDC_NODES - 1] = 1.0;
}

// S[m][j] = integral from 0 to c_m of node j's Lagrange polynomial, by 16-point
// Gauss-Legendre quadrature (nodes by Newton's method on P_16)
static void radau_integration(const double* c, double S[SDC_NODES][SDC_NODES]) {
  const int ng = 16;
  double xg[ng], wg[ng];
  for (int i = 0; i < ng; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (ng + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(ng, x, &p, &dp);
      const double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p, dp;
    legendre(ng, x, &p, &dp);
    xg[i] = x;
    wg[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  for (int m = 0; m < SDC_NODES; ++m)
    for (int j = 0; j < SDC_NODES; ++j) {
      double acc = 0.0;
      for (int q = 0; q < ng; ++q) {
        const double x = 0.5 * c[m] * (xg[q] + 1.0);
        double ell = 1.0;
        for (int k = 0; k < SDC_NODES; ++k)
          if (k != j) ell *= (x - c[k]) / (c[j] - c[k]);
        acc += wg[q] * ell;
      }
      S[m][j] = 0.5 * c[m] * acc;
    }
}

// The SDC15 step as an explicit method: rows 0..SDC_STAGES-1 give stage s's state
// y_0 + dt sum w K_j (slots j < s), row SDC_STAGES the step's result.  Slots: RK4 from
// node to node (4 per node), F at the last predicted node, then F at the nodes of each
// of the ten sweeps.
static void sdc_rows(int* cnt, int (*jt)[SDC_MAXNZ], double (*wt)[SDC_MAXNZ]) {
  double c[SDC_NODES], S[SDC_NODES][SDC_NODES];
  radau_nodes(c);
  radau_integration(c, S);
  std::vector<double> cur(SDC_STAGES, 0.0);   // the running state's weights on the slots
  auto put = [&](int row, const std::vector<double>& v) {
    int n = 0;
    for (int j = 0; j < SDC_STAGES; ++j)
      if (v[j] != 0.0) {
        jt[row][n] = j;
        wt[row][n] = v[j];
        ++n;
      }
    cnt[row] = n;
  };
  int slot = 0;
  double t = 0.0;
  int fnode[SDC_NODES];   // slot holding F at each node of the current iterate
  for (int m = 0; m < SDC_NODES; ++m) {
    const double h = c[m] - t;
    const int s1 = slot++, s2 = slot++, s3 = slot++, s4 = slot++;
    std::vector<double> v = cur;
    put(s1, v);
    v = cur;
    v[s1] += h / 2;
    put(s2, v);
    v = cur;
    v[s2] += h / 2;
    put(s3, v);
    v = cur;
    v[s3] += h;
    put(s4, v);
    cur[s1] += h / 6;
    cur[s2] += h / 3;
    cur[s3] += h / 3;
    cur[s4] += h / 6;
    if (m > 0) fnode[m - 1] = s1;   // F at the node just reached (k1 of the next interval)
    t = c[m];
  }
  fnode[SDC_NODES - 1] = slot;
  put(slot++, cur);
  for (int k = 0; k < SDC_SWEEPS; ++k) {
    int nf[SDC_NODES];
    for (int m = 0; m < SDC_NODES; ++m) {
      std::vector<double> v(SDC_STAGES, 0.0);
      for (int j = 0; j < SDC_NODES; ++j) v[fnode[j]] += S[m][j];
      nf[m] = slot;
      put(slot++, v);
    }
    for (int m = 0; m < SDC_NODES; ++m) fnode[m] = nf[m];
  }
  std::vector<double> v(SDC_STAGES, 0.0);
  for (int j = 0; j < SDC_NODES; ++j) v[fnode[j]] += S[SDC_NODES - 1][j];
  put(SDC_STAGES, v);
}

static int ensure_sdc(ww_ctx* c) {
  if (c->sdc_K) return 0;
  int rc;
  const size_t st = (size_t)2 * c->n_max * c->r_max;
  // each buffer once (a failed call leaves the others for the next)
  if (!c->sdc_y && (rc = dalloc(c, (void**)&c->sdc_y, st * 8))) return rc;
  if (!c->sdc_yn && (rc = dalloc(c, (void**)&c->sdc_yn, SDC_NODES * st * 8))) return rc;
  if (!c->sdc_ysn && (rc = dalloc(c, (void**)&c->sdc_ysn, SDC_NODES * st * 8))) return rc;
  if (!c->sdc_rhsn && (rc = dalloc(c, (void**)&c->sdc_rhsn, (size_t)SDC_NODES * c->np_max * 8))) return rc;
  if (!c->sdc_j && (rc = dalloc(c, (void**)&c->sdc_j, (SDC_STAGES + 1) * SDC_MAXNZ * sizeof(int)))) return rc;
  if (!c->sdc_w && (rc = dalloc(c, (void**)&c->sdc_w, (SDC_STAGES + 1) * SDC_MAXNZ * 8))) return rc;
  std::vector<int> jt((SDC_STAGES + 1) * SDC_MAXNZ, 0);
  std::vector<double> wt((SDC_STAGES + 1) * SDC_MAXNZ, 0.0);
  sdc_rows(c->sdc_cnt, reinterpret_cast<int(*)[SDC_MAXNZ]>(jt.data()), reinterpret_cast<double(*)[SDC_MAXNZ]>(wt.data()));
  HIPCHK(hipMemcpy(c->sdc_j, jt.data(), jt.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->sdc_w, wt.data(), wt.size() * 8, hipMemcpyHostToDevice));
  // sdc_K last: its presence marks the set-up as complete
  return dalloc(c, (void**)&c->sdc_K, (size_t)SDC_STAGES * st * 8);
}

// the base and column right-hand sides of an SDC stage (mapped-grid kernels on a
// non-uniform mesh)
static int sdc_base_rhs(ww_ctx* c, const double* Ys, const double* gphi, double* aux, double* kout) {
  if (c->mapped)
    hipLaunchKernelGGL(k_base_rhs_map, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, Ys, gphi, aux,
                       c->mesh, c->n_max, kout, (unsigned long long*)nullptr, 0.0, (int*)nullptr, c->tw, c->sig, c->N,
                       c->g, c->tau);
  else
    hipLaunchKernelGGL(k_base_rhs, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, Ys, gphi, aux, c->n_max,
                       kout, (unsigned long long*)nullptr, 0.0, (int*)nullptr, c->tw, c->sig, c->N, c->g, c->tau);
  LAUNCHCHK();
  return 0;
}
static int sdc_col_rhs(ww_ctx* c, const double* Ys, const double* aux, double* kout) {
  if (c->mapped)
    hipLaunchKernelGGL(k_col_rhs_map, dim3(c->M), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, Ys, c->Gpsi, c->Np,
                       aux, c->mesh, c->n_max, kout, c->tw, c->sig, c->N, c->g, c->tau);
  else
    hipLaunchKernelGGL(k_col_rhs, dim3(c->M), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, Ys, c->Gpsi, c->Np, aux,
                       c->n_max, kout, c->tw, c->sig, c->N, c->g, c->tau);
  LAUNCHCHK();
  return 0;
}

// the factor sets, the LU and column streams and the lane events of the two-stream form
// (first use)
static int ensure_sdc_groups(ww_ctx* c) {
  if (!c->lus[0]) HIPCHK(hipStreamCreateWithFlags(&c->lus[0], hipStreamNonBlocking));
  if (!c->side) HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  if (!c->sdc_ev) HIPCHK(hipEventCreateWithFlags(&c->sdc_ev, hipEventDisableTiming));
  for (int i = 0; i < SDC_NODES; ++i) {
    if (!c->sdc_evB[i]) HIPCHK(hipEventCreateWithFlags(&c->sdc_evB[i], hipEventDisableTiming));
    if (!c->sdc_evC[i]) HIPCHK(hipEventCreateWithFlags(&c->sdc_evC[i], hipEventDisableTiming));
    if (!c->sdc_evL[i]) HIPCHK(hipEventCreateWithFlags(&c->sdc_evL[i], hipEventDisableTiming));
  }
  int rc;
  if (!c->sdc_b2 && (rc = dalloc(c, (void**)&c->sdc_b2, (size_t)6 * c->np_max * 8))) return rc;
  return ensure_ring(c, SDC_NODES);
}

// The two-stream form of an SDC15 step.  Stage s runs in lane q (predictor stages
// s mod SDC_NODES, the nodes of a sweep their node index): the lane's factor set of the
// ring, stage state, stage-state copy and base Dirichlet data.  The main stream forms
// the base column of the stage state, the spectral prep, the assembly, the LU and the
// base chain; the column stream then forms the Jacobian columns of the stage state and
// runs the column chain, overlapping the next stages' base chains and LUs.  A lane is
// taken again only after its column chain has ended.  The nodes of a correction sweep
// read only slopes of earlier sweeps: they are assembled together and factored in two
// groups of four, the second on the LU stream, where its base chains follow.  The
// predictor's second and third RK4 stages solve their base equations on the factors of
// their interval's first stage (lagged(), below).  Without those lagged
// solves (WW_SDC_LAG=0) the kernels and their order per element are those of the
// one-stream form, and the results are the same bit for bit.
struct SdcStep {
  ww_ctx* c;
  bool cols;
  double dt;
  size_t ks;
  Fac F[SDC_NODES];
  int lastq = -1;   // lane of the last column chain
  // base-chain scratch: the context's (main stream), and a second set for the chains
  // that run on the LU stream
  struct Bs {
    double *y0t, *mu0, *gam0, *hg0, *gphi0, *rr0;
  } bm, b2;

  bool lag;   // lagged factors for the predictor's base solves

  SdcStep(ww_ctx* cc, bool cl, double d) : c(cc), cols(cl), dt(d), ks(kstride(cc)) {
    for (int m = 0; m < SDC_NODES; ++m) {
      F[m] = pipe_set(c, m, false);
      F[m].lag32 = false;
      F[m].Gm = nullptr;   // the chains read Gm row-major only
    }
    lag = c->sdc_lag && !(c->fb & WW_FB_DIRECT);
    bm = Bs{c->y0t, c->mu0, c->gam0, c->hg0, c->gphi0, c->rr0};
    const size_t np = c->np_max;
    double* w = c->sdc_b2;
    b2 = Bs{w, w + np, w + 2 * np, w + 3 * np, w + 4 * np, w + 5 * np};
  }
  double* yn(int q) const { return c->sdc_yn + q * ks; }
  double* ysn(int q) const { return c->sdc_ysn + q * ks; }
  double* rhsn(int q) const { return c->sdc_rhsn + (size_t)q * c->Np; }

  // combination of row s into lane q: the base column (part 0) or the Jacobian columns
  int combine(int s, int q, bool colpart) {
    const size_t off = colpart ? (size_t)2 * c->N : 0;
    const size_t n = (size_t)2 * c->N * (colpart ? c->M : 1);
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sdc_combine, dim3(blocks), dim3(256), 0, c->stream, c->y + off, c->sdc_K + off, ks,
                       c->sdc_j + s * SDC_MAXNZ, c->sdc_w + s * SDC_MAXNZ, c->sdc_cnt[s], dt, yn(q) + off, n);
    LAUNCHCHK();
    return 0;
  }
  // main stream: the lane is free, the stage state's base column, prep, assembly (with
  // the row-major FP64 A of the lagged solves' residuals when want_ar)
  int front(int s, int q, bool want_ar = false) {
    int rc;
    HIPCHK(hipStreamWaitEvent(c->stream, c->sdc_evC[q], 0));
    if ((rc = combine(s, q, false))) return rc;
    hipLaunchKernelGGL(k_base_prep, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, yn(q), c->K, ysn(q),
                       c->coef, 0, ks, F[q].aux, c->n_max, rhsn(q), c->Np, c->tw, c->N, c->hsurf, c->status);
    LAUNCHCHK();
    return enqueue_assemble(c, F[q], want_ar);
  }
  // A predictor stage on lagged factors (lane q, the factors of lane qb): its own LU on
  // the LU stream, read only by its column chain (so none without columns: the lane's
  // next assembly then has nothing to wait for); the base solve x = Mi_b psi refined
  // by LAG_SWEEPS sweeps (environment WW_SDC_LAG_SWEEPS) r = psi - A x, x += Mi_b r
  // against its own matrix, the 2^-43 test on the final residual (status bit 32: the
  // march is redone on direct factors),
  // then gamma, G phi and the right-hand side as in the direct chain
  int lagged(int s, int q, int qb) {
    int rc;
    if ((rc = front(s, q, true))) return rc;
    const hipStream_t main = c->stream, ls = c->lus[0];
    if (cols) {
      HIPCHK(hipEventRecord(c->sdc_ev, main));
      HIPCHK(hipStreamWaitEvent(ls, c->sdc_ev, 0));
      c->stream = ls;
      rc = enqueue_lu(c, F[q]);
      c->stream = main;
      if (rc) return rc;
      HIPCHK(hipEventRecord(c->sdc_evL[q], ls));
    }
    if ((rc = lagged_base(s, q, qb, bm))) return rc;
    double* kout = c->sdc_K + (size_t)s * ks;
    if (!cols) return 0;
    // the column chain: after the base chain and the stage's own LU
    HIPCHK(hipEventRecord(c->sdc_evB[q], main));
    HIPCHK(hipStreamWaitEvent(c->side, c->sdc_evB[q], 0));
    HIPCHK(hipStreamWaitEvent(c->side, c->sdc_evL[q], 0));
    c->stream = c->side;
    rc = col_chain(s, q, kout);
    c->stream = main;
    if (rc) return rc;
    HIPCHK(hipEventRecord(c->sdc_evC[q], c->side));
    lastq = q;
    return 0;
  }
  // The base solve of stage s (lane q, assembled with its row-major A) on the inverse of
  // lane qb, refined against its own matrix (the 2^-43 test, status bit 32), then gamma,
  // G phi and the right-hand side into slot s, on the current stream with scratch b
  int lagged_base(int s, int q, int qb, const Bs& b) {
    int rc;
    double* psi = rhsn(q);
    // x (+)= Mi_b B with the lagged inverse: FP64, or its FP32 copy in the mixed form
    auto lag_mul = [&](const double* B, const double* add, double* out) {
      return F[qb].use32 ? enqueue_gemm<float>(c, F[qb].Mi32, 0, B, add, 1.0, out, 1)
                         : enqueue_gemm<double>(c, F[qb].Mi, 0, B, add, 1.0, out, 1);
    };
    if ((rc = lag_mul(psi, nullptr, b.mu0))) return rc;
    for (int it = 0; it < c->sdc_lag_sweeps; ++it) {
      if ((rc = enqueue_gemm<double>(c, F[q].Ar, 0, b.mu0, psi, -1.0, b.rr0, 1))) return rc;
      if ((rc = lag_mul(b.rr0, b.mu0, b.mu0))) return rc;
    }
    if ((rc = enqueue_gemm<double>(c, F[q].Ar, 0, b.mu0, psi, -1.0, b.rr0, 1))) return rc;
    hipLaunchKernelGGL(k_gamma, dim3(1), dim3(WW_NT), fft_lds_bytes(c->N, 4), c->stream, b.mu0, c->Np, 1, b.gam0,
                       b.hg0, c->tw, c->N, b.rr0, psi, REFINE_TOL, c->status, 32);
    LAUNCHCHK();
    if ((rc = enqueue_gemm<double>(c, F[q].Gmr, 0, b.gam0, b.hg0, 1.0, b.gphi0, 1))) return rc;
    return sdc_base_rhs(c, ysn(q), b.gphi0, F[q].aux, c->sdc_K + (size_t)s * ks);
  }
  // the base solve and right-hand side (slot s) on the current stream with scratch b,
  // then the column chain on the column stream
  int chains(int s, int q, const Bs& b) {
    int rc;
    double* kout = c->sdc_K + (size_t)s * ks;
    if ((rc = enqueue_dtn_cols(c, F[q], rhsn(q), b.y0t, b.mu0, b.gam0, b.hg0, b.gphi0, b.rr0, 1))) return rc;
    if ((rc = sdc_base_rhs(c, ysn(q), b.gphi0, F[q].aux, kout))) return rc;
    if (!cols) return 0;
    HIPCHK(hipEventRecord(c->sdc_evB[q], c->stream));
    const hipStream_t main = c->stream;
    HIPCHK(hipStreamWaitEvent(c->side, c->sdc_evB[q], 0));
    c->stream = c->side;
    rc = col_chain(s, q, kout);
    c->stream = main;
    if (rc) return rc;
    HIPCHK(hipEventRecord(c->sdc_evC[q], c->side));
    lastq = q;
    return 0;
  }
  int col_chain(int s, int q, double* kout) {
    int rc;
    if ((rc = combine(s, q, true))) return rc;
    const int M = c->M;
    const size_t tot = (size_t)c->Np * M;
    const int cb = (int)std::min<size_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_col_pre, dim3(cb), dim3(256), 0, c->stream, yn(q), c->K, ysn(q), c->coef, 0, ks, F[q].aux,
                       c->n_max, c->Psi, c->Np, c->N, M);
    LAUNCHCHK();
    if ((rc = enqueue_dtn_cols(c, F[q], c->Psi, c->Ytmp, c->Mu, c->Gam, c->HG, c->Gpsi, c->Rr, M))) return rc;
    return sdc_col_rhs(c, ysn(q), F[q].aux, kout);
  }
  int sweep(int s0) {
    static_assert(SDC_NODES == 2 * BLU_GMAX, "a sweep is factored in two groups");
    int rc;
    const int G = BLU_GMAX;
    const hipStream_t main = c->stream, ls = c->lus[0];
    // the second group first, so that its LU runs beside the first group's work
    // Without columns, the sweeps after the first solve each node on the factors the
    // first sweep made for the same node (the node's surface moves only by the shrinking
    // Picard corrections), refined to the 2^-43 test; no LU
    if (!cols && lag && s0 > SDC_FIRST_SWEEP) {
      for (int m = G; m < SDC_NODES; ++m)
        if ((rc = front(s0 + m, m, true))) return rc;
      HIPCHK(hipEventRecord(c->sdc_ev, main));
      HIPCHK(hipStreamWaitEvent(ls, c->sdc_ev, 0));
      c->stream = ls;
      for (int m = G; m < SDC_NODES && !rc; ++m) rc = lagged_base(s0 + m, m, m, b2);
      c->stream = main;
      if (rc) return rc;
      HIPCHK(hipEventRecord(c->sdc_ev, ls));
      for (int m = 0; m < G; ++m) {
        if ((rc = front(s0 + m, m, true))) return rc;
        if ((rc = lagged_base(s0 + m, m, m, bm))) return rc;
      }
      HIPCHK(hipStreamWaitEvent(main, c->sdc_ev, 0));
      return 0;
    }
    // (its base chains follow on the LU stream with the second scratch set)
    for (int m = G; m < SDC_NODES; ++m)
      if ((rc = front(s0 + m, m))) return rc;
    HIPCHK(hipEventRecord(c->sdc_ev, main));
    HIPCHK(hipStreamWaitEvent(ls, c->sdc_ev, 0));
    c->stream = ls;
    rc = enqueue_lu_group(c, F + G, G);
    for (int m = G; m < SDC_NODES && !rc; ++m) rc = chains(s0 + m, m, b2);
    c->stream = main;
    if (rc) return rc;
    HIPCHK(hipEventRecord(c->sdc_ev, ls));
    for (int m = 0; m < G; ++m)
      if ((rc = front(s0 + m, m))) return rc;
    if ((rc = enqueue_lu_group(c, F, G))) return rc;
    for (int m = 0; m < G; ++m)
      if ((rc = chains(s0 + m, m, bm))) return rc;
    // the next stages read this sweep's slopes
    HIPCHK(hipStreamWaitEvent(main, c->sdc_ev, 0));
    return 0;
  }
  int step() {
    int rc;
    for (int s = 0; s < SDC_STAGES;) {
      if (s >= SDC_FIRST_SWEEP) {
        if ((rc = sweep(s))) return rc;
        s += SDC_NODES;
        continue;
      }
      const int q = s % SDC_NODES;
      // the second and third RK4 stages of each node interval (half an interval from its
      // first) solve with the first stage's factors when lagging; the others factor on
      // the main stream
      const int sb = s / 4 * 4;
      if (lag && s < 4 * SDC_NODES && (s % 4 == 1 || s % 4 == 2)) {
        if ((rc = lagged(s, q, sb % SDC_NODES))) return rc;
      } else {
        if ((rc = front(s, q))) return rc;
        if ((rc = enqueue_lu(c, F[q]))) return rc;
        if ((rc = chains(s, q, bm))) return rc;
      }
      ++s;
    }
    // the step's combination in place (after the last column chain) and the filter
    if (lastq >= 0) HIPCHK(hipStreamWaitEvent(c->stream, c->sdc_evC[lastq], 0));
    const size_t n = (size_t)2 * c->N * (cols ? c->M + 1 : 1);
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sdc_combine, dim3(blocks), dim3(256), 0, c->stream, c->y, c->sdc_K, ks,
                       c->sdc_j + SDC_STAGES * SDC_MAXNZ, c->sdc_w + SDC_STAGES * SDC_MAXNZ, c->sdc_cnt[SDC_STAGES],
                       dt, c->y, n);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_step_end, dim3(cols ? c->M + 1 : 1), dim3(WW_NT), fft_lds_bytes(c->N, 3), c->stream, c->y,
                       c->K, ks, 0, c->coef, c->tw, c->sig, c->N, 0, c->status);
    LAUNCHCHK();
    return 0;
  }
};

// the column chain of a stage whose state is ysrc (no stage combination), slopes to kout
static int enqueue_col_chain_at(ww_ctx* c, const double* ysrc, double* kout, const Fac& F) {
  int rc;
  const int M = c->M;
  const size_t tot = (size_t)c->Np * M;
  const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_col_pre, dim3(blocks), dim3(256), 0, c->stream, ysrc, c->K, c->Ys, c->coef, 0, kstride(c),
                     F.aux, c->n_max, c->Psi, c->Np, c->N, M);
  LAUNCHCHK();
  if ((rc = enqueue_dtn_cols(c, F, c->Psi, c->Ytmp, c->Mu, c->Gam, c->HG, c->Gpsi, c->Rr, M))) return rc;
  return sdc_col_rhs(c, c->Ys, F.aux, kout);
}

// one SDC15 step of dt: every stage's state by k_sdc_combine, its base chain and column
// chain on the context's stream (each stage on its own factors), then the step's
// combination in place and the filter
static int enqueue_sdc_step(ww_ctx* c, bool cols, double dt) {
  int rc;
  const size_t ks = kstride(c);
  const size_t n = (size_t)2 * c->N * (cols ? c->M + 1 : 1);
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  const Fac F = fac_default(c);
  for (int s = 0; s <= SDC_STAGES; ++s) {
    double* dst = s < SDC_STAGES ? c->sdc_y : c->y;
    hipLaunchKernelGGL(k_sdc_combine, dim3(blocks), dim3(256), 0, c->stream, c->y, c->sdc_K, ks,
                       c->sdc_j + s * SDC_MAXNZ, c->sdc_w + s * SDC_MAXNZ, c->sdc_cnt[s], dt, dst, n);
    LAUNCHCHK();
    if (s == SDC_STAGES) break;
    double* kout = c->sdc_K + (size_t)s * ks;
    if ((rc = enqueue_base_chain(c, c->sdc_y, 0, kout, F))) return rc;
    if (cols && (rc = enqueue_col_chain_at(c, c->sdc_y, kout, F))) return rc;
  }
  // the filter (no stage terms) and the step count
  hipLaunchKernelGGL(k_step_end, dim3(cols ? c->M + 1 : 1), dim3(WW_NT), fft_lds_bytes(c->N, 3), c->stream, c->y,
                     c->K, ks, 0, c->coef, c->tw, c->sig, c->N, 0, c->status);
  LAUNCHCHK();
  return 0;
}

static int sdc_steps(ww_ctx* c, bool cols, double dt, int nsteps, bool two) {
  int rc;
  if (!two) {
    for (int n = 0; n < nsteps; ++n)
      if ((rc = enqueue_sdc_step(c, cols, dt))) return rc;
    return 0;
  }
  // every lane starts free
  for (int q = 0; q < SDC_NODES; ++q) HIPCHK(hipEventRecord(c->sdc_evC[q], c->stream));
  for (int n = 0; n < nsteps; ++n) {
    SdcStep st(c, cols, dt);
    if ((rc = st.step())) {
      // nothing of the march may still run on the column or LU stream
      const std::string msg = g_err;
      (void)hipStreamSynchronize(c->side);
      (void)hipStreamSynchronize(c->lus[0]);
      (void)hipStreamSynchronize(c->stream);
      g_err = msg;
      return rc;
    }
  }
  return 0;
}

static int sdc_run(ww_ctx* c, const double* params, double T, int nsteps, double* r, double* J, double* drdT,
                   double* f, int* st, int* where) {
  const bool cols = (J != nullptr) && c->M > 0;
  int rc;
  if (pivoted(c) && (rc = ensure_pivot_buffers(c))) return rc;
  if ((rc = ensure_sdc(c))) return rc;
  const bool ug = c->use_graph;
  c->use_graph = false;   // the Runge-Kutta step graph is not used here
  rc = shoot_prepare(c, params, T, nsteps, cols, false);
  c->use_graph = ug;
  if (rc) return rc;
  // the two-stream form, except in the pivoted and GMRES forms (one row order, one
  // Krylov workspace per context) and in a one-stream context
  const bool two = c->overlap && !pivoted(c) && !c->gm_active;
  if (two && (rc = ensure_sdc_groups(c))) return rc;
  if ((rc = sdc_steps(c, cols, T / (4.0 * nsteps), nsteps, two))) return rc;
  if ((rc = shoot_finish(c, cols, r, J, drdT, f))) {
    const std::string msg = g_err;
    (void)hipStreamSynchronize(c->stream);
    g_err = msg;
    return rc;
  }
  return read_status(c, st, where);
}

// ----- the base march in double-double (SDC15 of the quadruple-precision workflow) -----
// P_n and P_{n-1} at x in double-double (three-term recurrence)
static void legendre_dd(int n, dd x, dd* pn, dd* pn1) {
  dd p0 = dd_of(1.0), p1 = x;
  for (int k = 2; k <= n; ++k) {
    const dd p2 = dd_div_d(dd_sub(dd_mul_d(dd_mul(x, p1), 2.0 * k - 1.0), dd_mul_d(p0, k - 1.0)), (double)k);
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *pn1 = p0;
}

// The Radau IIa nodes and the integration matrix to about 32 digits: the double nodes
// (and the double Gauss-Legendre rule) refined by Newton steps on the double-double
// polynomial values, then S_mj = (c_m / 2) sum_q w_q l_j(c_m (x_q + 1) / 2) in
// double-double
static void radau_dd(dd* c, dd S[SDC_NODES][SDC_NODES]) {
  double c0[SDC_NODES];
  radau_nodes(c0);
  for (int m = 0; m < SDC_NODES - 1; ++m) {
    dd x = dd_of(2.0 * c0[m] - 1.0);
    for (int it = 0; it < 3; ++it) {
      dd p8, p7;
      legendre_dd(SDC_NODES, x, &p8, &p7);
      double a, b, da, db;
      legendre(SDC_NODES, x.hi, &a, &da);
      legendre(SDC_NODES - 1, x.hi, &b, &db);
      x = dd_add_d(x, -dd_sub(p8, p7).hi / (da - db));
    }
    c[m] = dd_mul_d(dd_add_d(x, 1.0), 0.5);
  }
  c[SDC_NODES - 1] = dd_of(1.0);
  const int ng = 16;
  dd xg[ng], wg[ng];
  for (int i = 0; i < ng; ++i) {
    double x0 = std::cos(M_PI * (i + 0.75) / (ng + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(ng, x0, &p, &dp);
      const double dx = p / dp;
      x0 -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    dd x = dd_of(x0), pn, pn1;
    for (int it = 0; it < 3; ++it) {
      legendre_dd(ng, x, &pn, &pn1);
      double p, dp;
      legendre(ng, x.hi, &p, &dp);
      x = dd_add_d(x, -pn.hi / dp);
    }
    legendre_dd(ng, x, &pn, &pn1);
    const dd x2m1 = dd_add_d(dd_mul(x, x), -1.0);   // x^2 - 1
    const dd dp = dd_div(dd_mul_d(dd_sub(dd_mul(x, pn), pn1), (double)ng), x2m1);
    xg[i] = x;
    wg[i] = dd_div(dd_of(2.0), dd_mul(dd_neg(x2m1), dd_mul(dp, dp)));   // 2 / ((1 - x^2) P'^2)
  }
  for (int m = 0; m < SDC_NODES; ++m)
    for (int j = 0; j < SDC_NODES; ++j) {
      dd acc = dd_of(0.0);
      for (int q = 0; q < ng; ++q) {
        const dd x = dd_mul(dd_mul_d(c[m], 0.5), dd_add_d(xg[q], 1.0));
        dd ell = dd_of(1.0);
        for (int k = 0; k < SDC_NODES; ++k)
          if (k != j) ell = dd_mul(ell, dd_div(dd_sub(x, c[k]), dd_sub(c[j], c[k])));
        acc = dd_add(acc, dd_mul(wg[q], ell));
      }
      S[m][j] = dd_mul(dd_mul_d(c[m], 0.5), acc);
    }
}

// The stage rows of sdc_rows with double-double weights, each times dt
static void sdc_rows_dd(dd dt, int* cnt, int (*jt)[SDC_MAXNZ], double (*wh)[SDC_MAXNZ], double (*wl)[SDC_MAXNZ]) {
  dd c[SDC_NODES], S[SDC_NODES][SDC_NODES];
  radau_dd(c, S);
  const dd zero = dd_of(0.0);
  std::vector<dd> cur(SDC_STAGES, zero);
  auto put = [&](int row, const std::vector<dd>& v) {
    int n = 0;
    for (int j = 0; j < SDC_STAGES; ++j)
      if (v[j].hi != 0.0) {
        const dd w = dd_mul(v[j], dt);
        jt[row][n] = j;
        wh[row][n] = w.hi;
        wl[row][n] = w.lo;
        ++n;
      }
    cnt[row] = n;
  };
  int slot = 0;
  dd t = zero;
  int fnode[SDC_NODES];
  for (int m = 0; m < SDC_NODES; ++m) {
    const dd h = dd_sub(c[m], t);
    const dd h2 = dd_mul_d(h, 0.5), h3 = dd_div_d(h, 3.0), h6 = dd_div_d(h, 6.0);
    const int s1 = slot++, s2 = slot++, s3 = slot++, s4 = slot++;
    std::vector<dd> v = cur;
    put(s1, v);
    v = cur;
    v[s1] = dd_add(v[s1], h2);
    put(s2, v);
    v = cur;
    v[s2] = dd_add(v[s2], h2);
    put(s3, v);
    v = cur;
    v[s3] = dd_add(v[s3], h);
    put(s4, v);
    cur[s1] = dd_add(cur[s1], h6);
    cur[s2] = dd_add(cur[s2], h3);
    cur[s3] = dd_add(cur[s3], h3);
    cur[s4] = dd_add(cur[s4], h6);
    if (m > 0) fnode[m - 1] = s1;
    t = c[m];
  }
  fnode[SDC_NODES - 1] = slot;
  put(slot++, cur);
  for (int k = 0; k < SDC_SWEEPS; ++k) {
    int nf[SDC_NODES];
    for (int m = 0; m < SDC_NODES; ++m) {
      std::vector<dd> v(SDC_STAGES, zero);
      for (int j = 0; j < SDC_NODES; ++j) v[fnode[j]] = dd_add(v[fnode[j]], S[m][j]);
      nf[m] = slot;
      put(slot++, v);
    }
    for (int m = 0; m < SDC_NODES; ++m) fnode[m] = nf[m];
  }
  std::vector<dd> v(SDC_STAGES, zero);
  for (int j = 0; j < SDC_NODES; ++j) v[fnode[j]] = dd_add(v[fnode[j]], S[SDC_NODES - 1][j]);
  put(SDC_STAGES, v);
}

static int ensure_sdc_dd(ww_ctx* c) {
  if (c->sdd_fo) return 0;
  int rc;
  const size_t n2 = (size_t)2 * c->n_max, nm = c->n_max, rows = (size_t)(SDC_STAGES + 1) * SDC_MAXNZ;
  double** st[] = {&c->sdd_yh, &c->sdd_yl, &c->sdd_Yh, &c->sdd_Yl};
  for (double** q : st)
    if (!*q && (rc = dalloc(c, (void**)q, n2 * 8))) return rc;
  double** sl[] = {&c->sdd_Kh, &c->sdd_Kl};
  for (double** q : sl)
    if (!*q && (rc = dalloc(c, (void**)q, (SDC_STAGES + 1) * n2 * 8))) return rc;
  double** pt[] = {&c->sdd_Gh, &c->sdd_Gl, &c->sdd_fh, &c->sdd_fl};
  for (double** q : pt)
    if (!*q && (rc = dalloc(c, (void**)q, nm * 8))) return rc;
  double** wr[] = {&c->sdd_wh, &c->sdd_wl};
  for (double** q : wr)
    if (!*q && (rc = dalloc(c, (void**)q, rows * 8))) return rc;
  if (!c->sdd_j && (rc = dalloc(c, (void**)&c->sdd_j, rows * sizeof(int)))) return rc;
  return dalloc(c, (void**)&c->sdd_fo, 64);   // last: its presence marks the set-up as complete
}

// the status of the double-double march after step n (n < 0: at T/4), as an error
static int dd_march_status(ww_ctx* c, int n) {
  int st = 0, rc;
  if ((rc = read_status(c, &st))) return rc;
  const std::string at = n >= 0 ? " (double-double march, step " + std::to_string(n) + ")" : " (double-double march)";
  if (st & 16) return fail(WW_EDOMAIN, "finite depth: surface height h + eta <= 0" + at);
  if (st & 2) return fail(WW_ENONFINITE, "non-finite surface" + at);
  if (st & (1 | 8)) return fail(WW_EPIVOT, "double-double DtN: pivot below the guard" + at);
  if (st & 4) return fail(WW_EREFINE, "double-double DtN: residual above 2^-96 of the right-hand side" + at);
  return 0;
}

// the base right-hand side in double-double at the state (yh, yl) into (kh, kl)
// (no host synchronisation: the domain, pivot and residual tests set bits of the status
// word, read once per step)
// the solve and right-hand side of a stage whose lane L is assembled and factored
// (G phi into gh, gl; the residual maxima in mx)
static int dd_rhs_tail(ww_ctx* c, const DdLane& L, const double* yh, const double* yl, double tau, double g,
                       double* kh, double* kl, double* gh, double* gl, unsigned long long* mx) {
  int rc;
  const int N = c->N;
  if ((rc = dd_solve_enqueue(c, L, yh + N, yl + N, 1, gh, gl, nullptr, nullptr, mx))) return rc;
  hipLaunchKernelGGL(k_dd_restest, dim3(1), dim3(64), 0, c->stream, mx, DD_TOL, c->status);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dd_base_rhs, dim3(1), dim3(WW_NT), dd_lds_bytes(N), c->stream, yh, yl, gh, gl, c->sdd_fh,
                     c->sdd_fl, c->dd_tw, N, g, tau, kh, kl);
  LAUNCHCHK();
  return 0;
}
static int dd_rhs(ww_ctx* c, const double* yh, const double* yl, double tau, double g, double* kh, double* kl) {
  int rc;
  if ((rc = dd_setup_enqueue(c, yh, yl, c->status))) return rc;
  return dd_rhs_tail(c, dd_lane(c), yh, yl, tau, g, kh, kl, c->sdd_Gh, c->sdd_Gl,
                     (unsigned long long*)(c->sdd_fo + 2));
}

// the lanes of the grouped sweeps (first use): per node, double-double A and Gm, the
// per-point quantities and the stage state; the second group's solve workspace; the
// ring's factor sets, the LU stream
static int ensure_sdd_lanes(ww_ctx* c) {
  int rc;
  if ((rc = ensure_sdc_groups(c))) return rc;
  if (c->sdd_lane) return 0;
  const size_t np = c->np_max, nm = c->n_max;
  const size_t per = 4 * np * np + 8 * nm + 4 * nm;   // A, Gm (hi, lo); 4 point planes (hi, lo); state (hi, lo)
  // the second group's solve workspace (its solves run on the LU stream) and G phi
  if (!c->sdd_w2 && (rc = dalloc(c, (void**)&c->sdd_w2, (size_t)DD_WORK * np * c->r_max * 8))) return rc;
  if (!c->sdd_part2 && (rc = dalloc(c, (void**)&c->sdd_part2, (size_t)2 * DDGV_KS * np * 8))) return rc;
  if (!c->sdd_G2 && (rc = dalloc(c, (void**)&c->sdd_G2, 2 * nm * 8))) return rc;
  return dalloc(c, (void**)&c->sdd_lane, SDC_NODES * per * 8);
}
static DdLane dd_sweep_lane(ww_ctx* c, int m, double** yh, double** yl) {
  const size_t np = c->np_max, nm = c->n_max, nn = np * np;
  double* b = c->sdd_lane + (size_t)m * (4 * nn + 12 * nm);
  *yh = b + 4 * nn + 8 * nm;
  *yl = *yh + 2 * nm;
  const bool second = m >= BLU_GMAX;   // the second group's workspace
  return DdLane{b + 4 * nn, b + 4 * nn + 4 * nm,   b,
                b + nn,     b + 2 * nn,            b + 3 * nn,
                dd_fac(c, pipe_set(c, m, false)), second ? c->sdd_w2 : c->dd_w, second ? c->sdd_part2 : c->dd_part};
}

// The nodes of one correction sweep (stages s0 .. s0 + SDC_NODES - 1) read only slopes of
// earlier sweeps: each node's stage state, per-point quantities and double-double
// assembly in its lane, the FP64 (or FP32) LUs in two groups of four, then each node's
// solve and right-hand side.  The second group's LU, solves and right-hand sides run on
// the LU stream with the second workspace, beside the first group's on the main stream.
// The kernels per lane are those of the stage-by-stage form: the same bits.
static int dd_sweep(ww_ctx* c, int s0, double tau, double g,
                    const std::function<int(int, double*, double*)>& combine) {
  static_assert(SDC_NODES == 2 * BLU_GMAX, "a sweep is factored in two groups");
  int rc;
  const int G = BLU_GMAX;
  const size_t n2 = (size_t)2 * c->N;
  DdLane L[SDC_NODES];
  double *yh[SDC_NODES], *yl[SDC_NODES];
  for (int m = 0; m < SDC_NODES; ++m) L[m] = dd_sweep_lane(c, m, &yh[m], &yl[m]);
  auto front = [&](int m) -> int {
    int e;
    if ((e = combine(s0 + m, yh[m], yl[m]))) return e;
    return dd_prep_assemble(c, L[m], yh[m], yl[m], c->status);
  };
  auto lu = [&](int m0) -> int {
    Fac F[BLU_GMAX];
    for (int q = 0; q < G; ++q) F[q] = L[m0 + q].F;
    return enqueue_lu_group(c, F, G);
  };
  const hipStream_t main = c->stream, ls = c->lus[0];
  unsigned long long* mx1 = (unsigned long long*)(c->sdd_fo + 2);
  unsigned long long* mx2 = (unsigned long long*)(c->sdd_fo + 4);
  auto tail = [&](int m, double* gh, double* gl, unsigned long long* mx) {
    return dd_rhs_tail(c, L[m], yh[m], yl[m], tau, g, c->sdd_Kh + (s0 + m) * n2, c->sdd_Kl + (s0 + m) * n2, gh, gl,
                       mx);
  };
  // the second group first: its LU, solves and right-hand sides on the LU stream with
  // the second workspace, beside the first group's on the main stream
  for (int m = G; m < SDC_NODES; ++m)
    if ((rc = front(m))) return rc;
  HIPCHK(hipEventRecord(c->sdc_ev, main));
  HIPCHK(hipStreamWaitEvent(ls, c->sdc_ev, 0));
  c->stream = ls;
  rc = lu(G);
  for (int m = G; m < SDC_NODES && !rc; ++m) rc = tail(m, c->sdd_G2, c->sdd_G2 + c->n_max, mx2);
  c->stream = main;
  if (rc) return rc;
  HIPCHK(hipEventRecord(c->sdc_ev, ls));
  for (int m = 0; m < G; ++m)
    if ((rc = front(m))) return rc;
  if ((rc = lu(0))) return rc;
  for (int m = 0; m < G; ++m)
    if ((rc = tail(m, c->sdd_Gh, c->sdd_Gl, mx1))) return rc;
  HIPCHK(hipStreamWaitEvent(main, c->sdc_ev, 0));   // the next stages read this sweep's slopes
  return 0;
}

extern "C" {

int shoot_eval(ww_ctx* c, const double* params, double T, int nsteps, double* r, double* J, double* drdT,
               double* f) {
  if (!c || !r || (!params && c->M > 0)) return fail(WW_EINVAL, "null argument");
  return shoot_eval_fb(c, params, T, nsteps, r, J, drdT, f, c->lag_off ? WW_FB_DIRECT : 0);
}

int shoot_eval_sdc(ww_ctx* c, const double* params, double T, int nsteps, double* r, double* J, double* drdT,
                   double* f) {
  if (!c || !r || (!params && c->M > 0)) return fail(WW_EINVAL, "null argument");
  if (int rj = pipe_join(c)) return rj;
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "shoot_eval_sdc before shoot_setup");
  if (nsteps < 1 || !std::isfinite(T)) return fail(WW_EINVAL, "nsteps >= 1 and finite T required");
  c->fb = 0;
  for (;;) {
    int st = 0, where = 0, rc;
    if ((rc = sdc_run(c, params, T, nsteps, r, J, drdT, f, &st, &where))) return rc;
    const unsigned nf = next_fallback(c, st);
    if (!nf) {
      if ((rc = status_error(c, st, where))) return rc;
      c->fb_last = c->fb;
      return 0;
    }
    c->fb |= nf;
  }
}

int shoot_eval_sdc_dd(ww_ctx* c, int N, double h, double tau, double g, const double* q0_hi, const double* q0_lo,
                      double T_hi, double T_lo, int nsteps, double* r_hi, double* r_lo, double* drdT_hi,
                      double* drdT_lo, double* f) {
  if (!c || !q0_hi || !r_hi || !r_lo || !f || (!drdT_hi != !drdT_lo)) return fail(WW_EINVAL, "null argument");
  if (N < 16 || (N & (N - 1)) || N > c->n_max || N > 1024)
    return fail(WW_EINVAL, "double-double march: N must be a power of two, 16 <= N <= min(n_max, 1024)");
  if (nsteps < 1 || !std::isfinite(T_hi) || !std::isfinite(T_lo) || !std::isfinite(g) || !(tau >= 0.0) ||
      !std::isfinite(tau) || !(h > 0.0))
    return fail(WW_EINVAL, "nsteps >= 1, finite T and g, finite tau >= 0 and h > 0 required");
  if (int rj = pipe_join(c)) return rj;
  int rc;
  if ((rc = set_grid(c, N, h))) return rc;
  if ((rc = ensure_dd(c))) return rc;
  if ((rc = dd_tables(c, N))) return rc;
  if ((rc = ensure_sdc_dd(c))) return rc;
  // the sweeps' nodes together (a one-stream context: stage by stage)
  const bool grouped = c->overlap;
  if (grouped && (rc = ensure_sdd_lanes(c))) return rc;
  c->dd_ready = false;    // the march replaces the double-double and FP64 factors
  c->dtn_ready = false;
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dd_mx_reset, dim3(1), dim3(64), 0, c->stream, (unsigned long long*)(c->sdd_fo + 2));
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dd_mx_reset, dim3(1), dim3(64), 0, c->stream, (unsigned long long*)(c->sdd_fo + 4));
  LAUNCHCHK();
  // the stage rows with this call's dt, the filter symbol, the initial state
  {
    const int rows = SDC_STAGES + 1;
    std::vector<int> jt((size_t)rows * SDC_MAXNZ, 0), cnt(rows, 0);
    std::vector<double> wh((size_t)rows * SDC_MAXNZ, 0.0), wl((size_t)rows * SDC_MAXNZ, 0.0);
    const dd dt = dd_div_d(dd_two_sum(T_hi, T_lo), 4.0 * nsteps);
    sdc_rows_dd(dt, cnt.data(), reinterpret_cast<int(*)[SDC_MAXNZ]>(jt.data()),
                reinterpret_cast<double(*)[SDC_MAXNZ]>(wh.data()), reinterpret_cast<double(*)[SDC_MAXNZ]>(wl.data()));
    HIPCHK(hipStreamSynchronize(c->stream));   // queued work of an earlier call may still read the rows
    HIPCHK(hipMemcpy(c->sdd_j, jt.data(), jt.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->sdd_wh, wh.data(), wh.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->sdd_wl, wl.data(), wl.size() * 8, hipMemcpyHostToDevice));
    for (int q = 0; q < rows; ++q) c->sdd_cnt[q] = cnt[q];
  }
  hipLaunchKernelGGL(k_dd_filter_tab, dim3((N / 2 + 256) / 256), dim3(256), 0, c->stream, N, c->sdd_fh, c->sdd_fl);
  LAUNCHCHK();
  const size_t n2 = (size_t)2 * N;
  HIPCHK(hipMemcpyAsync(c->sdd_yh, q0_hi, n2 * 8, hipMemcpyDeviceToDevice, c->stream));
  if (q0_lo)
    HIPCHK(hipMemcpyAsync(c->sdd_yl, q0_lo, n2 * 8, hipMemcpyDeviceToDevice, c->stream));
  else
    HIPCHK(hipMemsetAsync(c->sdd_yl, 0, n2 * 8, c->stream));
  const int blocks = (int)std::min<size_t>((n2 + 255) / 256, 4096);
  const std::function<int(int, double*, double*)> combine = [&](int row, double* oh, double* ol) -> int {
    hipLaunchKernelGGL(k_dd_sdc_combine, dim3(blocks), dim3(256), 0, c->stream, c->sdd_yh, c->sdd_yl, c->sdd_Kh,
                       c->sdd_Kl, n2, c->sdd_j + row * SDC_MAXNZ, c->sdd_wh + row * SDC_MAXNZ,
                       c->sdd_wl + row * SDC_MAXNZ, c->sdd_cnt[row], oh, ol, n2);
    LAUNCHCHK();
    return 0;
  };
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < SDC_STAGES; ++s) {
      if (grouped && s >= SDC_FIRST_SWEEP) {
        if ((rc = dd_sweep(c, s, tau, g, combine))) {
          const std::string msg = g_err;   // nothing may still run on the LU stream
          (void)hipStreamSynchronize(c->lus[0]);
          (void)hipStreamSynchronize(c->stream);
          g_err = msg;
          return rc;
        }
        s += SDC_NODES - 1;
        continue;
      }
      if ((rc = combine(s, c->sdd_Yh, c->sdd_Yl))) return rc;
      if ((rc = dd_rhs(c, c->sdd_Yh, c->sdd_Yl, tau, g, c->sdd_Kh + s * n2, c->sdd_Kl + s * n2))) return rc;
    }
    if ((rc = combine(SDC_STAGES, c->sdd_yh, c->sdd_yl))) return rc;
    hipLaunchKernelGGL(k_dd_filter_state, dim3(1), dim3(WW_NT), dd_lds_bytes(N), c->stream, c->sdd_yh, c->sdd_yl,
                       c->sdd_fh, c->sdd_fl, c->dd_tw, N);
    LAUNCHCHK();
    if ((rc = dd_march_status(c, n))) return rc;
  }
  // the right-hand side at the final state (dr/dT), then the outputs
  double* kfh = c->sdd_Kh + SDC_STAGES * n2;
  double* kfl = c->sdd_Kl + SDC_STAGES * n2;
  if (drdT_hi && (rc = dd_rhs(c, c->sdd_yh, c->sdd_yl, tau, g, kfh, kfl))) return rc;
  if ((rc = dd_march_status(c, -1))) return rc;
  hipLaunchKernelGGL(k_dd_outputs, dim3(1), dim3(WW_NT), 0, c->stream, c->sdd_yh, c->sdd_yl, kfh, kfl, N, r_hi, r_lo,
                     drdT_hi, drdT_lo, c->sdd_fo);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(f, c->sdd_fo, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return 0;
}

}   // extern "C"

// the segmented march (DOP853, or SDC15 steps) with its fallbacks
static int segments_eval(ww_ctx* c, const double* params, double T, int nseg, const ww_segment* segs, double* r,
                         double* J, double* drdT, double* f, bool sdc) {
  if (!c || !r || (!params && c->M > 0)) return fail(WW_EINVAL, "null argument");
  if (int rj = pipe_join(c)) return rj;
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "shoot_eval_segments before shoot_setup");
  if (!std::isfinite(T)) return fail(WW_EINVAL, "finite T required");
  int rc;
  if ((rc = seg_check(c, nseg, segs))) return rc;
  struct Mapped {   // the mapped-grid kernels for this call only
    ww_ctx* c;
    explicit Mapped(ww_ctx* cc) : c(cc) { c->mapped = true; }
    ~Mapped() { c->mapped = false; }
  } mapped_scope(c);
  c->fb = (c->lag_off && !sdc) ? WW_FB_DIRECT : 0;
  for (;;) {
    int st = 0, where = 0;
    if ((rc = seg_run(c, params, T, nseg, segs, r, J, drdT, f, &st, &where, sdc))) return rc;
    const unsigned nf = next_fallback(c, st);
    if ((st & 32) && !strict(c)) c->lag_off = true;
    if (!nf) {
      if ((rc = status_error(c, st, where))) return rc;
      c->fb_last = c->fb;
      return 0;
    }
    c->fb |= nf;
  }
}

extern "C" {

int shoot_eval_segments(ww_ctx* c, const double* params, double T, int nseg, const ww_segment* segs, double* r,
                        double* J, double* drdT, double* f) {
  return segments_eval(c, params, T, nseg, segs, r, J, drdT, f, false);
}

int shoot_eval_segments_sdc(ww_ctx* c, const double* params, double T, int nseg, const ww_segment* segs, double* r,
                            double* J, double* drdT, double* f) {
  return segments_eval(c, params, T, nseg, segs, r, J, drdT, f, true);
}

int shoot_eval_batch(int n_inst, ww_ctx* const* ctx, const double* const* params, const double* T,
                     const int* nsteps, double* const* r, double* const* J, double* const* drdT, double* f) {
  if (n_inst < 1 || !ctx || !params || !T || !nsteps || !r) return fail(WW_EINVAL, "null argument");
  for (int i = 0; i < n_inst; ++i) {
    if (!ctx[i] || !r[i]) return fail(WW_EINVAL, "null context or output");
    for (int k = 0; k < i; ++k)
      if (ctx[k] == ctx[i]) return fail(WW_EINVAL, "the contexts of a batch must be distinct");
  }
  int rc;
  int maxsteps = 0;
  // An error part-way leaves work of the instances enqueued so far (writes into the
  // caller's r, J, drdT and, for f, a host copy into the caller's array): wait for all
  // of it before returning, so that no write lands after the caller has freed them.
  auto settle = [&](int code) {
    const std::string msg = g_err;
    for (int i = 0; i < n_inst; ++i) {
      (void)pipe_join(ctx[i]);
      (void)hipStreamSynchronize(ctx[i]->stream);
      int st = 0;
      (void)read_status(ctx[i], &st);
    }
    g_err = msg;
    return code;
  };
  // one instance: the two-stream step graph of shoot_eval; several: one-stream graphs,
  // which the hardware overlaps across instances (two-stream graphs of several
  // instances run one after the other)
  const bool two = n_inst == 1 && ctx[0]->overlap;
  for (int i = 0; i < n_inst; ++i) {
    const bool cols = J && J[i] && ctx[i]->M > 0;
    ctx[i]->fb = ctx[i]->lag_off ? WW_FB_DIRECT : 0;
    if ((rc = shoot_prepare(ctx[i], params[i], T[i], nsteps[i], cols, two))) return settle(rc);
    maxsteps = std::max(maxsteps, nsteps[i]);
  }
  // interleave the instances step by step: each context replays its own step graph on
  // its own stream, so the hardware queues overlap the instances
  for (int n = 0; n < maxsteps; ++n)
    for (int i = 0; i < n_inst; ++i)
      if (n < nsteps[i])
        if ((rc = shoot_one_step(ctx[i], J && J[i] && ctx[i]->M > 0, two))) return settle(rc);
  for (int i = 0; i < n_inst; ++i) {
    const bool cols = J && J[i] && ctx[i]->M > 0;
    if ((rc = shoot_finish(ctx[i], cols, r[i], J ? J[i] : nullptr, drdT ? drdT[i] : nullptr, f ? &f[i] : nullptr)))
      return settle(rc);
  }
  int first_err = 0;
  for (int i = 0; i < n_inst; ++i) {
    ww_ctx* c = ctx[i];
    int st = 0, where = 0, e;
    if ((e = read_status(c, &st, &where)) == 0) {
      if ((st & 32) && !strict(c)) c->lag_off = true;
      const unsigned nf = next_fallback(c, st);
      if (nf)   // this instance alone, in its fallback mode
        e = shoot_eval_fb(c, params[i], T[i], nsteps[i], r[i], J ? J[i] : nullptr, drdT ? drdT[i] : nullptr,
                          f ? &f[i] : nullptr, nf);
      else if ((e = status_error(c, st, where)) == 0)
        c->fb_last = c->fb;
    }
    if (e && !first_err) first_err = e;
  }
  return first_err;
}

}  // extern "C"

// one adjoint evaluation in the current fallback mode; *stout receives the status bits
static int adjoint_run(ww_ctx* c, const double* params, double T, int nsteps, int ckpt_every, double* grad,
                       double* dfdT, double* f, int* stout, int* where) {
  int rc;
  if ((rc = set_grid(c, c->shootN, c->shootH))) return rc;
  c->dtn_ready = false;
  c->gm_active = false;   // the transposed solves need the factors
  const int N = c->N, Np = c->Np, M = c->M, nst = c->nst;
  const int C = std::min(ckpt_every, nsteps);
  const int nseg = (nsteps + C - 1) / C;
  // buffers: checkpoints, per-stage factor sets of one segment, adjoint work vectors
  const size_t n2 = (size_t)2 * N;
  const size_t slot = (size_t)3 * Np * Np + (size_t)3 * N;   // X, Z, Gm, saux
  const size_t nslot = (size_t)C * nst;
  if (c->ckpt_cap < (size_t)(nseg + 1) * n2) {
    if (c->ckpt) HIPCHK(hipFree(c->ckpt));
    c->ckpt = nullptr;
    c->ckpt_cap = 0;
    HIPCHK(hipMalloc(&c->ckpt, (size_t)(nseg + 1) * n2 * 8));
    c->ckpt_cap = (size_t)(nseg + 1) * n2;
  }
  if (c->seg_cap < nslot * slot) {
    if (c->seg) HIPCHK(hipFree(c->seg));
    c->seg = nullptr;
    c->seg_cap = 0;
    HIPCHK(hipMalloc(&c->seg, nslot * slot * 8));
    c->seg_cap = nslot * slot;
  }
  if (pivoted(c)) {
    if ((rc = ensure_pivot_buffers(c))) return rc;
    if (c->seg_perm_cap < nslot * c->np_max) {
      if (c->seg_perm) HIPCHK(hipFree(c->seg_perm));
      c->seg_perm = nullptr;
      c->seg_perm_cap = 0;
      HIPCHK(hipMalloc(&c->seg_perm, nslot * c->np_max * sizeof(int)));
      c->seg_perm_cap = nslot * c->np_max;
    }
  }
  if (!c->adj) HIPCHK(hipMalloc(&c->adj, (size_t)(20 * 2 * c->n_max + 9 * c->np_max) * 8));
  double* lam = c->adj;
  double* mu = lam + 2 * c->n_max;
  double* ups = mu + 2 * c->n_max;                 // 16 x 2N
  const size_t ustride = 2 * (size_t)c->n_max;
  double* gt = ups + 16 * ustride;
  double* hd = gt + c->np_max;
  double* e1 = hd + c->np_max;
  double* qv = e1 + c->np_max;
  double* g2 = qv + c->np_max;
  double* zeta = g2 + c->np_max;
  double* y1 = zeta + c->np_max;
  double* y2 = y1 + c->np_max;
  double* rv = y2 + c->np_max;       // r (N)
  double* dv = rv + c->n_max;        // drdT (N)
  double* y2p = dv + c->n_max;       // P^T y2 (Np), pivoted factors
  auto slot_fac = [&](size_t k) {
    double* b = c->seg + k * slot;
    Fac F = fac_set(c, 0, false);
    F.Gm = b + 2 * (size_t)Np * Np;
    F.X = b;
    F.Z = b + (size_t)Np * Np;
    F.use32 = false;
    F.perm = pivoted(c) ? c->seg_perm + k * c->np_max : nullptr;
    return F;
  };
  auto slot_aux = [&](size_t k) { return c->seg + k * slot + (size_t)3 * Np * Np; };
  // step coefficients
  double coef[COEF_SIZE];
  std::memset(coef, 0, sizeof(coef));
  const double dt = T / (4.0 * nsteps);
  for (int s = 0; s < nst; ++s) {
    for (int j = 0; j < s; ++j) coef[s * 16 + j] = c->ta[s * 16 + j] * dt;
    coef[COEF_B + s] = c->tb[s] * dt;
  }
  coef[COEF_DT] = dt;
  HIPCHK(hipMemcpyAsync(c->coef, coef, sizeof(coef), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
  LAUNCHCHK();
  {
    const size_t tot = (size_t)2 * N * (M + 1);
    const int blocks = (int)std::min<size_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, c->stream, c->y, c->basis, c->qfix, params, N, M);
    LAUNCHCHK();
  }
  // 1. forward base march with checkpoints (FP64 factors)
  Fac F0 = fac_set(c, 0, false);
  F0.use32 = false;
  auto base_step = [&](const Fac* per_stage_base, size_t slot0) -> int {
    for (int s = 0; s < nst; ++s) {
      const Fac F = per_stage_base ? slot_fac(slot0 + s) : F0;
      int r2 = enqueue_base_chain(c, c->y, s, c->K + (size_t)s * kstride(c), F);
      if (r2) return r2;
      if (per_stage_base) {
        hipLaunchKernelGGL(k_save_aux, dim3((N + 255) / 256), dim3(256), 0, c->stream, F.aux, c->n_max, N,
                           slot_aux(slot0 + s));
        LAUNCHCHK();
      }
    }
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 3), c->stream, c->y, c->K, kstride(c), nst,
                       c->coef, c->tw, c->sig, N, 0, c->status);
    LAUNCHCHK();
    return 0;
  };
  for (int n = 0; n < nsteps; ++n) {
    if (n % C == 0) HIPCHK(hipMemcpyAsync(c->ckpt + (size_t)(n / C) * n2, c->y, n2 * 8, hipMemcpyDeviceToDevice, c->stream));
    if ((rc = base_step(nullptr, 0))) return rc;
  }
  hipLaunchKernelGGL(k_check_finite, dim3(64), dim3(256), 0, c->stream, c->y, n2, c->status);
  LAUNCHCHK();
  // outputs r, drdT, f at T/4
  if ((rc = enqueue_base_chain(c, c->y, 0, c->Kx, F0))) return rc;
  hipLaunchKernelGGL(k_outputs, dim3((N + 255) / 256), dim3(256), 0, c->stream, c->y, c->Kx, rv, nullptr, dv, N, 0);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(WW_NT), 0, c->stream, rv, N, c->fdev, (const double*)dv);
  LAUNCHCHK();
  // 2. adjoint seed (0, w r) and the reverse sweep, segment by segment
  hipLaunchKernelGGL(k_adj_seed, dim3((2 * N + 255) / 256), dim3(256), 0, c->stream, rv, N, lam);
  LAUNCHCHK();
  const double g = c->g, tau = c->tau;
  bool first = true;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int n0 = sg * C, n1 = std::min(n0 + C, nsteps);
    HIPCHK(hipMemcpyAsync(c->y, c->ckpt + (size_t)sg * n2, n2 * 8, hipMemcpyDeviceToDevice, c->stream));
    for (int n = n0; n < n1; ++n)
      if ((rc = base_step(&F0, (size_t)(n - n0) * nst))) return rc;
    for (int n = n1 - 1; n >= n0; --n) {
      // lambda_{n+1} (seed, or mu + sum ups of the step after) and mu = S_F lambda_{n+1}
      hipLaunchKernelGGL(k_adj_step, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 3), c->stream, lam, mu, ups, ustride, nst,
                         first ? 1 : 0, c->tw, c->sig, N);
      LAUNCHCHK();
      first = false;
      for (int s = nst - 1; s >= 0; --s) {
        const size_t k = (size_t)(n - n0) * nst + s;
        const Fac F = slot_fac(k);
        const double* sa = slot_aux(k);
        hipLaunchKernelGGL(k_adj_pre, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 4), c->stream, mu, ups, ustride, c->coef,
                           s, nst, sa, c->tw, c->sig, N, Np, g, tau, gt, hd, e1, qv);
        LAUNCHCHK();
        const int gblk = (Np * 64 + WW_NT - 1) / WW_NT;
        hipLaunchKernelGGL(k_gemv_t, dim3(gblk), dim3(WW_NT), 0, c->stream, F.Gm, Np, 0, gt, nullptr, g2);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_adj_mid, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 3), c->stream, g2, hd, c->tw, N, Np, zeta);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_gemv_t, dim3(gblk), dim3(WW_NT), 0, c->stream, F.Z, Np, 2, zeta, nullptr, y1);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_gemv_t, dim3(gblk), dim3(WW_NT), 0, c->stream, F.X, Np, 1, y1, y1, y2);
        LAUNCHCHK();
        const double* yt = y2;   // A^{-T} zeta; with P A = Lt Ut it is P^T (Lt Ut)^{-T} zeta
        if (F.perm) {
          hipLaunchKernelGGL(k_permute_rows, dim3((Np + 255) / 256), dim3(256), 0, c->stream, y2, y2p, F.perm, Np, 1,
                             1);
          LAUNCHCHK();
          yt = y2p;
        }
        hipLaunchKernelGGL(k_adj_post, dim3((N + 255) / 256), dim3(256), 0, c->stream, yt, qv, e1, sa, N,
                           ups + (size_t)s * ustride);
        LAUNCHCHK();
      }
    }
  }
  // lambda_0 = mu + sum ups, gradient basis^T lambda_0
  hipLaunchKernelGGL(k_adj_step, dim3(1), dim3(WW_NT), fft_lds_bytes(N, 3), c->stream, lam, mu, ups, ustride, nst, 0,
                     c->tw, c->sig, N);
  LAUNCHCHK();
  if (M > 0) {
    hipLaunchKernelGGL(k_adj_grad, dim3((M * 64 + WW_NT - 1) / WW_NT), dim3(WW_NT), 0, c->stream, c->basis, lam, N, M,
                       grad);
    LAUNCHCHK();
  }
  double fh[2] = {0.0, 0.0};   // f and df/dT = r . dr/dT, reduced on the device
  HIPCHK(hipMemcpyAsync(fh, c->fdev, sizeof(fh), hipMemcpyDeviceToHost, c->stream));
  int st = 0;
  if ((rc = read_status(c, &st, where))) return rc;
  if (f) *f = fh[0];
  if (dfdT) *dfdT = fh[1];
  *stout = st;
  return 0;
}

extern "C" {

int shoot_adjoint(ww_ctx* c, const double* params, double T, int nsteps, int ckpt_every, double* grad,
                  double* dfdT, double* f) {
  if (!c || !grad || (!params && c->M > 0)) return fail(WW_EINVAL, "null argument");
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "shoot_adjoint before shoot_setup");
  if (c->nst < 1) return fail(WW_EINVAL, "no tableau set");
  if (nsteps < 1 || !std::isfinite(T) || ckpt_every < 1) return fail(WW_EINVAL, "nsteps, ckpt_every >= 1 required");
  c->fb = 0;
  for (;;) {
    int st = 0, where = 0, rc;
    if ((rc = adjoint_run(c, params, T, nsteps, ckpt_every, grad, dfdT, f, &st, &where))) return rc;
    const unsigned nf = next_fallback(c, st & ~4);   // FP64 factors throughout
    if (!nf) {
      if ((rc = status_error(c, st, where))) return rc;
      c->fb_last = c->fb;
      return 0;
    }
    c->fb |= nf;
  }
}

int ww_fallbacks(ww_ctx* c, unsigned* bits) {
  if (!c || !bits) return fail(WW_EINVAL, "null argument");
  *bits = c->fb_last;
  return 0;
}

}  // extern "C"

// ----- thin SVD and the Levenberg-Marquardt driver (App. C) -----
static const double SVD_TOL = 1e-15;     // pair orthogonality |w_a.w_b| <= tol ||w_a|| ||w_b||
static const int SVD_MAX_SWEEPS = 60;

static int ensure_lm(ww_ctx* c) {
  if (c->lmW) return 0;
  int rc;
  const size_t nm = c->n_max, R = c->r_max;
  if ((rc = dalloc(c, (void**)&c->lmW, nm * R * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmr, nm * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmrn, nm * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmp, R * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmV, R * R * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmsig, R * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmdot, R * 8))) return rc;
  if ((rc = dalloc(c, (void**)&c->lmflag, 64))) return rc;
  return dalloc(c, (void**)&c->lmperm, R * sizeof(int));
}

// One-sided Jacobi on W (N x n, device) with V := rotations (device); sweeps until no
// pair rotates.  Non-finite input: WW_ENONFINITE.
static int jacobi_svd(ww_ctx* c, double* W, int N, int n, double* V) {
  {
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, c->stream, c->status);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_check_finite, dim3(64), dim3(256), 0, c->stream, W, (size_t)N * n, c->status);
    LAUNCHCHK();
    int st = 0;
    int rc;
    if ((rc = read_status(c, &st))) return rc;
    if (st & 2) return fail(WW_ENONFINITE, "thin SVD: non-finite matrix entry");
  }
  const int n2 = (n + 1) & ~1;
  hipLaunchKernelGGL(k_svd_eye, dim3(std::max(1, std::min(1024, (n * n + 255) / 256))), dim3(256), 0, c->stream, V, n);
  LAUNCHCHK();
  if (n < 2) return 0;
  for (int sw = 0; sw < SVD_MAX_SWEEPS; ++sw) {
    HIPCHK(hipMemsetAsync(c->lmflag, 0, sizeof(int), c->stream));
    for (int rd = 0; rd + 1 < n2; ++rd) {
      hipLaunchKernelGGL(k_jacobi_round, dim3(n2 / 2), dim3(SVD_NT), 0, c->stream, W, N, V, n, n2, rd, SVD_TOL,
                         c->lmflag);
      LAUNCHCHK();
    }
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, c->lmflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (!h) return 0;
  }
  return fail(WW_ENOCONV, "thin SVD: Jacobi sweeps did not converge");
}

// Levenberg-Marquardt state on the host: the SVD of the current Jacobian (sigma, V) and
// the residual r on the device (c->lmr).
struct LmSvd {
  int n = 0;
  std::vector<double> s, V;   // singular values (small ones zeroed), V column-major
};

// Jacobian at cv: r -> c->lmr, J = [dr/dT | dr/dparams] -> c->lmW, then its SVD
static int lm_jacobian(ww_ctx* c, const std::vector<double>& cv, int nsteps, double* f, LmSvd& sv) {
  const int N = c->N, M = c->M, n = M + 1;
  int rc;
  if (M > 0) HIPCHK(hipMemcpyAsync(c->lmp, cv.data() + 1, (size_t)M * 8, hipMemcpyHostToDevice, c->stream));
  if ((rc = shoot_eval(c, c->lmp, cv[0], nsteps, c->lmr, M > 0 ? c->lmW + N : nullptr, c->lmW, f))) return rc;
  if ((rc = jacobi_svd(c, c->lmW, N, n, c->lmV))) return rc;
  hipLaunchKernelGGL(k_svd_cols, dim3(n), dim3(SVD_NT), 0, c->stream, c->lmW, N, nullptr, c->lmsig, nullptr);
  LAUNCHCHK();
  sv.n = n;
  sv.s.assign(n, 0.0);
  sv.V.assign((size_t)n * n, 0.0);
  HIPCHK(hipMemcpyAsync(sv.s.data(), c->lmsig, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(sv.V.data(), c->lmV, (size_t)n * n * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double smax = *std::max_element(sv.s.begin(), sv.s.end());
  const double cut = n * 2.220446049250313e-16 * smax;   // small singular values count as zero
  for (double& x : sv.s)
    if (x < cut) x = 0.0;
  return 0;
}

// r~ = U^T r = (W^T r) / sigma for the residual on the device at rdev
static int lm_rtilde(ww_ctx* c, const double* rdev, const LmSvd& sv, std::vector<double>& rt) {
  const int n = sv.n;
  hipLaunchKernelGGL(k_svd_cols, dim3(n), dim3(SVD_NT), 0, c->stream, c->lmW, c->N, rdev, nullptr, c->lmdot);
  LAUNCHCHK();
  rt.assign(n, 0.0);
  HIPCHK(hipMemcpyAsync(rt.data(), c->lmdot, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) rt[k] = sv.s[k] > 0.0 ? rt[k] / sv.s[k] : 0.0;
  return 0;
}

// eq. (trust:tilde): p~ = -sigma r~ / (sigma^2 + lambda), lambda by Newton's method on
// tau(lambda) = 1/||p~|| - 1/Delta from lambda = 0 (the Newton step of tau divides by
// p~^T (S^2 + lambda)^{-1} p~)
static void trust_subproblem(const std::vector<double>& s, const std::vector<double>& rt, double delta,
                             std::vector<double>& p) {
  const int n = (int)s.size();
  auto step = [&](double lam) {
    for (int k = 0; k < n; ++k) p[k] = s[k] > 0.0 ? -s[k] * rt[k] / (s[k] * s[k] + lam) : 0.0;
  };
  auto norm = [&]() {
    double a = 0.0;
    for (double x : p) a += x * x;
    return std::sqrt(a);
  };
  p.assign(n, 0.0);
  step(0.0);
  if (norm() <= delta) return;
  double lam = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double pn = norm();
    if (std::fabs(pn - delta) / delta <= 1e-12) break;
    double q = 0.0;
    for (int k = 0; k < n; ++k)
      if (s[k] > 0.0) q += p[k] * p[k] / (s[k] * s[k] + lam);
    lam += (pn * pn / q) * ((pn - delta) / delta);
    step(lam);
  }
}

extern "C" {

int ww_thin_svd(ww_ctx* c, const double* A, int N, int n, double* sigma, double* V, double* U) {
  if (!c || !A || !sigma) return fail(WW_EINVAL, "null argument");
  if (N < 1 || n < 1 || n > N || N > c->n_max || n > c->r_max)
    return fail(WW_EINVAL, "thin SVD: need 1 <= n <= N, N <= n_max, n <= r_max");
  int rc;
  if ((rc = ensure_lm(c))) return rc;
  HIPCHK(hipMemcpyAsync(c->lmW, A, (size_t)N * n * 8, hipMemcpyDeviceToDevice, c->stream));
  if ((rc = jacobi_svd(c, c->lmW, N, n, c->lmV))) return rc;
  hipLaunchKernelGGL(k_svd_cols, dim3(n), dim3(SVD_NT), 0, c->stream, c->lmW, N, nullptr, c->lmsig, nullptr);
  LAUNCHCHK();
  std::vector<double> s(n), v((size_t)n * n);
  HIPCHK(hipMemcpyAsync(s.data(), c->lmsig, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(v.data(), c->lmV, (size_t)n * n * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return s[a] > s[b]; });
  for (int k = 0; k < n; ++k) sigma[k] = s[perm[k]];
  if (V)
    for (int k = 0; k < n; ++k) std::memcpy(V + (size_t)k * n, v.data() + (size_t)perm[k] * n, (size_t)n * 8);
  if (U) {
    HIPCHK(hipMemcpyAsync(c->lmperm, perm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, c->stream));
    const size_t tot = (size_t)N * n;
    hipLaunchKernelGGL(k_svd_u, dim3((int)std::min<size_t>((tot + 255) / 256, 4096)), dim3(256), 0, c->stream, c->lmW,
                       N, c->lmsig, c->lmperm, n, U);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->stream));   // perm is a host temporary of this call
  }
  return 0;
}

int ww_levmar(ww_ctx* c, double* cvec, int nsteps, const ww_lm_opts* opts, ww_lm_report* rep) {
  if (!c || !cvec) return fail(WW_EINVAL, "null argument");
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "ww_levmar before shoot_setup");
  if (nsteps < 1) return fail(WW_EINVAL, "nsteps >= 1 required");
  ww_lm_opts o;
  ww_lm_default_opts(&o);
  if (opts) o = *opts;
  if (!(o.delta0 > 0.0) || o.max_steps_J < 1 || o.max_evals < 1) return fail(WW_EINVAL, "bad options");
  int rc;
  if ((rc = ensure_lm(c))) return rc;
  const int M = c->M, n = M + 1;
  const double RHO0 = 0.25, RHO1 = 0.85, A0 = 3.0 / 8.0, A1 = 1.875, A2 = 0.2;
  std::vector<double> cv(cvec, cvec + n), cn(n), rt, pt, p(n), g(n);
  LmSvd sv;
  double f = 0.0, fn = 0.0;
  if ((rc = lm_jacobian(c, cv, nsteps, &f, sv))) return rc;
  int evals_r = 0, evals_J = 1, steps_J = 0, nh = 0, reason = 0;
  double delta = o.delta0, dfr = -1.0;   // dfr < 0: delta_first_rejected undefined
  bool roundoff = false, acc_since_J = false;
  for (;;) {
    if (f == 0.0) {
      reason = WW_LM_F_ZERO;
      break;
    }
    if (evals_r + evals_J >= o.max_evals) {
      reason = WW_LM_MAX_EVALS;
      break;
    }
    if ((rc = lm_rtilde(c, c->lmr, sv, rt))) return rc;
    trust_subproblem(sv.s, rt, delta, pt);
    double df = 0.0, gn = 0.0, pn = 0.0;
    for (int k = 0; k < n; ++k) df += sv.s[k] * rt[k] * pt[k] + 0.5 * (sv.s[k] * pt[k]) * (sv.s[k] * pt[k]);
    for (int i = 0; i < n; ++i) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < n; ++k) {
        a += sv.V[(size_t)k * n + i] * pt[k];
        b += sv.V[(size_t)k * n + i] * sv.s[k] * rt[k];
      }
      p[i] = a;
      g[i] = b;
      pn += a * a;
      gn += b * b;
    }
    pn = std::sqrt(pn);
    gn = std::sqrt(gn);
    if (f < o.f_tol || delta < o.g_tol) roundoff = true;
    if (steps_J == 0 && (gn < o.g_tol || std::fabs(df) / f < o.df_tol)) roundoff = true;
    bool same = true;
    for (int i = 0; i < n; ++i) {
      cn[i] = cv[i] + p[i];
      if (cn[i] != cv[i]) same = false;
    }
    if (same) {
      reason = WW_LM_C_UNCHANGED;
      break;
    }
    if (M > 0) HIPCHK(hipMemcpyAsync(c->lmp, cn.data() + 1, (size_t)M * 8, hipMemcpyHostToDevice, c->stream));
    if ((rc = shoot_eval(c, c->lmp, cn[0], nsteps, c->lmrn, nullptr, nullptr, &fn))) return rc;
    ++evals_r;
    const double rho = df != 0.0 ? (fn - f) / df : -1.0;
    const bool accepted = rho > 0.0;
    if (rep && rep->history && nh < rep->hist_cap) {
      double* h = rep->history + (size_t)nh * (n + 2);
      for (int i = 0; i < n; ++i) h[i] = cn[i];
      h[n] = fn;
      h[n + 1] = accepted ? 1.0 : 0.0;
    }
    ++nh;
    if (accepted) acc_since_J = true;
    if (rho < RHO0) {
      if (dfr < 0.0 && acc_since_J) dfr = delta;
      delta = A0 * pn;
    } else if (rho > RHO1 && pn > 0.9 * delta) {
      delta = A1 * delta;
    }
    if (accepted) {
      cv = cn;
      f = fn;
      std::swap(c->lmr, c->lmrn);
      ++steps_J;
    }
    if (roundoff && (!accepted || steps_J >= o.max_steps_J)) {
      reason = accepted ? WW_LM_ROUNDOFF_MAX_STEPS_J : WW_LM_ROUNDOFF_REJECTED;
      break;
    }
    const double trigger = dfr >= 0.0 ? A2 * dfr : -INFINITY;
    if (!roundoff && (steps_J >= o.max_steps_J || (steps_J > 0 && delta < trigger) ||
                      (steps_J > 0 && f > 0.0 && std::fabs(df) / f < o.df_tol))) {
      if (dfr >= 0.0) delta = dfr / A1;
      if ((rc = lm_jacobian(c, cv, nsteps, &f, sv))) return rc;
      ++evals_J;
      steps_J = 0;
      dfr = -1.0;
      acc_since_J = false;
    }
  }
  for (int i = 0; i < n; ++i) cvec[i] = cv[i];
  if (rep) {
    rep->f = f;
    rep->delta = delta;
    rep->evals_r = evals_r;
    rep->evals_J = evals_J;
    rep->reason = reason;
    rep->n_hist = nh;
  }
  return 0;
}

}  // extern "C"

// ----- BFGS with a strong-Wolfe line search (the adjoint minimiser of Sec. 3.2) -----
// f and its gradient g = (df/dT, grad_params f) from one shoot_adjoint call
static int bfgs_fg(ww_ctx* c, const std::vector<double>& cv, int nsteps, int ckpt, double* f, std::vector<double>& g) {
  const int M = c->M;
  if (M > 0) HIPCHK(hipMemcpyAsync(c->lmp, cv.data() + 1, (size_t)M * 8, hipMemcpyHostToDevice, c->stream));
  double dfdT = 0.0;
  int rc;
  if ((rc = shoot_adjoint(c, c->lmp, cv[0], nsteps, ckpt, c->lmdot, &dfdT, f))) return rc;
  g.assign(M + 1, 0.0);
  g[0] = dfdT;
  if (M > 0) {
    HIPCHK(hipMemcpyAsync(g.data() + 1, c->lmdot, (size_t)M * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return 0;
}

static double dotv(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// Strong Wolfe conditions (c1 = 1e-4, c2 = 0.9): bracketing by doubling, zoom by
// bisection.  On return: *a the step, *fa, ga the values there, *ok whether the
// conditions hold (else the best point met).
static int bfgs_line_search(ww_ctx* c, int nsteps, int ckpt, const std::vector<double>& cv, double f0,
                            const std::vector<double>& g0, const std::vector<double>& p, double a1, double* a_out,
                            double* f_out, std::vector<double>& g_out, int* evals, bool* ok) {
  const double C1 = 1e-4, C2 = 0.9;
  const int n = (int)cv.size();
  const double d0 = dotv(g0, p);
  std::vector<double> x(n), g;
  double f = 0.0;
  int rc;
  auto eval = [&](double a) -> int {
    for (int i = 0; i < n; ++i) x[i] = cv[i] + a * p[i];
    ++*evals;
    return bfgs_fg(c, x, nsteps, ckpt, &f, g);
  };
  double best_a = 0.0, best_f = f0;
  std::vector<double> best_g = g0;
  auto keep = [&](double a) {
    if (f < best_f) {
      best_a = a;
      best_f = f;
      best_g = g;
    }
  };
  auto done = [&](double a, bool good) {
    *a_out = a;
    *f_out = good ? f : best_f;
    g_out = good ? g : best_g;
    if (!good) *a_out = best_a;
    *ok = good;
    return 0;
  };
  double a_prev = 0.0, f_prev = f0, a = a1, lo = 0.0, hi = 0.0, flo = 0.0;
  bool bracket = false;
  for (int i = 0; i < 20; ++i) {
    if ((rc = eval(a))) return rc;
    keep(a);
    if (f > f0 + C1 * a * d0 || (i > 0 && f >= f_prev)) {
      lo = a_prev;
      flo = f_prev;
      hi = a;
      bracket = true;
      break;
    }
    const double d = dotv(g, p);
    if (std::fabs(d) <= -C2 * d0) return done(a, true);
    if (d >= 0.0) {
      lo = a;
      flo = f;
      hi = a_prev;
      bracket = true;
      break;
    }
    a_prev = a;
    f_prev = f;
    a = 2.0 * a;
  }
  if (!bracket) return done(0.0, false);
  for (int j = 0; j < 30; ++j) {
    a = 0.5 * (lo + hi);
    if ((rc = eval(a))) return rc;
    keep(a);
    if (f > f0 + C1 * a * d0 || f >= flo) {
      hi = a;
    } else {
      const double d = dotv(g, p);
      if (std::fabs(d) <= -C2 * d0) return done(a, true);
      if (d * (hi - lo) >= 0.0) hi = lo;
      lo = a;
      flo = f;
    }
  }
  return done(0.0, false);
}

extern "C" {

int ww_bfgs_default_opts(ww_bfgs_opts* o) {
  if (!o) return fail(WW_EINVAL, "null argument");
  o->f_tol = 1e-26;
  o->g_tol = 1e-13;
  o->delta0 = 0.1;
  o->max_iter = 200;
  o->ckpt_every = 16;
  return 0;
}

int ww_bfgs(ww_ctx* c, double* cvec, int nsteps, const ww_bfgs_opts* opts, ww_bfgs_report* rep) {
  if (!c || !cvec) return fail(WW_EINVAL, "null argument");
  if (!c->shoot_ready) return fail(WW_ENOSETUP, "ww_bfgs before shoot_setup");
  if (nsteps < 1) return fail(WW_EINVAL, "nsteps >= 1 required");
  ww_bfgs_opts o;
  ww_bfgs_default_opts(&o);
  if (opts) o = *opts;
  if (!(o.delta0 > 0.0) || o.max_iter < 1 || o.ckpt_every < 1) return fail(WW_EINVAL, "bad options");
  int rc;
  if ((rc = ensure_lm(c))) return rc;
  const int n = c->M + 1;
  std::vector<double> cv(cvec, cvec + n), g, gn, p(n), cn(n), s(n), y(n), Hy(n);
  std::vector<double> H((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) H[(size_t)i * n + i] = 1.0;
  double f = 0.0, fn = 0.0;
  if ((rc = bfgs_fg(c, cv, nsteps, o.ckpt_every, &f, g))) return rc;
  int evals = 1, iters = 0, nh = 0, reason = WW_BFGS_MAX_ITER;
  bool first = true;
  for (iters = 0; iters < o.max_iter; ++iters) {
    if (f < o.f_tol) {
      reason = WW_BFGS_F_TOL;
      break;
    }
    if (std::sqrt(dotv(g, g)) < o.g_tol) {
      reason = WW_BFGS_G_TOL;
      break;
    }
    for (int i = 0; i < n; ++i) {
      double a = 0.0;
      for (int j = 0; j < n; ++j) a += H[(size_t)i * n + j] * g[j];
      p[i] = -a;
    }
    if (dotv(g, p) >= 0.0) {   // not a descent direction: steepest descent
      std::fill(H.begin(), H.end(), 0.0);
      for (int i = 0; i < n; ++i) {
        H[(size_t)i * n + i] = 1.0;
        p[i] = -g[i];
      }
    }
    const double a1 = first ? std::min(1.0, o.delta0 / std::sqrt(dotv(p, p))) : 1.0;
    double a = 0.0;
    bool ok = false;
    if ((rc = bfgs_line_search(c, nsteps, o.ckpt_every, cv, f, g, p, a1, &a, &fn, gn, &evals, &ok))) return rc;
    if (!ok && !(fn < f)) {
      reason = WW_BFGS_LINE_SEARCH;
      break;
    }
    bool same = true;
    for (int i = 0; i < n; ++i) {
      cn[i] = cv[i] + a * p[i];
      if (cn[i] != cv[i]) same = false;
      s[i] = cn[i] - cv[i];
      y[i] = gn[i] - g[i];
    }
    if (same) {
      reason = WW_BFGS_C_UNCHANGED;
      break;
    }
    const double sy = dotv(s, y);
    if (sy > 0.0) {
      if (first) {
        const double sc = sy / dotv(y, y);
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) H[(size_t)i * n + j] = i == j ? sc : 0.0;
      }
      // H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, expanded
      const double rho = 1.0 / sy;
      for (int i = 0; i < n; ++i) {
        double a2 = 0.0;
        for (int j = 0; j < n; ++j) a2 += H[(size_t)i * n + j] * y[j];
        Hy[i] = a2;
      }
      const double yHy = dotv(y, Hy);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          H[(size_t)i * n + j] += -rho * (s[i] * Hy[j] + Hy[i] * s[j]) + (rho * rho * yHy + rho) * s[i] * s[j];
      first = false;
    }
    cv = cn;
    f = fn;
    g = gn;
    if (rep && rep->history && nh < rep->hist_cap) {
      double* h = rep->history + (size_t)nh * (n + 1);
      for (int i = 0; i < n; ++i) h[i] = cv[i];
      h[n] = f;
    }
    ++nh;
  }
  for (int i = 0; i < n; ++i) cvec[i] = cv[i];
  if (rep) {
    rep->f = f;
    rep->gnorm = std::sqrt(dotv(g, g));
    rep->iters = iters;
    rep->evals = evals;
    rep->reason = reason;
    rep->n_hist = nh;
  }
  return 0;
}

int ww_lm_default_opts(ww_lm_opts* o) {
  if (!o) return fail(WW_EINVAL, "null argument");
  o->f_tol = 1e-26;
  o->g_tol = 1e-13;
  o->df_tol = 1e-5;
  o->delta0 = 0.1;
  o->max_steps_J = 10;
  o->max_evals = 200;
  return 0;
}

}  // extern "C"
