// SDC15 time stepping (Wilkening & Yu, Sec. 2.2): the stage states of one step are
// linear combinations y_0 + dt sum_t w_t K_{j_t} of the step's start state and earlier
// stage slopes (the step written as an explicit Runge-Kutta method of 113 stages, each
// row sparse); this kernel forms one of them for every state column.
#pragma once
#include "ww_kernels.hpp"

#define SDC_NODES 8
#define SDC_SWEEPS 10
#define SDC_STAGES (4 * SDC_NODES + 1 + SDC_SWEEPS * SDC_NODES)   // 113
#define SDC_MAXNZ 32
// the first stage of the correction sweeps (after the predictor's RK4 stages and F at the
// last predicted node)
#define SDC_FIRST_SWEEP (4 * SDC_NODES + 1)
// refinement sweeps of a predictor stage's base solve on lagged factors
#define LAG_SWEEPS 4

// out[e] = y0[e] + dt sum_{t < cnt} w[t] K[j[t] kstride + e], e < n, in increasing t
// (out may be y0: every element is read before it is written, by the same thread)
__global__ void k_sdc_combine(const double* y0, const double* __restrict__ K, size_t kstride,
                              const int* __restrict__ jt, const double* __restrict__ wt, int cnt, double dt,
                              double* out, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double acc = y0[e];
    for (int t = 0; t < cnt; ++t) acc = fma(dt * wt[t], K[(size_t)jt[t] * kstride + e], acc);
    out[e] = acc;
  }
}
