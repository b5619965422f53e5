// Warm start of the interior-point solve from the network's prediction of
// every scenario's converged stage states.
//
// Because each scenario's MESH block is square in its own states (the paper's
// problem (10): the states of a scenario are fixed by its feeds, only the
// hydraulic rows and the objective involve d), a scenario's optimal states do
// not depend on the other scenarios, and a network trained on single-scenario
// solutions predicts them for any scenario set.  The encoding of a stage
// vector for the network: mole fractions (liquid 0-8, vapour 9-12) by their
// natural logarithm, flows, temperature and extents as they are.  The
// starting diameter is the largest hydraulic diameter of the predicted states
// times (1 + margin), so every hydraulic row starts feasible.
#include <hip/hip_runtime.h>

#include <math.h>

#include <chrono>

#include "internal.h"

namespace absorber {
namespace {

constexpr int WB = 256;
constexpr int NLOG = 13;            // stage-local entries encoded by their logarithm
constexpr double LOG_FLOOR = 1e-30;

__global__ void k_features(const double* __restrict__ feeds, int S, float* __restrict__ X) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= S) return;
  const double* F = feeds + (long long)w * NF;
  X[w * 3 + 0] = (float)F[0];  // flue-gas flow
  X[w * 3 + 1] = (float)F[1];  // CO2 fraction of the flue gas
  X[w * 3 + 2] = (float)F[5];  // flue-gas temperature
}

__global__ void k_targets(const double* __restrict__ x, long long n, float* __restrict__ T) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = (int)(i % NV);
  const double v = x[i];
  T[i] = (float)(k < NLOG ? log(fmax(v, LOG_FLOOR)) : v);
}

// decode the predicted stage vectors; each stage's hydraulic diameter into dh
__global__ void k_decode(const float* __restrict__ Y, const double* __restrict__ feeds, ModelParams p,
                         const StageInfo* __restrict__ sinfo, long long nst, double* __restrict__ x0,
                         double* __restrict__ dh) {
  const long long t = (long long)blockIdx.x * WB + threadIdx.x;
  if (t >= nst) return;
  const float* y = Y + t * NV;
  double* z = x0 + t * NV;
#pragma unroll
  for (int k = 0; k < NV; ++k) z[k] = k < NLOG ? exp((double)y[k]) : (double)y[k];
  const double P = feeds[(long long)sinfo[t].w * NF + 17];
  const double V = z[IV], T = z[IT];
  const double a = 4.0 * V * p.R * T / (M_PI * p.u_max * P);
  dh[t] = a > 0.0 ? sqrt(a) : 0.0;
}

// d_p = (1 + margin) * the largest hydraulic diameter of problem p (one block per problem)
__global__ void k_decode_d(const double* __restrict__ dh, const long long* __restrict__ pstage, double margin,
                           double* __restrict__ d0) {
  __shared__ double sm[WB];
  const int pb = blockIdx.x;
  double m = 0.0;
  for (long long t = pstage[pb] + threadIdx.x; t < pstage[pb + 1]; t += WB) m = fmax(m, dh[t]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = WB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) d0[pb] = (1.0 + margin) * sm[0];
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace absorber

using absorber::Handle;
using absorber::NV;
using absorber::set_error;

extern "C" {

int absorber_warm_features(absorber_t* ah, float* X_dev, void* stream) {
  if (!ah || !X_dev) {
    set_error("absorber_warm_features: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  hipLaunchKernelGGL(absorber::k_features, dim3(absorber::nblk(h.S, 256)), dim3(256), 0, (hipStream_t)stream,
                     h.feeds, h.S, X_dev);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

int absorber_warm_targets(absorber_t* ah, const double* x_dev, float* T_dev, void* stream) {
  if (!ah || !x_dev || !T_dev) {
    set_error("absorber_warm_targets: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  const long long n = h.nst * NV;
  hipLaunchKernelGGL(absorber::k_targets, dim3(absorber::nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, x_dev,
                     n, T_dev);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

int absorber_warm_point(absorber_t* ah, const float* Y_dev, double d_margin, double* x0_dev, void* stream) {
  if (!ah || !Y_dev || !x0_dev || !(d_margin >= 0.0)) {
    set_error("absorber_warm_point: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  const long long nst = h.nst;
  hipStream_t st = (hipStream_t)stream;
  double* dh = h.kden;  // per-stage scratch
  hipLaunchKernelGGL(absorber::k_decode, dim3(absorber::nblk(nst, absorber::WB)), dim3(absorber::WB), 0, st, Y_dev,
                     h.feeds, h.mp, h.sinfo, nst, x0_dev, dh);
  hipLaunchKernelGGL(absorber::k_decode_d, dim3(h.P), dim3(absorber::WB), 0, st, dh, h.pstage, d_margin,
                     x0_dev + nst * NV);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

int absorber_warm_start(absorber_t* ah, absorber_mlp* net, float* X_work_dev, float* Y_work_dev, double d_margin,
                        double* x0_dev, void* stream) {
  if (!ah || !net || !X_work_dev || !Y_work_dev || !x0_dev) {
    set_error("absorber_warm_start: bad argument");
    return ABS_ERR_ARG;
  }
  absorber_mlp_config cfg;
  int rc = absorber_mlp_get_config(net, &cfg);
  if (rc) return rc;
  bool fits = cfg.n_in == 3;
  for (int n : ah->h.pN) fits = fits && cfg.n_out == NV * n;
  if (!fits) {
    set_error("absorber_warm_start: the network needs 3 inputs and 21 N outputs (every problem N stages)");
    return ABS_ERR_ARG;
  }
  rc = absorber_warm_features(ah, X_work_dev, stream);
  if (!rc) rc = absorber_mlp_forward(net, X_work_dev, ah->h.S, Y_work_dev, stream);
  if (!rc) rc = absorber_warm_point(ah, Y_work_dev, d_margin, x0_dev, stream);
  return rc;
}

int absorber_warm_solve(absorber_t* ah, absorber_mlp* net, const absorber_ipm_options* opts, double d_margin,
                        double* x_out_dev, double* lambda_out_dev, absorber_ipm_result* result, int32_t* used_warm) {
  if (!ah || !net || !opts || !result) {
    set_error("absorber_warm_solve: bad argument");
    return ABS_ERR_ARG;
  }
  if (ah->h.P != 1) {
    set_error("absorber_warm_solve: single-problem handles only");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  if (!h.warm_X) {
    HIP_TRY(hipMalloc((void**)&h.warm_X, sizeof(float) * 3 * (size_t)h.S));
    HIP_TRY(hipMalloc((void**)&h.warm_Y, sizeof(float) * (size_t)NV * h.nst));
    HIP_TRY(hipMalloc((void**)&h.warm_x0, sizeof(double) * (size_t)h.nx));
  }
  const auto t0 = std::chrono::steady_clock::now();
  int rc = absorber_warm_start(ah, net, h.warm_X, h.warm_Y, d_margin, h.warm_x0, h.stream);
  if (rc) return rc;
  absorber_ipm_options ow = *opts;
  ow.warm_start = 1;
  rc = absorber_ipm_solve(ah, &ow, h.warm_x0, nullptr, x_out_dev, lambda_out_dev, result);
  const bool ok = rc == ABS_OK && result->status == ABS_OK;
  if (used_warm) *used_warm = ok ? 1 : 0;
  if (!ok) {  // cold-start fallback
    absorber_ipm_options oc = *opts;
    oc.warm_start = 0;
    const int it_warm = result->iterations;
    rc = absorber_ipm_solve(ah, &oc, nullptr, nullptr, x_out_dev, lambda_out_dev, result);
    result->iterations += it_warm;
  }
  result->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

}  // extern "C"
