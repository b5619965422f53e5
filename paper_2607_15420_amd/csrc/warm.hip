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
#include <mutex>

#include "internal.h"

namespace absorber {
namespace {

constexpr int WB = 256;
constexpr int NLOG = 13;            // stage-local entries encoded by their logarithm
constexpr double LOG_FLOOR = 1e-30;
constexpr double DUAL_SCALE = 1e-6;  // multipliers are encoded as asinh(lambda / DUAL_SCALE): signed, log-like

__global__ void k_features(const double* __restrict__ feeds, int S, float* __restrict__ X) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= S) return;
  const double* F = feeds + (long long)w * NF;
  X[w * 3 + 0] = (float)F[0];  // flue-gas flow
  X[w * 3 + 1] = (float)F[1];  // CO2 fraction of the flue gas
  X[w * 3 + 2] = (float)F[5];  // flue-gas temperature
}

// network row of chain w: its N stage vectors (21 each), then, for a
// primal-dual network, its N row-multiplier vectors (22 each); ld = 21 N or 43 N
__global__ void k_targets(const double* __restrict__ x, const double* __restrict__ lam,
                          const StageInfo* __restrict__ sinfo, long long nst, int ld, float* __restrict__ T) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nst) return;
  const StageInfo si = sinfo[t];
  float* row = T + (long long)si.w * ld;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double v = x[t * NV + k];
    row[si.n * NV + k] = (float)(k < NLOG ? log(fmax(v, LOG_FLOOR)) : v);
  }
  if (lam)
#pragma unroll
    for (int r = 0; r < NR; ++r) row[si.N * NV + si.n * NR + r] = (float)asinh(lam[t * NR + r] / DUAL_SCALE);
}

// decode the predicted stage vectors; each stage's hydraulic diameter into dh
__global__ void k_decode(const float* __restrict__ Y, int ld, const double* __restrict__ feeds, ModelParams p,
                         const StageInfo* __restrict__ sinfo, long long nst, double* __restrict__ x0,
                         double* __restrict__ dh) {
  const long long t = (long long)blockIdx.x * WB + threadIdx.x;
  if (t >= nst) return;
  const StageInfo si = sinfo[t];
  const float* y = Y + (long long)si.w * ld + si.n * NV;
  double* z = x0 + t * NV;
#pragma unroll
  for (int k = 0; k < NV; ++k) z[k] = k < NLOG ? exp((double)y[k]) : (double)y[k];
  const double P = stage_pressure(p, feeds[(long long)si.w * NF + 17], si.n, si.N);
  const double V = z[IV], T = z[IT];
  const double a = 4.0 * V * p.R * T / (M_PI * p.u_max * P);
  dh[t] = a > 0.0 ? sqrt(a) : 0.0;
}

// per problem (one block each): d_p = (1 + margin) * the largest stage diameter,
// wmax[p] = the chain holding it (lowest stage index on ties)
__global__ void k_decode_d(const double* __restrict__ dh, const long long* __restrict__ pstage,
                           const StageInfo* __restrict__ sinfo, double margin, double* __restrict__ d0,
                           int* __restrict__ wmax) {
  __shared__ double sm[WB];
  __shared__ long long si[WB];
  const int pb = blockIdx.x;
  double m = -1.0;
  long long at = pstage[pb];
  for (long long t = pstage[pb] + threadIdx.x; t < pstage[pb + 1]; t += WB)
    if (dh[t] > m) {
      m = dh[t];
      at = t;
    }
  sm[threadIdx.x] = m;
  si[threadIdx.x] = at;
  __syncthreads();
  for (int s = WB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = sm[threadIdx.x + s];
      const long long oi = si[threadIdx.x + s];
      if (o > sm[threadIdx.x] || (o == sm[threadIdx.x] && oi < si[threadIdx.x])) {
        sm[threadIdx.x] = o;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d0[pb] = (1.0 + margin) * fmax(sm[0], 0.0);
    if (wmax) wmax[pb] = sinfo[si[0]].w;
  }
}

// predicted row multipliers for the worst scenario of each problem (the only one
// whose hydraulic rows are active at the optimum), zero for the others
__global__ void k_decode_duals(const float* __restrict__ Y, int ld, const StageInfo* __restrict__ sinfo,
                               long long nst, const int* __restrict__ wmax, double* __restrict__ lam0) {
  const long long t = (long long)blockIdx.x * WB + threadIdx.x;
  if (t >= nst) return;
  const StageInfo si = sinfo[t];
  const bool worst = si.w == wmax[si.p];
  const float* y = Y + (long long)si.w * ld + si.N * NV + si.n * NR;
#pragma unroll
  for (int r = 0; r < NR; ++r) lam0[t * NR + r] = worst ? DUAL_SCALE * sinh((double)y[r]) : 0.0;
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Workspace of absorber_warm_start_noalloc: the network inputs [S][3], its
// outputs [S][n_out] and the worst scenario of each problem [P], in one
// static device array that every GPU the library runs on holds until the
// process ends.  Host code never passes the array's name to a kernel: it
// keeps the array's device address, looked up once per device.
constexpr size_t NOALLOC_BYTES = (size_t)32 << 20;
__device__ __align__(256) char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_ptr[MAX_DEVICES] = {};

// device address of the scratch array on the current device
int scratch_address(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("absorber_warm_start_noalloc: device index out of range");
    return ABS_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = scratch_ptr[dev];
  return ABS_OK;
}

inline size_t al256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

// decode Y into x0 (and lambda0) with the per-problem index buffer wmax [P]
static int warm_point(Handle& h, const float* Y_dev, int32_t n_out, double d_margin, double* x0_dev,
                      double* lambda0_dev, int* wmax, hipStream_t st) {
  if (h.npar != 1 && lambda0_dev) {
    set_error("warm start: a section handle takes the predicted states only (the network's multipliers belong to "
              "one diameter)");
    return ABS_ERR_ARG;
  }
  const long long nst = h.nst;
  double* dh = h.kden;  // per-stage scratch
  hipLaunchKernelGGL(k_decode, dim3(nblk(nst, WB)), dim3(WB), 0, st, Y_dev, n_out, h.feeds, h.mp, h.sinfo, nst, x0_dev,
                     dh);
  if (h.npar != 1) {  // each section's diameter: (1 + margin) x its largest predicted hydraulic diameter
    const int rc = set_hydraulic_diameters(h, x0_dev, d_margin, st);
    HIP_TRY(hipGetLastError());
    return rc;
  }
  hipLaunchKernelGGL(k_decode_d, dim3(h.P), dim3(WB), 0, st, dh, h.pstage, h.sinfo, d_margin, x0_dev + nst * NV, wmax);
  if (lambda0_dev)
    hipLaunchKernelGGL(k_decode_duals, dim3(nblk(nst, WB)), dim3(WB), 0, st, Y_dev, n_out, h.sinfo, nst, wmax,
                       lambda0_dev);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

}  // namespace absorber

using absorber::Handle;
using absorber::NR;
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

int absorber_warm_targets(absorber_t* ah, const double* x_dev, const double* lambda_dev, float* T_dev,
                          void* stream) {
  if (!ah || !x_dev || !T_dev) {
    set_error("absorber_warm_targets: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  for (int n : h.pN)
    if (n != h.N) {
      set_error("absorber_warm_targets: every problem must have the same stage count");
      return ABS_ERR_ARG;
    }
  const int ld = (lambda_dev ? NV + NR : NV) * h.N;
  hipLaunchKernelGGL(absorber::k_targets, dim3(absorber::nblk(h.nst, 256)), dim3(256), 0, (hipStream_t)stream, x_dev,
                     lambda_dev, h.sinfo, h.nst, ld, T_dev);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

int absorber_warm_point(absorber_t* ah, const float* Y_dev, int32_t n_out, double d_margin, double* x0_dev,
                        double* lambda0_dev, void* stream) {
  if (!ah || !Y_dev || !x0_dev || !(d_margin >= 0.0)) {
    set_error("absorber_warm_point: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  bool same = true;
  for (int n : h.pN) same = same && n == h.N;
  const bool pd = n_out == (NV + NR) * h.N;
  if (!same || !(n_out == NV * h.N || pd) || (lambda0_dev && !pd)) {
    set_error("absorber_warm_point: n_out must be 21 N (primal) or 43 N (primal-dual, needed for lambda0), "
              "every problem N stages");
    return ABS_ERR_ARG;
  }
  if (!h.warm_w) HIP_TRY(hipMalloc((void**)&h.warm_w, sizeof(int) * (size_t)h.P));
  return absorber::warm_point(h, Y_dev, n_out, d_margin, x0_dev, lambda0_dev, h.warm_w, (hipStream_t)stream);
}

int absorber_warm_start(absorber_t* ah, absorber_mlp* net, float* X_work_dev, float* Y_work_dev, double d_margin,
                        double* x0_dev, double* lambda0_dev, void* stream) {
  if (!ah || !net || !X_work_dev || !Y_work_dev || !x0_dev) {
    set_error("absorber_warm_start: bad argument");
    return ABS_ERR_ARG;
  }
  absorber_mlp_config cfg;
  int rc = absorber_mlp_get_config(net, &cfg);
  if (rc) return rc;
  if (cfg.n_in != 3) {
    set_error("absorber_warm_start: the network needs 3 inputs");
    return ABS_ERR_ARG;
  }
  rc = absorber_warm_features(ah, X_work_dev, stream);
  if (!rc) rc = absorber_mlp_forward(net, X_work_dev, ah->h.S, Y_work_dev, stream);
  if (!rc) rc = absorber_warm_point(ah, Y_work_dev, cfg.n_out, d_margin, x0_dev, lambda0_dev, stream);
  return rc;
}

int absorber_warm_start_noalloc(absorber_t* ah, absorber_mlp* net, double d_margin, double* x0_dev,
                                double* lambda0_dev, void* stream) {
  if (!ah || !net || !x0_dev || !(d_margin >= 0.0)) {
    set_error("absorber_warm_start_noalloc: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  absorber_mlp_config cfg;
  int rc = absorber_mlp_get_config(net, &cfg);
  if (rc) return rc;
  bool same = true;
  for (int n : h.pN) same = same && n == h.N;
  const bool pd = cfg.n_out == (NV + NR) * h.N;
  if (cfg.n_in != 3 || !same || !(cfg.n_out == NV * h.N || pd) || (lambda0_dev && !pd)) {
    set_error("absorber_warm_start_noalloc: the network needs 3 inputs and 21 N (primal) or 43 N (primal-dual, "
              "needed for lambda0) outputs, every problem N stages");
    return ABS_ERR_ARG;
  }
  const size_t bx = absorber::al256(sizeof(float) * 3 * (size_t)h.S);
  const size_t by = absorber::al256(sizeof(float) * (size_t)cfg.n_out * (size_t)h.S);
  const size_t bw = absorber::al256(sizeof(int) * (size_t)h.P);
  if (bx + by + bw > absorber::NOALLOC_BYTES) {
    set_error("absorber_warm_start_noalloc: " + std::to_string(h.S) + " scenarios x " + std::to_string(cfg.n_out) +
              " network outputs need " + std::to_string(bx + by + bw) + " bytes of workspace, more than its " +
              std::to_string(absorber::NOALLOC_BYTES) + "-byte maximum (use absorber_warm_start)");
    return ABS_ERR_ARG;
  }
  char* ws = nullptr;
  rc = absorber::scratch_address(&ws);
  if (rc) return rc;
  float* X = reinterpret_cast<float*>(ws);
  float* Y = reinterpret_cast<float*>(ws + bx);
  int* wmax = reinterpret_cast<int*>(ws + bx + by);
  rc = absorber_warm_features(ah, X, stream);
  if (!rc) rc = absorber_mlp_forward(net, X, h.S, Y, stream);
  if (!rc) rc = absorber::warm_point(h, Y, cfg.n_out, d_margin, x0_dev, lambda0_dev, wmax, (hipStream_t)stream);
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
  absorber_mlp_config cfg;
  int rc = absorber_mlp_get_config(net, &cfg);
  if (rc) return rc;
  // primal-dual network: predicted multipliers (one diameter only; a section
  // handle starts from the predicted states with least-squares multipliers)
  const bool pd = cfg.n_out == (NV + NR) * h.N && h.npar == 1;
  if (!h.warm_X) {
    HIP_TRY(hipMalloc((void**)&h.warm_X, sizeof(float) * 3 * (size_t)h.S));
    HIP_TRY(hipMalloc((void**)&h.warm_Y, sizeof(float) * (size_t)(NV + NR) * h.nst));
    HIP_TRY(hipMalloc((void**)&h.warm_x0, sizeof(double) * (size_t)h.nx));
    HIP_TRY(hipMalloc((void**)&h.warm_l0, sizeof(double) * (size_t)h.nc));
  }
  const auto t0 = std::chrono::steady_clock::now();
  rc = absorber_warm_start(ah, net, h.warm_X, h.warm_Y, d_margin, h.warm_x0, pd ? h.warm_l0 : nullptr, h.stream);
  if (rc) return rc;
  absorber_ipm_options ow = *opts;
  ow.warm_start = 1;
  rc = absorber_ipm_solve(ah, &ow, h.warm_x0, pd ? h.warm_l0 : nullptr, x_out_dev, lambda_out_dev, result);
  if (rc < 0 && rc > ABS_ERR_INERTIA) return rc;  // argument, device or allocation error
  const bool converged = rc == ABS_OK && result->status == ABS_OK;
  // the network's start counts only when that run converged by itself, not
  // through the feasibility restart (which starts from simulated states)
  if (used_warm) *used_warm = converged && result->feasibility_restarts == 0 ? 1 : 0;
  if (!converged) {  // cold-start fallback
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
