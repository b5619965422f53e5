// Process simulation on the device: every scenario's MESH equations form a
// square system in its own stage states once the feeds are fixed (the paper's
// degrees-of-freedom argument for the equilibrium model), so they can be
// solved scenario by scenario by Newton's method, independently of d.
//
// One Newton step for all chains at once reuses the bordered KKT machinery:
// with zero Hessian weights, Sigma_x = Sigma_s = 0, delta_w = 1 and delta_c = 0
// the primal-dual system [[I, J^T], [J, 0]] [dx; l] = [0; -c] yields J_F dx =
// -c_F exactly in the MESH rows (the hydraulic rows and d are left free and
// do not enter J_F).  As in the process-simulation oracle, the mole fractions
// are stepped in their logarithm (x <- x exp(a dx / x), which keeps them
// positive and leaves the Newton direction unchanged), the largest log-step
// is capped at 5, and each chain backtracks on its own scaled residual
// inf-norm with a sufficient-decrease test.
//
// A scenario whose Newton iteration stalls starts again (at most twice) from the
// converged states of the closest scenario (in feed) of the same problem.
//
// Used by the interior-point driver as a feasibility restart: a problem whose
// cold-started solve stops (line-search failure, inertia failure, iteration
// limit) is solved again from its simulated states.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace absorber {
namespace {

constexpr int BS = 256;
constexpr int NLOG = 13;  // stage-local entries stepped in their logarithm (mole fractions)
inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Newton right-hand side in KKT layout: 0 for primals, hydraulic duals and the
// d's, -c~ for the MESH rows
// Newton right-hand side -F on the MESH rows; zero on the chains whose mask entry is 0
__global__ void k_newton_rhs(const double* __restrict__ c, const int* __restrict__ chmask,
                             const StageInfo* __restrict__ sinfo, long long nks, long long nkkt,
                             double* __restrict__ rhs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nkkt) return;
  double v = 0.0;
  if (i < nks) {
    const long long t = i / NK;
    const int k = (int)(i % NK);
    if (k >= NV && k < NV + NE && chmask[sinfo[t].w]) v = -c[t * NR + (k - NV)];
  }
  rhs[i] = v;
}

// primal part of a KKT-layout vector
__global__ void k_primal_of(const double* __restrict__ sol, long long nxs, long long nx, long long nks,
                            double* __restrict__ dx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  dx[i] = i >= nxs ? sol[nks + (i - nxs)] : sol[(i / NV) * NK + (i % NV)];
}

// per chain: out[2w] = inf-norm of the MESH residuals (inf if one is not
// finite); with dx, out[2w+1] = the largest |dx / x| over the mole fractions
__global__ void k_chain_stats(const double* __restrict__ c, const double* __restrict__ x,
                              const double* __restrict__ dx, const int* __restrict__ chain0, int W,
                              double* __restrict__ out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  double nr = 0.0, big = 0.0;
  for (long long t = chain0[w]; t < chain0[w + 1]; ++t) {
    for (int r = 0; r < NE; ++r) {
      const double v = c[t * NR + r];
      nr = isfinite(v) ? fmax(nr, fabs(v)) : INFINITY;
    }
    if (dx)
      for (int k = 0; k < NLOG; ++k) big = fmax(big, fabs(dx[t * NV + k] / x[t * NV + k]));
  }
  out[2 * w] = nr;
  out[2 * w + 1] = big;
}

// trial point: each chain steps by its own a_w (0 leaves it unchanged); d's copied
__global__ void k_newton_trial(const double* __restrict__ x, const double* __restrict__ dx,
                               const double* __restrict__ aw, const StageInfo* __restrict__ sinfo, long long nxs,
                               long long nx, double* __restrict__ xt) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  if (i >= nxs) {
    xt[i] = x[i];
    return;
  }
  const double a = aw[sinfo[i / NV].w];
  const int k = (int)(i % NV);
  xt[i] = k < NLOG ? x[i] * exp(a * dx[i] / x[i]) : x[i] + a * dx[i];
}

// restart chains from the states of another chain of the same stage count:
// xt[stage n of chain w] = xt[stage n of chain src[w]] for src[w] >= 0
__global__ void k_copy_chain(double* __restrict__ xt, const int* __restrict__ src, const int* __restrict__ chain0,
                             const StageInfo* __restrict__ sinfo, long long nxs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nxs) return;
  const StageInfo si = sinfo[i / NV];
  const int s = src[si.w];
  if (s < 0) return;
  xt[i] = xt[((long long)chain0[s] + si.n) * NV + (i % NV)];
}

__global__ void k_scale(const double* __restrict__ x, Scaling sc, long long nx, long long nxs, int divide,
                        double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  const double s = i >= nxs ? sc.Dd : sc.D[i % NV];
  out[i] = divide ? x[i] / s : x[i] * s;
}

__global__ void k_rowscale_n(const double* __restrict__ rowmax, double gmax, long long n, double* __restrict__ cs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cs[i] = fmin(1.0, gmax / fmax(rowmax[i], 1e-300));
}

__global__ void k_fill_n(double* __restrict__ p, double v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// hydraulic diameter sqrt(4 V R T / (pi u_max P)) of every stage of x (unscaled)
__global__ void k_stage_diam(const double* __restrict__ x, const double* __restrict__ feeds, ModelParams p,
                             const StageInfo* __restrict__ sinfo, long long nst, double* __restrict__ dh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nst) return;
  const StageInfo si = sinfo[t];
  const double P = stage_pressure(p, feeds[(long long)si.w * NF + 17], si.n, si.N);
  const double a = 4.0 * x[t * NV + IV] * p.R * x[t * NV + IT] / (M_PI * p.u_max * P);
  dh[t] = a > 0.0 ? sqrt(a) : 0.0;
}

// design entry k of problem p = (1 + margin) max over the problem's stages in
// section k (one block per entry; one section: d_p over all of its stages)
__global__ void k_problem_max(const double* __restrict__ dh, const long long* __restrict__ pstage,
                              const StageInfo* __restrict__ sinfo, int npar, double margin, double* __restrict__ d) {
  __shared__ double sm[BS];
  const int pb = blockIdx.x / npar, k = blockIdx.x % npar;
  double m = 0.0;
  for (long long t = pstage[pb] + threadIdx.x; t < pstage[pb + 1]; t += BS)
    if (npar == 1 || section_of(sinfo[t].n, sinfo[t].N, npar) == k) m = fmax(m, dh[t]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) d[blockIdx.x] = (1.0 + margin) * sm[0];
}

struct Buf {
  std::vector<void*> dev, host;
  ~Buf() {
    for (void* p : dev) (void)hipFree(p);
    for (void* p : host) (void)hipHostFree(p);
  }
  template <class T>
  hipError_t d(T** p, long long n) {
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)std::max<long long>(n, 1));
    if (e == hipSuccess) dev.push_back((void*)*p);
    return e;
  }
  template <class T>
  hipError_t h(T** p, long long n) {
    hipError_t e = hipHostMalloc((void**)p, sizeof(T) * (size_t)std::max<long long>(n, 1), 0);
    if (e == hipSuccess) host.push_back((void*)*p);
    return e;
  }
};

}  // namespace

int simulate(Handle& h, double* x_dev, const unsigned char* pmask, double tol, int max_iter, int* conv,
             int* iters) {
  hipStream_t st = h.stream;
  const int P = h.P, W = h.S;
  const long long nx = h.nx, nst = h.nst, nkkt = h.nkkt, nxs = nst * NV, nks = nst * NK;
  Buf B;
  double *xt, *xtt, *c, *ct, *rhs, *sol, *dx, *rowmax, *aw, *stats;
  HIP_TRY(B.d(&xt, nx));
  HIP_TRY(B.d(&xtt, nx));
  HIP_TRY(B.d(&c, h.nc));
  HIP_TRY(B.d(&ct, h.nc));
  HIP_TRY(B.d(&rhs, nkkt));
  HIP_TRY(B.d(&sol, nkkt));
  HIP_TRY(B.d(&dx, nx));
  HIP_TRY(B.d(&rowmax, h.nc));
  HIP_TRY(B.d(&aw, W));
  HIP_TRY(B.d(&stats, 2LL * W));
  double *aw_h, *st_h;
  HIP_TRY(B.h(&aw_h, W));
  HIP_TRY(B.h(&st_h, 2LL * W));
  int *src, *src_h, *cm, *cm_h;
  HIP_TRY(B.d(&src, W));
  HIP_TRY(B.h(&src_h, W));
  HIP_TRY(B.d(&cm, W));
  HIP_TRY(B.h(&cm_h, W));
  std::vector<int> wp((size_t)W);  // problem of each chain
  for (int p = 0; p < P; ++p)
    for (long long w = h.pchain_h[(size_t)p]; w < h.pchain_h[(size_t)p + 1]; ++w) wp[(size_t)w] = p;
  // work only on the requested problems (factorisation, evaluation, solves, residuals)
  int* pm_h = nullptr;
  HIP_TRY(B.h(&pm_h, P));
  for (int p = 0; p < P; ++p) pm_h[p] = !pmask || pmask[p];
  HIP_TRY(hipMemcpyAsync(h.pact, pm_h, sizeof(int) * P, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(h.fmask, pm_h, sizeof(int) * P, hipMemcpyHostToDevice, st));
  struct PactGuard {
    Handle& h;
    ~PactGuard() {
      h.pact_on = false;
      h.chmask = nullptr;
    }
  } pact_guard{h};
  h.pact_on = true;
  // scaling as in the interior-point method: variables by the cold point,
  // rows by their largest scaled gradient entry at the starting point
  for (int k = 0; k < NV; ++k) h.sc.D[k] = h.x0[k] != 0.0 ? fabs(h.x0[k]) : 1.0;
  h.sc.Dd = h.x0[NV] != 0.0 ? fabs(h.x0[NV]) : 1.0;
  hipLaunchKernelGGL(k_scale, dim3(nblk(nx, BS)), dim3(BS), 0, st, x_dev, h.sc, nx, nxs, 1, xt);
  HIP_TRY(launch_rowmax(h, xt, 1, rowmax, st));
  hipLaunchKernelGGL(k_rowscale_n, dim3(nblk(h.nc, BS)), dim3(BS), 0, st, rowmax, 100.0, h.nc, h.cs);
  // Newton matrix regularisation: delta_w = 1, delta_c = 0, no barrier diagonals
  hipLaunchKernelGGL(k_fill_n, dim3(nblk(nx, BS)), dim3(BS), 0, st, h.diagx, 0.0, nx);
  hipLaunchKernelGGL(k_fill_n, dim3(nblk(nst, BS)), dim3(BS), 0, st, h.diags, 0.0, nst);
  hipLaunchKernelGGL(k_fill_n, dim3(nblk(P, BS)), dim3(BS), 0, st, h.dwv, 1.0, (long long)P);
  hipLaunchKernelGGL(k_fill_n, dim3(nblk(P, BS)), dim3(BS), 0, st, h.dcv, 0.0, (long long)P);
  HIP_TRY(launch_eval(h, xt, 1, nullptr, 1, c, st));
  hipLaunchKernelGGL(k_chain_stats, dim3(nblk(W, 64)), dim3(64), 0, st, c, xt, nullptr, h.chain0, W, stats);
  HIP_TRY(hipMemcpyAsync(st_h, stats, sizeof(double) * 2 * W, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<double> nr((size_t)W);
  for (int w = 0; w < W; ++w) nr[(size_t)w] = st_h[2 * w];
  std::vector<char> stalled((size_t)W, 0);  // backtracking exhausted without decrease
  // Slow chains: in the first two rounds a chain whose residual has not fallen
  // tenfold over ten steps pauses when its problem already has a converged
  // chain; the round then ends sooner and the paused chain starts again from
  // the closest converged neighbour.
  std::vector<char> slow((size_t)W, 0);
  std::vector<double> mark((size_t)W);
  std::vector<char> pconv((size_t)P);
  auto wanted = [&](int w) {
    return (!pmask || pmask[wp[(size_t)w]]) && !stalled[(size_t)w] && !slow[(size_t)w];
  };
  int it = 0, it_total = 0;
  constexpr int ROUNDS = 3, SLOW_EVERY = 10;
  for (int round = 0; round < ROUNDS; ++round) {
    mark = nr;
    for (it = 0; it < max_iter; ++it, ++it_total) {
      bool any = false;
      for (int w = 0; w < W; ++w) any = any || (wanted(w) && !(nr[(size_t)w] <= tol));
      if (!any) break;
      // only the chains still iterating are factorised and solved: the others
      // take a zero step
      for (int w = 0; w < W; ++w) cm_h[w] = wanted(w) && !(nr[(size_t)w] <= tol) ? 1 : 0;
      HIP_TRY(hipMemcpyAsync(cm, cm_h, sizeof(int) * W, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_newton_rhs, dim3(nblk(nkkt, BS)), dim3(BS), 0, st, c, cm, h.sinfo, nks, nkkt, rhs);
      h.chmask = cm;
      HIP_TRY(launch_factor(h, h.diagx, h.diags, rhs, true, st));
      HIP_TRY(launch_schur(h, h.diagx, rhs, 1, sol, st));
      double rel = 0.0;
      {
        // a Newton step needs no 1e-10 solve: each step's residual is then at
        // most about 1e-6 of the previous one plus the second-order terms
        const int rc = kkt_solve_refined(h, rhs, sol, true, &rel, st, false, nullptr, 1e-6);
        h.chmask = nullptr;
        if (rc) return rc;
      }
      hipLaunchKernelGGL(k_primal_of, dim3(nblk(nx, BS)), dim3(BS), 0, st, sol, nxs, nx, nks, dx);
      hipLaunchKernelGGL(k_chain_stats, dim3(nblk(W, 64)), dim3(64), 0, st, c, xt, dx, h.chain0, W, stats);
      HIP_TRY(hipMemcpyAsync(st_h, stats, sizeof(double) * 2 * W, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      std::vector<char> searching((size_t)W, 0);
      for (int w = 0; w < W; ++w) {
        const bool go = wanted(w) && !(nr[(size_t)w] <= tol);
        const double big = st_h[2 * w + 1];
        aw_h[w] = go ? (big > 5.0 ? 5.0 / big : 1.0) : 0.0;
        searching[(size_t)w] = go;
      }
      while (true) {  // backtracking, every chain on its own residual
        HIP_TRY(hipMemcpyAsync(aw, aw_h, sizeof(double) * W, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_newton_trial, dim3(nblk(nx, BS)), dim3(BS), 0, st, xt, dx, aw, h.sinfo, nxs, nx, xtt);
        HIP_TRY(launch_eval(h, xtt, 1, nullptr, 0, ct, st));
        hipLaunchKernelGGL(k_chain_stats, dim3(nblk(W, 64)), dim3(64), 0, st, ct, xtt, nullptr, h.chain0, W, stats);
        HIP_TRY(hipMemcpyAsync(st_h, stats, sizeof(double) * 2 * W, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        bool more = false;
        for (int w = 0; w < W; ++w) {
          if (!searching[(size_t)w]) continue;
          const double a = aw_h[w], nt = st_h[2 * w];
          const bool dec = std::isfinite(nt) && nt < (1.0 - 1e-4 * a) * nr[(size_t)w];
          if (dec || a < 1e-10) {
            searching[(size_t)w] = 0;
            if (!dec) stalled[(size_t)w] = 1;  // no decrease even for a tiny step: give up on this chain
            nr[(size_t)w] = nt;
            continue;
          }
          aw_h[w] = 0.5 * a;
          more = true;
        }
        if (!more) break;
      }
      std::swap(xt, xtt);
      HIP_TRY(launch_eval(h, xt, 1, nullptr, 1, c, st));
      if (round < ROUNDS - 1 && it % SLOW_EVERY == SLOW_EVERY - 1) {
        std::fill(pconv.begin(), pconv.end(), 0);
        for (int w = 0; w < W; ++w)
          if (nr[(size_t)w] <= tol) pconv[(size_t)wp[(size_t)w]] = 1;
        for (int w = 0; w < W; ++w) {
          if (wanted(w) && !(nr[(size_t)w] <= tol) && pconv[(size_t)wp[(size_t)w]] &&
              !(nr[(size_t)w] < 0.1 * mark[(size_t)w]))
            slow[(size_t)w] = 1;
          mark[(size_t)w] = nr[(size_t)w];
        }
      }
    }
    // chains that did not converge start again from the states of the converged
    // chain of the same problem whose feed is closest (scenarios differ only in
    // their feeds, so a neighbour's solution is a close starting point)
    bool any_src = false;
    for (int w = 0; w < W; ++w) {
      src_h[w] = -1;
      if (!(!pmask || pmask[wp[(size_t)w]]) || nr[(size_t)w] <= tol) continue;
      const int p = wp[(size_t)w];
      const double* fw = &h.feeds_h[(size_t)w * NF];
      double best = INFINITY;
      for (long long v = h.pchain_h[(size_t)p]; v < h.pchain_h[(size_t)p + 1]; ++v) {
        if (!(nr[(size_t)v] <= tol)) continue;
        const double* fv = &h.feeds_h[(size_t)v * NF];
        const double dist = fabs(fv[0] - fw[0]) / fabs(fw[0]) + fabs(fv[1] - fw[1]) / fabs(fw[1]) +
                            fabs(fv[5] - fw[5]) / fabs(fw[5]);
        if (dist < best) {
          best = dist;
          src_h[w] = (int)v;
        }
      }
      any_src = any_src || src_h[w] >= 0;
    }
    if (!any_src) break;
    HIP_TRY(hipMemcpyAsync(src, src_h, sizeof(int) * W, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_copy_chain, dim3(nblk(nxs, BS)), dim3(BS), 0, st, xt, src, h.chain0, h.sinfo, nxs);
    HIP_TRY(launch_eval(h, xt, 1, nullptr, 1, c, st));
    hipLaunchKernelGGL(k_chain_stats, dim3(nblk(W, 64)), dim3(64), 0, st, c, xt, nullptr, h.chain0, W, stats);
    HIP_TRY(hipMemcpyAsync(st_h, stats, sizeof(double) * 2 * W, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int w = 0; w < W; ++w) {
      if (src_h[w] >= 0) {
        nr[(size_t)w] = st_h[2 * w];
        stalled[(size_t)w] = 0;
      }
      slow[(size_t)w] = 0;  // paused chains without a neighbour continue where they were
    }
  }
  it = it_total;
  hipLaunchKernelGGL(k_scale, dim3(nblk(nx, BS)), dim3(BS), 0, st, xt, h.sc, nx, nxs, 0, x_dev);
  HIP_TRY(hipStreamSynchronize(st));
  if (conv)
    for (int p = 0; p < P; ++p) {
      int ok = 1;
      for (long long w = h.pchain_h[(size_t)p]; w < h.pchain_h[(size_t)p + 1]; ++w) ok = ok && nr[(size_t)w] <= tol;
      conv[p] = ok;
    }
  if (iters) *iters = it;
  h.factored = false;  // the stored factors are the Newton matrix's, not a KKT matrix the caller asked for
  return ABS_OK;
}

int set_hydraulic_diameters(Handle& h, double* x_dev, double margin, hipStream_t st) {
  double* dh = h.kden;  // per-stage scratch
  hipLaunchKernelGGL(k_stage_diam, dim3(nblk(h.nst, BS)), dim3(BS), 0, st, x_dev, h.feeds, h.mp, h.sinfo, h.nst, dh);
  hipLaunchKernelGGL(k_problem_max, dim3(h.P * h.npar), dim3(BS), 0, st, dh, h.pstage, h.sinfo, h.npar, margin,
                     x_dev + h.nst * NV);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

}  // namespace absorber

using absorber::Handle;
using absorber::set_error;

extern "C" {

int absorber_simulate(absorber_t* ah, double* x_dev, double tol, int32_t max_iter, int32_t* converged_host,
                      int32_t* iterations_host) {
  if (!ah || !x_dev || !(tol > 0.0) || max_iter < 0) {
    set_error("absorber_simulate: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = ah->h;
  std::vector<int> conv((size_t)h.P);
  int it = 0;
  int rc = absorber::simulate(h, x_dev, nullptr, tol, max_iter, conv.data(), &it);
  if (rc) return rc;
  rc = absorber::set_hydraulic_diameters(h, x_dev, 0.0, h.stream);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h.stream));
  if (converged_host)
    for (int p = 0; p < h.P; ++p) converged_host[p] = conv[(size_t)p];
  if (iterations_host) *iterations_host = it;
  return ABS_OK;
}

}  // extern "C"
