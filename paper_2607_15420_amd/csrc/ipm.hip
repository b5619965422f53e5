// Filter line-search primal-dual interior-point method (the algorithm MadNLP
// implements, Waechter & Biegler 2006) for problem (10), driven from the host
// with every vector operation, reduction, evaluation and linear solve on the
// device.  Host work is scalar control flow: barrier update, inertia
// correction, filter and step acceptance.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <utility>
#include <vector>

#include "internal.h"

namespace absorber {
namespace {

constexpr int BS = 256;
inline unsigned grid_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// scaled bounds per stage-local index (0-20) and d (21)
struct Bnd {
  double lo[NV + 1], hi[NV + 1];
};

__device__ __forceinline__ int lidx(long long i, long long nx) { return i == nx - 1 ? NV : (int)(i % NV); }

// primal index -> KKT index
__device__ __forceinline__ long long kkt_of_primal(long long i, long long nx, long long nkkt) {
  return i == nx - 1 ? nkkt - 1 : (i / NV) * NK + (i % NV);
}
// row index -> KKT index
__device__ __forceinline__ long long kkt_of_row(long long j) {
  const long long t = j / NR;
  const int r = (int)(j % NR);
  return t * NK + (r < NE ? NV + r : NK - 1);
}

template <int K>
struct Part {
  double v[K];
};

// block reduction of K values: op 0 sum, 1 max, 2 min; per-block partials
template <int K>
__device__ void block_reduce(Part<K> p, const int* ops, double* out) {
  __shared__ double sm[K][BS];
  for (int k = 0; k < K; ++k) sm[k][threadIdx.x] = p.v[k];
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < K; ++k) {
        const double a = sm[k][threadIdx.x], b = sm[k][threadIdx.x + s];
        sm[k][threadIdx.x] = ops[k] == 0 ? a + b : (ops[k] == 1 ? fmax(a, b) : fmin(a, b));
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) out[blockIdx.x * K + k] = sm[k][0];
}

// ---- Lagrangian gradient g = grad f~ + J~^T y for the stage primals; d part in dpart
__global__ void k_lag_grad(const double* __restrict__ rec, const int* __restrict__ jtab,
                           const double* __restrict__ y, int N, int S, double* __restrict__ g,
                           double* __restrict__ dpart) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int n = (int)(t % N);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const double* R = rec + t * REC;
  const double* yy = y + t * NR;
  double dp = 0.0;
  for (int e = 0; e < NJO; ++e) {
    const int rc = jtab[e];
    const int r = rc & 255, col = (rc >> 8) & 255, blk = rc >> 16;
    if (blk == BLK_D) dp += R[REC_OWN + e] * yy[r];
    else acc[col] += R[REC_OWN + e] * yy[r];
  }
  if (n > 0) {  // rows of stage n-1 depend on this stage through the liquid it receives
    const double* R0 = R - REC;
    const double* y0 = yy - NR;
    for (int e = 0; e < NJU; ++e) {
      const int rc = jtab[NJO + e];
      acc[(rc >> 8) & 255] += R0[REC_UP + e] * y0[rc & 255];
    }
  }
  if (n < N - 1) {  // rows of stage n+1 depend on this stage through the vapour it receives
    const double* R1 = R + REC;
    const double* y1 = yy + NR;
    for (int e = 0; e < NJD; ++e) {
      const int rc = jtab[NJO + NJU + e];
      acc[(rc >> 8) & 255] += R1[REC_DOWN + e] * y1[rc & 255];
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) g[t * NV + k] = acc[k];
  dpart[t] = dp;
}

// g_d = sf * D_d + sum over all hydraulic rows (one block, fixed order)
__global__ void k_grad_d(const double* __restrict__ dpart, long long nst, double gf, double* __restrict__ gd) {
  __shared__ double sm[BS];
  double a = 0.0;
  for (long long t = threadIdx.x; t < nst; t += BS) a += dpart[t];
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *gd = gf + sm[0];
}

// ---- optimality-error partials
// 0 max|g - zL + zU|, 1 max|vU - y_hyd|, 2 max|cE|, 3 max|c_hyd - s|, 4 min compl product,
// 5 max compl product, 6 sum|y|, 7 sum|z| (zL, zU, vU), 8 nonfinite count
__global__ void k_opt_parts(const double* __restrict__ x, const double* __restrict__ zL, const double* __restrict__ zU,
                            const double* __restrict__ g, const double* __restrict__ y, const double* __restrict__ c,
                            const double* __restrict__ s, const double* __restrict__ vU, Bnd b, long long nx,
                            long long nc, long long nst, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  Part<9> p;
  p.v[0] = p.v[1] = p.v[2] = p.v[3] = 0.0;
  p.v[4] = INFINITY;
  p.v[5] = -INFINITY;
  p.v[6] = p.v[7] = p.v[8] = 0.0;
  if (i < nx) {
    const int k = lidx(i, nx);
    const double gi = g[i] - zL[i] + zU[i];
    p.v[0] = fabs(gi);
    if (!isfinite(gi)) p.v[8] += 1.0;
    if (isfinite(b.lo[k])) {
      const double pr = (x[i] - b.lo[k]) * zL[i];
      p.v[4] = fmin(p.v[4], pr);
      p.v[5] = fmax(p.v[5], pr);
      p.v[7] += fabs(zL[i]);
    }
    if (isfinite(b.hi[k])) {
      const double pr = (b.hi[k] - x[i]) * zU[i];
      p.v[4] = fmin(p.v[4], pr);
      p.v[5] = fmax(p.v[5], pr);
      p.v[7] += fabs(zU[i]);
    }
  }
  if (i < nc) {
    const double cj = c[i];
    if (!isfinite(cj)) p.v[8] += 1.0;
    p.v[6] += fabs(y[i]);
    if (i % NR != NR - 1) p.v[2] = fabs(cj);
  }
  if (i < nst) {
    p.v[1] = fabs(vU[i] - y[i * NR + NR - 1]);
    p.v[3] = fabs(c[i * NR + NR - 1] - s[i]);
    const double pr = -s[i] * vU[i];
    p.v[4] = fmin(p.v[4], pr);
    p.v[5] = fmax(p.v[5], pr);
    p.v[7] += fabs(vU[i]);
  }
  const int ops[9] = {1, 1, 1, 1, 2, 1, 0, 0, 0};
  block_reduce<9>(p, ops, out);
}

// ---- barrier diagonals
__global__ void k_sigma(const double* __restrict__ x, const double* __restrict__ zL, const double* __restrict__ zU,
                        const double* __restrict__ s, const double* __restrict__ vU, Bnd b, long long nx,
                        long long nst, double* __restrict__ dx, double* __restrict__ ds) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) {
    const int k = lidx(i, nx);
    double sg = 0.0;
    if (isfinite(b.lo[k])) sg += zL[i] / (x[i] - b.lo[k]);
    if (isfinite(b.hi[k])) sg += zU[i] / (b.hi[k] - x[i]);
    dx[i] = sg;
  }
  if (i < nst) ds[i] = vU[i] / (-s[i]);
}

// barrier gradient of a primal entry (without J^T y)
__device__ __forceinline__ double barrier_grad(double xi, int k, const Bnd& b, double mu, double kd, double gf) {
  double v = (k == NV) ? gf : 0.0;
  const bool hl = isfinite(b.lo[k]), hu = isfinite(b.hi[k]);
  if (hl) v -= mu / (xi - b.lo[k]);
  if (hu) v += mu / (b.hi[k] - xi);
  if (hl && !hu) v += kd * mu;
  if (hu && !hl) v -= kd * mu;
  return v;
}

// ---- right-hand side of the slack-reduced primal-dual system
__global__ void k_rhs(const double* __restrict__ x, const double* __restrict__ g, const double* __restrict__ y,
                      const double* __restrict__ c, const double* __restrict__ s, const double* __restrict__ ds,
                      Bnd b, double mu, double kd, double gf, double dw, long long nx, long long nc, long long nst,
                      long long nkkt, double* __restrict__ rhs) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) {
    const int k = lidx(i, nx);
    // g holds grad f~ + J~^T y; remove grad f~ for d since barrier_grad adds it
    const double gl = (k == NV) ? g[i] - gf : g[i];
    rhs[kkt_of_primal(i, nx, nkkt)] = -(gl + barrier_grad(x[i], k, b, mu, kd, gf));
  }
  if (i < nc && i % NR != NR - 1) rhs[kkt_of_row(i)] = -c[i];
  if (i < nst) {
    const double yh = y[i * NR + NR - 1];
    const double rs = mu / (-s[i]) - kd * mu - yh;
    const double rd = c[i * NR + NR - 1] - s[i];
    rhs[i * NK + NK - 1] = -rd - rs / (ds[i] + dw);
  }
}

// ---- search direction pieces, fraction to the boundary and grad(phi)^T dx
// partials: 0 min alpha primal, 1 min alpha dual, 2 sum grad phi . d
__global__ void k_direction(const double* __restrict__ x, const double* __restrict__ zL,
                            const double* __restrict__ zU, const double* __restrict__ y, const double* __restrict__ s,
                            const double* __restrict__ vU, const double* __restrict__ dss,
                            const double* __restrict__ sol, Bnd b, double mu, double kd, double gf, double dw,
                            double tau, long long nx, long long nc, long long nst, long long nkkt,
                            double* __restrict__ dx, double* __restrict__ dy, double* __restrict__ dzL,
                            double* __restrict__ dzU, double* __restrict__ dsl, double* __restrict__ dvU,
                            double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  Part<3> p;
  p.v[0] = 1.0;
  p.v[1] = 1.0;
  p.v[2] = 0.0;
  if (i < nx) {
    const int k = lidx(i, nx);
    const double d = sol[kkt_of_primal(i, nx, nkkt)];
    dx[i] = d;
    const double xi = x[i];
    double a = 0.0, bz = 0.0;
    if (isfinite(b.lo[k])) {
      const double sl = xi - b.lo[k];
      a = mu / sl - zL[i] - zL[i] / sl * d;
      if (d < 0.0) p.v[0] = fmin(p.v[0], -tau * sl / d);
      if (a < 0.0) p.v[1] = fmin(p.v[1], -tau * zL[i] / a);
    }
    if (isfinite(b.hi[k])) {
      const double su = b.hi[k] - xi;
      bz = mu / su - zU[i] + zU[i] / su * d;
      if (d > 0.0) p.v[0] = fmin(p.v[0], tau * su / d);
      if (bz < 0.0) p.v[1] = fmin(p.v[1], -tau * zU[i] / bz);
    }
    dzL[i] = a;
    dzU[i] = bz;
    p.v[2] += barrier_grad(xi, k, b, mu, kd, gf) * d;
  }
  if (i < nc) dy[i] = sol[kkt_of_row(i)];
  if (i < nst) {
    const double si = -s[i];  // distance of the slack to its bound 0
    const double yh = y[i * NR + NR - 1];
    const double rs = mu / si - kd * mu - yh;
    const double dyh = sol[i * NK + NK - 1];
    const double d = (dyh - rs) / (dss[i] + dw);
    dsl[i] = d;
    const double dv = mu / si - vU[i] + vU[i] / si * d;
    dvU[i] = dv;
    if (d > 0.0) p.v[0] = fmin(p.v[0], tau * si / d);
    if (dv < 0.0) p.v[1] = fmin(p.v[1], -tau * vU[i] / dv);
    p.v[2] += (mu / si - kd * mu) * d;
  }
  const int ops[3] = {2, 2, 0};
  block_reduce<3>(p, ops, out);
}

__global__ void k_trial(const double* __restrict__ x, const double* __restrict__ dx, const double* __restrict__ s,
                        const double* __restrict__ dsl, double a, long long nx, long long nst, double* __restrict__ xt,
                        double* __restrict__ st) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) xt[i] = x[i] + a * dx[i];
  if (i < nst) st[i] = s[i] + a * dsl[i];
}

// line-search partials at a trial point: 0 theta (1-norm), 1 barrier sum, 2 infeasible count
__global__ void k_ls_parts(const double* __restrict__ xt, const double* __restrict__ st, const double* __restrict__ c,
                           Bnd b, double mu, double kd, long long nx, long long nc, long long nst,
                           double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  Part<3> p;
  p.v[0] = p.v[1] = p.v[2] = 0.0;
  if (i < nx) {
    const int k = lidx(i, nx);
    const bool hl = isfinite(b.lo[k]), hu = isfinite(b.hi[k]);
    if (hl) {
      const double sl = xt[i] - b.lo[k];
      if (!(sl > 0.0)) p.v[2] += 1.0;
      else p.v[1] -= mu * log(sl);
      if (!hu) p.v[1] += kd * mu * sl;
    }
    if (hu) {
      const double su = b.hi[k] - xt[i];
      if (!(su > 0.0)) p.v[2] += 1.0;
      else p.v[1] -= mu * log(su);
      if (!hl) p.v[1] += kd * mu * su;
    }
  }
  if (i < nc) {
    if (i % NR != NR - 1) p.v[0] += fabs(c[i]);
    if (!isfinite(c[i])) p.v[2] += 1.0;
  }
  if (i < nst) {
    const double si = -st[i];
    if (!(si > 0.0)) p.v[2] += 1.0;
    else p.v[1] += -mu * log(si) + kd * mu * si;
    p.v[0] += fabs(c[i * NR + NR - 1] - st[i]);
  }
  const int ops[3] = {0, 0, 0};
  block_reduce<3>(p, ops, out);
}

// accept the step: multipliers, bound multipliers with their own step and the safeguard
__global__ void k_accept(const double* __restrict__ xn, const double* __restrict__ sn, double* __restrict__ y,
                         const double* __restrict__ dy, double* __restrict__ zL, const double* __restrict__ dzL,
                         double* __restrict__ zU, const double* __restrict__ dzU, double* __restrict__ vU,
                         const double* __restrict__ dvU, Bnd b, double a, double az, double mu, double ksig,
                         long long nx, long long nc, long long nst) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) {
    const int k = lidx(i, nx);
    if (isfinite(b.lo[k])) {
      const double sl = xn[i] - b.lo[k];
      const double z = zL[i] + az * dzL[i];
      zL[i] = fmax(fmin(z, ksig * mu / sl), mu / (ksig * sl));
    }
    if (isfinite(b.hi[k])) {
      const double su = b.hi[k] - xn[i];
      const double z = zU[i] + az * dzU[i];
      zU[i] = fmax(fmin(z, ksig * mu / su), mu / (ksig * su));
    }
  }
  if (i < nc) y[i] += a * dy[i];
  if (i < nst) {
    const double si = -sn[i];
    const double v = vU[i] + az * dvU[i];
    vU[i] = fmax(fmin(v, ksig * mu / si), mu / (ksig * si));
  }
}

// bound push, multiplier initialisation and the least-squares right-hand side
__global__ void k_init_point(double* __restrict__ x, double* __restrict__ zL, double* __restrict__ zU, Bnd b,
                             double push, double frac, int warm, double mu, double zinit, long long nx) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= nx) return;
  const int k = lidx(i, nx);
  const double lo = b.lo[k], hi = b.hi[k];
  const bool hl = isfinite(lo), hu = isfinite(hi);
  double xi = x[i];
  if (hl) {
    double pl = push * fmax(1.0, fabs(lo));
    if (hu) pl = fmin(pl, frac * (hi - lo));
    xi = fmax(xi, lo + pl);
  }
  if (hu) {
    double pu = push * fmax(1.0, fabs(hi));
    if (hl) pu = fmin(pu, frac * (hi - lo));
    xi = fmin(xi, hi - pu);
  }
  x[i] = xi;
  zL[i] = hl ? (warm ? mu / (xi - lo) : zinit) : 0.0;
  zU[i] = hu ? (warm ? mu / (hi - xi) : zinit) : 0.0;
}

__global__ void k_init_slack(const double* __restrict__ c, double* __restrict__ s, double* __restrict__ vU,
                             double push, int warm, double mu, double zinit, long long nst) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= nst) return;
  const double si = fmin(c[i * NR + NR - 1], -push);
  s[i] = si;
  vU[i] = warm ? mu / (-si) : zinit;
}

// rhs of the least-squares multiplier system [[I, J^T], [J, 0]] (slack block eliminated)
__global__ void k_ls_rhs(const double* __restrict__ zL, const double* __restrict__ zU, const double* __restrict__ vU,
                         double gf, long long nx, long long nst, long long nkkt, double* __restrict__ rhs) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) rhs[kkt_of_primal(i, nx, nkkt)] = -((i == nx - 1 ? gf : 0.0) - zL[i] + zU[i]);
  if (i < nst) rhs[i * NK + NK - 1] = -vU[i];
}

__global__ void k_copy_duals(const double* __restrict__ sol, long long nc, double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nc) y[i] = sol[kkt_of_row(i)];
}

__global__ void k_fill(double* __restrict__ p, double v, long long n) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_absmax_parts(const double* __restrict__ v, long long n, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  Part<1> p;
  p.v[0] = i < n ? fabs(v[i]) : 0.0;
  if (i < n && !isfinite(v[i])) p.v[0] = INFINITY;
  const int ops[1] = {1};
  block_reduce<1>(p, ops, out);
}

// unscale x = D * xt, y = y~ (multipliers of scaled rows) * cs
__global__ void k_unscale(const double* __restrict__ xt, Scaling sc, long long nx, double* __restrict__ x) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) x[i] = xt[i] * (i == nx - 1 ? sc.Dd : sc.D[i % NV]);
}
__global__ void k_scale_x(const double* __restrict__ x, Scaling sc, long long nx, double* __restrict__ xt) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) xt[i] = x[i] / (i == nx - 1 ? sc.Dd : sc.D[i % NV]);
}
__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ b, long long n, int divide,
                      double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < n) out[i] = divide ? a[i] / b[i] : a[i] * b[i];
}
__global__ void k_rowscale(const double* __restrict__ rowmax, double gmax, long long n, double* __restrict__ cs) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < n) cs[i] = fmin(1.0, gmax / fmax(rowmax[i], 1e-300));
}

}  // namespace

// ------------------------------------------------------------------ host driver
namespace {

struct Work {
  double *xt = nullptr, *xtt = nullptr, *zL = nullptr, *zU = nullptr, *y = nullptr, *s = nullptr, *st = nullptr,
         *vU = nullptr, *c = nullptr, *ct = nullptr, *g = nullptr, *dpart = nullptr, *rhs = nullptr, *sol = nullptr,
         *dx = nullptr, *dy = nullptr, *dzL = nullptr, *dzU = nullptr, *ds = nullptr, *dvU = nullptr,
         *rowmax = nullptr, *omega = nullptr, *best = nullptr;
  std::vector<void*> all;
  ~Work() {
    for (void* p : all) (void)hipFree(p);
  }
  hipError_t alloc(double** p, long long n) {
    hipError_t e = hipMalloc((void**)p, sizeof(double) * (size_t)std::max<long long>(n, 1));
    if (e == hipSuccess) all.push_back(*p);
    return e;
  }
};

struct Filter {
  std::vector<std::pair<double, double>> pts;
  bool acceptable(double th, double ph) const {
    for (auto& p : pts)
      if (th >= p.first && ph >= p.second) return false;
    return true;
  }
};

// Ipopt's constants (Waechter & Biegler 2006, and the Ipopt defaults)
struct Consts {
  double kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5, tau_min = 0.99, kappa_sigma = 1e10, kappa_d = 1e-5;
  double s_max = 100.0, gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0, s_theta = 1.1, s_phi = 2.3;
  double eta_phi = 1e-8, gamma_alpha = 0.05, theta_max_fact = 1e4, theta_min_fact = 1e-4;
  double dw_init = 1e-4, dw_min = 1e-20, dw_max = 1e40, kw_minus = 1.0 / 3.0, kw_plus = 8.0, kw_plus_bar = 100.0;
  double dc_bar = 1e-8, kappa_c = 0.25, constr_mult_init_max = 1e3, zinit = 1.0;
};

}  // namespace

// host-side reduction of per-block partials
static int reduce_parts(Handle& h, int nblocks, int K, const int* ops, double* outv, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(h.redbuf_h, h.redbuf, sizeof(double) * nblocks * K, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int k = 0; k < K; ++k) {
    double a = ops[k] == 0 ? 0.0 : (ops[k] == 1 ? -INFINITY : INFINITY);
    for (int b = 0; b < nblocks; ++b) {
      const double v = h.redbuf_h[b * K + k];
      a = ops[k] == 0 ? a + v : (ops[k] == 1 ? fmax(a, v) : fmin(a, v));
    }
    outv[k] = a;
  }
  return ABS_OK;
}

static int absmax(Handle& h, const double* v, long long n, double* out, hipStream_t st) {
  const int nb = (int)grid_for(n, BS);
  if (nb > h.red_cap) {
    set_error("reduction buffer too small");
    return ABS_ERR_ARG;
  }
  hipLaunchKernelGGL(k_absmax_parts, dim3(nb), dim3(BS), 0, st, v, n, h.redbuf);
  const int ops[1] = {1};
  return reduce_parts(h, nb, 1, ops, out, st);
}

int kkt_solve_refined(Handle& h, const double* rhs, double* sol, bool fused_first, double* rel, hipStream_t st) {
  const long long nkk = h.nkkt - 1;
  const double* diagd = h.diagx + (h.nx - 1);
  if (!fused_first) {
    HIP_TRY(launch_solve(h, rhs, st));
    HIP_TRY(launch_schur(h, diagd, h.fdw, rhs + nkk, 2, sol, st));
  }
  double rn = 0.0;
  int rc = absmax(h, rhs, h.nkkt, &rn, st);
  if (rc) return rc;
  double* om_d = h.kden + 3 * ((long long)h.N * h.S);  // two doubles after the residual block partials
  double best_om = INFINITY, best_rel = INFINITY;
  bool have_best = false;
  for (int it = 0; it <= 10; ++it) {
    HIP_TRY(launch_residual(h, h.diagx, h.diags, h.fdw, h.fdc, sol, rhs, h.kres, om_d, st));
    double om[2];
    HIP_TRY(hipMemcpyAsync(om, om_d, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    double resn = 0.0;
    rc = absmax(h, h.kres, h.nkkt, &resn, st);  // synchronises the stream
    if (rc) return rc;
    const double omega = fmax(om[0], om[1]);
    const double relr = rn > 0.0 ? resn / rn : resn;
    if (!(omega < best_om)) {  // no further improvement: restore the best iterate
      if (have_best) HIP_TRY(hipMemcpyAsync(sol, h.kcor, sizeof(double) * h.nkkt, hipMemcpyDeviceToDevice, st));
      break;
    }
    best_om = omega;
    best_rel = relr;
    if (omega <= 1e-13 || it == 10) break;  // same stop rule as the reference solve
    HIP_TRY(hipMemcpyAsync(h.kcor, sol, sizeof(double) * h.nkkt, hipMemcpyDeviceToDevice, st));
    have_best = true;
    HIP_TRY(launch_solve(h, h.kres, st));
    HIP_TRY(launch_schur(h, diagd, h.fdw, h.kres + nkk, 2, h.kres, st));  // correction in place
    HIP_TRY(launch_axpy(sol, h.kres, 1.0, h.nkkt, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (rel) *rel = best_rel;
  return ABS_OK;
}

int ipm_solve(Handle& h, const absorber_ipm_options& o, const double* x0_dev, const double* y0_dev, double* xout,
              double* yout, absorber_ipm_result* res) {
  const auto t_start = std::chrono::steady_clock::now();
  const Consts C;
  hipStream_t st = h.stream;
  const long long nx = h.nx, nc = h.nc, nst = (long long)h.N * h.S, nkkt = h.nkkt;
  const long long nmax = std::max(nx, nc);
  const int nb = (int)grid_for(nmax, BS);
  if (nb * 9 > h.red_cap) {
    set_error("ipm_solve: problem too large for the reduction buffer");
    return ABS_ERR_ARG;
  }
  Work W;
  double** bufs_nx[] = {&W.xt, &W.xtt, &W.zL, &W.zU, &W.g, &W.dx, &W.dzL, &W.dzU};
  for (double** p : bufs_nx) HIP_TRY(W.alloc(p, nx));
  double** bufs_nc[] = {&W.y, &W.c, &W.ct, &W.dy, &W.rowmax};
  for (double** p : bufs_nc) HIP_TRY(W.alloc(p, nc));
  double** bufs_ns[] = {&W.s, &W.st, &W.vU, &W.ds, &W.dvU, &W.dpart};
  for (double** p : bufs_ns) HIP_TRY(W.alloc(p, nst));
  HIP_TRY(W.alloc(&W.rhs, nkkt));
  HIP_TRY(W.alloc(&W.sol, nkkt));
  HIP_TRY(W.alloc(&W.omega, 8));

  // ---- variable scaling from the cold-start point: x = D * xt
  const double* zc = h.x0;
  for (int k = 0; k < NV; ++k) h.sc.D[k] = zc[k] != 0.0 ? fabs(zc[k]) : 1.0;
  h.sc.Dd = zc[NV] != 0.0 ? fabs(zc[NV]) : 1.0;
  Bnd b;
  for (int k = 0; k < NV; ++k) {
    b.lo[k] = h.xL[k] / h.sc.D[k];
    b.hi[k] = h.xU[k] / h.sc.D[k];
  }
  b.lo[NV] = h.dL / h.sc.Dd;
  b.hi[NV] = h.dU / h.sc.Dd;
  const bool warm = o.warm_start && x0_dev;
  const unsigned gx = grid_for(nx, BS), gc = grid_for(nc, BS), gm = grid_for(nmax, BS);
  // ---- bound-pushed cold point and gradient-based row scaling there (A-1)
  {
    int rc = initial_point(h, W.xtt, st);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_scale_x, dim3(gx), dim3(BS), 0, st, W.xtt, h.sc, nx, W.xt);
  hipLaunchKernelGGL(k_init_point, dim3(gx), dim3(BS), 0, st, W.xt, W.zL, W.zU, b, o.bound_push, o.bound_push, 0,
                     0.0, C.zinit, nx);
  HIP_TRY(launch_rowmax(h, W.xt, 1, W.rowmax, st));
  hipLaunchKernelGGL(k_rowscale, dim3(gc), dim3(BS), 0, st, W.rowmax, o.nlp_scaling_max_gradient, nc, h.cs);
  h.sf = std::min(1.0, o.nlp_scaling_max_gradient / h.sc.Dd);
  const double gf = h.sf * h.sc.Dd;  // gradient of f~ = sf * d with respect to xt_d
  double mu = warm ? o.warm_mu_init : o.mu_init;
  if (warm) {
    hipLaunchKernelGGL(k_scale_x, dim3(gx), dim3(BS), 0, st, x0_dev, h.sc, nx, W.xt);
    hipLaunchKernelGGL(k_init_point, dim3(gx), dim3(BS), 0, st, W.xt, W.zL, W.zU, b, o.warm_bound_push,
                       o.warm_bound_push, 1, mu, C.zinit, nx);
  }
  HIP_TRY(launch_eval(h, W.xt, 1, nullptr, 0, W.c, st));
  hipLaunchKernelGGL(k_init_slack, dim3(grid_for(nst, BS)), dim3(BS), 0, st, W.c, W.s, W.vU,
                     warm ? o.warm_bound_push : o.bound_push, warm ? 1 : 0, mu, C.zinit, nst);
  hipLaunchKernelGGL(k_fill, dim3(gc), dim3(BS), 0, st, W.y, 0.0, nc);
  double rel = 0.0, max_rel = 0.0;
  int nfact = 0, ncorr_tot = 0;
  if (warm && y0_dev) {
    // multipliers of the unscaled rows -> multipliers of the scaled rows
    hipLaunchKernelGGL(k_mul, dim3(gc), dim3(BS), 0, st, y0_dev, h.cs, nc, 1, W.y);
  } else {
    // least-squares multipliers: [[I, J^T], [J, 0]] (slack block eliminated)
    HIP_TRY(launch_eval(h, W.xt, 1, W.y, 1, W.ct, st));
    hipLaunchKernelGGL(k_fill, dim3(gx), dim3(BS), 0, st, h.diagx, 0.0, nx);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(nst, BS)), dim3(BS), 0, st, h.diags, 0.0, nst);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(nkkt, BS)), dim3(BS), 0, st, W.rhs, 0.0, nkkt);
    hipLaunchKernelGGL(k_ls_rhs, dim3(grid_for(nkkt, BS)), dim3(BS), 0, st, W.zL, W.zU, W.vU, gf, nx, nst, nkkt,
                       W.rhs);
    HIP_TRY(launch_factor(h, h.diagx, h.diags, 1.0, 0.0, W.rhs, st));
    ++nfact;
    HIP_TRY(launch_schur(h, h.diagx + (nx - 1), 1.0, W.rhs + (nkkt - 1), 1, W.sol, st));
    int rc = kkt_solve_refined(h, W.rhs, W.sol, true, &rel, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy_duals, dim3(gc), dim3(BS), 0, st, W.sol, nc, W.y);
    double ymax = 0.0;
    rc = absmax(h, W.y, nc, &ymax, st);
    if (rc) return rc;
    if (!(ymax <= C.constr_mult_init_max)) hipLaunchKernelGGL(k_fill, dim3(gc), dim3(BS), 0, st, W.y, 0.0, nc);
  }
  // host copy of the scaled diameter (kept in step with the device copy)
  double xd = 0.0;
  HIP_TRY(hipMemcpyAsync(&xd, W.xt + (nx - 1), sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // ---- filter bounds from theta(x0)
  const int ls_ops[3] = {0, 0, 0};
  double lsv[3];
  hipLaunchKernelGGL(k_ls_parts, dim3(gm), dim3(BS), 0, st, W.xt, W.s, W.c, b, 0.0, C.kappa_d, nx, nc, nst,
                     h.redbuf);
  {
    int rc = reduce_parts(h, gm, 3, ls_ops, lsv, st);
    if (rc) return rc;
  }
  const double theta0 = lsv[0];
  const double theta_max = C.theta_max_fact * std::max(1.0, theta0);
  const double theta_min = C.theta_min_fact * std::max(1.0, theta0);
  Filter filt;
  double dw_last = 0.0;
  double tau = std::max(C.tau_min, 1.0 - mu);
  int status = ABS_ERR_MAXITER, it = 0;
  double E0 = INFINITY, inf_pr = 0, inf_du = 0, compl0 = 0;
  const double n_mult = (double)nc + 0.0;
  // counts of bound multipliers (per-local pattern times the stages, plus d)
  long long nbL = 0, nbU = 0;
  for (int k = 0; k < NV; ++k) {
    nbL += std::isfinite(b.lo[k]) ? nst : 0;
    nbU += std::isfinite(b.hi[k]) ? nst : 0;
  }
  nbL += std::isfinite(b.lo[NV]);
  nbU += std::isfinite(b.hi[NV]);
  const double n_all = n_mult + (double)(nbL + nbU + nst);
  const double n_b = (double)(nbL + nbU + nst);
  const int opt_ops[9] = {1, 1, 1, 1, 2, 1, 0, 0, 0};
  const int dir_ops[3] = {2, 2, 0};
  while (true) {
    // ---- evaluation at (x_k, y_k): residuals, Jacobian, Hessian, Lagrangian gradient
    HIP_TRY(launch_eval(h, W.xt, 1, W.y, 1, W.c, st));
    hipLaunchKernelGGL(k_lag_grad, dim3(grid_for(nst, 128)), dim3(128), 0, st, h.rec, h.jtab, W.y, h.N, h.S, W.g,
                       W.dpart);
    hipLaunchKernelGGL(k_grad_d, dim3(1), dim3(BS), 0, st, W.dpart, nst, gf, W.g + (nx - 1));
    hipLaunchKernelGGL(k_opt_parts, dim3(gm), dim3(BS), 0, st, W.xt, W.zL, W.zU, W.g, W.y, W.c, W.s, W.vU, b, nx,
                       nc, nst, h.redbuf);
    double ov[9];
    {
      int rc = reduce_parts(h, gm, 9, opt_ops, ov, st);
      if (rc) return rc;
    }
    const double dual = std::max(ov[0], ov[1]);
    const double primal = std::max(ov[2], ov[3]);
    const double sd = std::max(C.s_max, (ov[6] + ov[7]) / n_all) / C.s_max;
    const double sc = std::max(C.s_max, ov[7] / n_b) / C.s_max;
    auto Emu = [&](double m) {
      const double comp = std::max(fabs(ov[5] - m), fabs(ov[4] - m));
      return std::max(std::max(dual / sd, primal), comp / sc);
    };
    E0 = Emu(0.0);
    inf_pr = primal;
    inf_du = dual;
    compl0 = std::max(fabs(ov[4]), fabs(ov[5]));
    if (ov[8] > 0 || !std::isfinite(E0)) {
      status = ABS_ERR_NAN;
      break;
    }
    if (E0 <= o.tol) {
      status = ABS_OK;
      break;
    }
    if (it >= o.max_iter) {
      status = ABS_ERR_MAXITER;
      break;
    }
    // ---- A-3: monotone barrier update (repeated while the barrier problem is solved)
    while (Emu(mu) <= C.kappa_eps * mu) {
      mu = std::max(o.tol / 10.0, std::min(C.kappa_mu * mu, pow(mu, C.theta_mu)));
      tau = std::max(C.tau_min, 1.0 - mu);
      filt.pts.clear();
    }
    // ---- A-4: search direction with inertia correction
    hipLaunchKernelGGL(k_sigma, dim3(gm), dim3(BS), 0, st, W.xt, W.zL, W.zU, W.s, W.vU, b, nx, nst, h.diagx,
                       h.diags);
    double dw = 0.0, dc = 0.0;
    int ncorr = 0;
    bool ok = false;
    while (true) {
      hipLaunchKernelGGL(k_rhs, dim3(gm), dim3(BS), 0, st, W.xt, W.g, W.y, W.c, W.s, h.diags, b, mu, C.kappa_d, gf,
                         dw, nx, nc, nst, nkkt, W.rhs);
      HIP_TRY(launch_factor(h, h.diagx, h.diags, dw, dc, W.rhs, st));
      ++nfact;
      HIP_TRY(launch_schur(h, h.diagx + (nx - 1), dw, W.rhs + (nkkt - 1), 1, W.sol, st));
      HIP_TRY(hipMemcpyAsync(h.scal_h, h.scal, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      const DevScalars& D = *h.scal_h;
      if (D.npos == nx && D.nneg == nc && D.nzero == 0) {
        if (dw > 0.0) dw_last = dw;
        ok = true;
        break;
      }
      ++ncorr;
      if (D.nzero > 0) dc = C.dc_bar * pow(mu, C.kappa_c);
      if (dw == 0.0) dw = dw_last == 0.0 ? C.dw_init : std::max(C.dw_min, C.kw_minus * dw_last);
      else dw = (dw_last == 0.0 ? C.kw_plus_bar : C.kw_plus) * dw;
      if (dw > C.dw_max) break;
    }
    if (!ok) {
      status = ABS_ERR_INERTIA;
      break;
    }
    ncorr_tot += ncorr;
    {
      int rc = kkt_solve_refined(h, W.rhs, W.sol, true, &rel, st);
      if (rc) return rc;
      max_rel = std::max(max_rel, rel);
    }
    // ---- A-5: step pieces and fraction to the boundary
    hipLaunchKernelGGL(k_direction, dim3(gm), dim3(BS), 0, st, W.xt, W.zL, W.zU, W.y, W.s, W.vU, h.diags, W.sol, b,
                       mu, C.kappa_d, gf, dw, tau, nx, nc, nst, nkkt, W.dx, W.dy, W.dzL, W.dzU, W.ds, W.dvU,
                       h.redbuf);
    double dv[3];
    {
      int rc = reduce_parts(h, gm, 3, dir_ops, dv, st);
      if (rc) return rc;
    }
    double dxd = 0.0;
    HIP_TRY(hipMemcpyAsync(&dxd, W.dx + (nx - 1), sizeof(double), hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_ls_parts, dim3(gm), dim3(BS), 0, st, W.xt, W.s, W.c, b, mu, C.kappa_d, nx, nc, nst,
                       h.redbuf);
    {
      int rc = reduce_parts(h, gm, 3, ls_ops, lsv, st);
      if (rc) return rc;
    }
    const double alpha_max = dv[0], alpha_z = dv[1], gdx = dv[2];
    const double th = lsv[0];
    const double phi = h.sf * h.sc.Dd * xd + lsv[1];
    double amin;
    if (gdx < 0 && th <= theta_min)
      amin = C.gamma_alpha * std::min({C.gamma_theta, C.gamma_phi * th / (-gdx),
                                       C.delta * pow(th, C.s_theta) / pow(-gdx, C.s_phi)});
    else if (gdx < 0)
      amin = C.gamma_alpha * std::min(C.gamma_theta, C.gamma_phi * th / (-gdx));
    else
      amin = C.gamma_alpha * C.gamma_theta;
    double alpha = alpha_max;
    bool accepted = false, ftype = false;
    int nls = 0;
    while (true) {
      hipLaunchKernelGGL(k_trial, dim3(gx), dim3(BS), 0, st, W.xt, W.dx, W.s, W.ds, alpha, nx, nst, W.xtt, W.st);
      HIP_TRY(launch_eval(h, W.xtt, 1, nullptr, 0, W.ct, st));
      hipLaunchKernelGGL(k_ls_parts, dim3(gm), dim3(BS), 0, st, W.xtt, W.st, W.ct, b, mu, C.kappa_d, nx, nc, nst,
                         h.redbuf);
      double tv[3];
      {
        int rc = reduce_parts(h, gm, 3, ls_ops, tv, st);
        if (rc) return rc;
      }
      ++nls;
      const double tht = tv[0];
      const double phit = tv[2] > 0 ? INFINITY : h.sf * h.sc.Dd * (xd + alpha * dxd) + tv[1];
      bool okt = std::isfinite(phit) && std::isfinite(tht) && tht < theta_max && filt.acceptable(tht, phit);
      if (okt) {
        const double ma = alpha * gdx;
        const bool switching =
            ma < 0 && pow(-ma, C.s_phi) * pow(alpha, 1 - C.s_phi) > C.delta * pow(th, C.s_theta);
        if (th <= theta_min && switching) {
          if (phit <= phi + C.eta_phi * ma) {
            accepted = true;
            ftype = true;
          }
        } else if (tht <= (1 - C.gamma_theta) * th || phit <= phi - C.gamma_phi * th) {
          accepted = true;
          ftype = false;
        }
      }
      if (accepted) break;
      alpha *= 0.5;
      if (alpha < amin) break;
    }
    if (!accepted) {
      status = ABS_ERR_LS;
      break;
    }
    if (!ftype) filt.pts.push_back({(1 - C.gamma_theta) * th, phi - C.gamma_phi * th});
    hipLaunchKernelGGL(k_accept, dim3(gm), dim3(BS), 0, st, W.xtt, W.st, W.y, W.dy, W.zL, W.dzL, W.zU, W.dzU, W.vU,
                       W.dvU, b, alpha, alpha_z, mu, C.kappa_sigma, nx, nc, nst);
    std::swap(W.xt, W.xtt);
    std::swap(W.s, W.st);
    xd = xd + alpha * dxd;
    ++it;
    if (o.print_level > 0)
      fprintf(stderr, "it %4d mu %9.2e th %9.2e a %9.2e az %9.2e ls %2d dw %8.1e d %.10f E0 %9.2e res %8.1e\n", it,
              mu, th, alpha, alpha_z, nls, dw, xd * h.sc.Dd, E0, rel);
    if (fabs(xd) > 1e20) {
      status = ABS_ERR_DIVERGE;
      break;
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (xout) hipLaunchKernelGGL(k_unscale, dim3(gx), dim3(BS), 0, st, W.xt, h.sc, nx, xout);
  if (yout) hipLaunchKernelGGL(k_mul, dim3(gc), dim3(BS), 0, st, W.y, h.cs, nc, 0, yout);
  HIP_TRY(hipStreamSynchronize(st));
  if (res) {
    res->status = status;
    res->iterations = it;
    res->E0 = E0;
    res->inf_pr = inf_pr;
    res->inf_du = inf_du;
    res->compl_ = compl0;
    res->d = xd * h.sc.Dd;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    res->n_inertia_corrections = ncorr_tot;
    res->n_factorizations = nfact;
    res->max_lin_resid = max_rel;
  }
  return status;
}

}  // namespace absorber

using namespace absorber;

extern "C" {

void absorber_ipm_default_options(absorber_ipm_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_iter = 500;
  o->warm_start = 0;
  o->mu_init = 0.1;
  o->warm_mu_init = 1e-6;
  o->bound_push = 1e-2;
  o->warm_bound_push = 1e-8;
  o->nlp_scaling_max_gradient = 100.0;
  o->print_level = 0;
  o->use_graph = 0;
}

int absorber_ipm_solve(absorber_t* H, const absorber_ipm_options* opts, const double* x0_dev,
                       const double* lambda0_dev, double* x_out_dev, double* lambda_out_dev,
                       absorber_ipm_result* result) {
  if (!H) {
    set_error("absorber_ipm_solve: bad argument");
    return ABS_ERR_ARG;
  }
  absorber_ipm_options o;
  if (opts) o = *opts;
  else absorber_ipm_default_options(&o);
  if (!(o.tol > 0) || o.max_iter < 0) {
    set_error("absorber_ipm_solve: bad options");
    return ABS_ERR_ARG;
  }
  return ipm_solve(H->h, o, x0_dev, lambda0_dev, x_out_dev, lambda_out_dev, result);
}

int absorber_kkt_solve(absorber_t* H, const double* rhs_dev, double* sol_dev, double* rel_resid_host, void* stream) {
  if (!H || !rhs_dev || !sol_dev) {
    set_error("absorber_kkt_solve: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  if (!h.factored) {
    set_error("absorber_kkt_solve: no factorisation (call absorber_kkt_factor first)");
    return ABS_ERR_STATE;
  }
  double rel = 0.0;
  const int rc = kkt_solve_refined(h, rhs_dev, sol_dev, false, &rel, (hipStream_t)stream);
  if (rc) return rc;
  if (rel_resid_host) *rel_resid_host = rel;
  return ABS_OK;
}

}  // extern "C"
