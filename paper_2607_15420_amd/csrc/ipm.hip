// Filter line-search primal-dual interior-point method (the algorithm MadNLP
// implements, Waechter & Biegler 2006) for problem (10), run in lockstep over
// the P independent problems a handle holds (P = 1 for a single problem).
// Every vector operation, reduction, evaluation and linear solve is one launch
// over all problems; each problem keeps its own barrier parameter, filter,
// step sizes, regularisation and convergence state.  Those scalars live on the
// host, which runs the per-problem control flow (barrier update, inertia
// correction, filter and step acceptance), and reach the kernels through a
// small per-problem array on the device.
//
// Work units: element-wise kernels run over segments, at most SEG consecutive
// stages of one problem per 256-thread block (the block covers their primal,
// row and stage entries, and the problem's first segment also its d), so each
// block's partial reductions belong to one problem; a second launch reduces
// the partials of every problem in a fixed order.
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
static_assert(NR * SEG < BS, "a segment's rows and the d entry must fit one block");
inline unsigned grid_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// per-problem scalars read by the kernels
struct PS {
  double mu, tau, alpha, alpha_z;
  int active;  // still iterating
  int search;  // in the line search: the trial point is (re)written
  int accept;  // the trial point is accepted in this iteration
  int zero_y;  // drop the least-squares multiplier estimate
  int write;   // write this problem's final iterate to the caller's vectors
  int pad;
};

// scaled bounds per stage-local index (0-20) and d (21)
struct Bnd {
  double lo[NV + 1], hi[NV + 1];
};

// The scaled objective f~ = sf sum_k (c_k theta_k + a_k theta_k^-4), theta_k =
// D_d xt_k: the design cost and the expected operating cost of eq. (8a) (a = 0
// without it).  g[k] = sf D_d c_k is the gradient of the linear part; a holds
// a_k per design entry (problem-major), null when there is no operating cost.
struct Obj {
  double g[MAX_NPAR], c[MAX_NPAR];
  const double* a;
  double sf, Dd;
  int npar;
};
// gradient with respect to design entry i (0 for a stage entry) at its value xi
__device__ __forceinline__ double obj_g(const Obj& o, long long i, long long nxs, double xi) {
  if (i < nxs) return 0.0;
  const long long j = i - nxs;
  const double g = o.g[j % o.npar];
  if (!o.a) return g;
  const double th = o.Dd * xi, t2 = th * th;
  return g - o.sf * o.Dd * 4.0 * o.a[j] / (t2 * t2 * th);
}
// curvature of the operating cost at design entry i (0 without it)
__device__ __forceinline__ double obj_h(const Obj& o, long long i, long long nxs, double xi) {
  if (i < nxs || !o.a) return 0.0;
  const double th = o.Dd * xi, t2 = th * th;
  return o.sf * o.Dd * o.Dd * 20.0 * o.a[i - nxs] / (t2 * t2 * t2);
}
// the operating-cost part of f~ contributed by design entry i
__device__ __forceinline__ double obj_fnl(const Obj& o, long long i, long long nxs, double xi) {
  if (i < nxs || !o.a) return 0.0;
  const double th = o.Dd * xi, t2 = th * th;
  return o.sf * o.a[i - nxs] / (t2 * t2);
}

__device__ __forceinline__ int lidx(long long i, long long nxs) { return i >= nxs ? NV : (int)(i % NV); }

// primal index -> KKT index
__device__ __forceinline__ long long kkt_of_primal(long long i, long long nxs, long long nks) {
  return i >= nxs ? nks + (i - nxs) : (i / NV) * NK + (i % NV);
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
template <int K>
struct Ops {
  int op[K];  // 0 sum, 1 max, 2 min
};


// block reduction of K values in a fixed order (a DPP tree inside each wave,
// then across the BS / 64 waves); per-block partials out[blockIdx.x * K + k]
template <int K>
__device__ void block_reduce(Part<K> p, const Ops<K>& ops, double* out) {
  __shared__ double sm[K][BS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) p.v[k] = wave_reduce(ops.op[k], p.v[k]);
  if (lane == 63)
    for (int k = 0; k < K; ++k) sm[k][wv] = p.v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) {
      double a = sm[k][0];
      for (int i = 1; i < BS / 64; ++i) a = red_op(ops.op[k], a, sm[k][i]);
      out[blockIdx.x * K + k] = a;
    }
}

// per-problem reduction of segment partials: one block of RS threads per
// problem; thread i takes segments i, i + RS, ... (four at a time, their loads
// in flight together), then a fixed shuffle tree within each wave and across
// the waves.  The order depends only on the segment count: deterministic.
constexpr int RS = 1024;
template <int K>
__global__ __launch_bounds__(RS) void k_seg_reduce(const double* __restrict__ parts,
                                                   const int* __restrict__ pseg, Ops<K> ops,
                                                   double* __restrict__ out) {
  __shared__ double sm[K][RS / 64];
  const int p = blockIdx.x;
  double acc[K];
  for (int k = 0; k < K; ++k) acc[k] = ops.op[k] == 0 ? 0.0 : (ops.op[k] == 1 ? -INFINITY : INFINITY);
  const int b1 = pseg[p + 1];
  int b = pseg[p] + (int)threadIdx.x;
  for (; b + 3 * RS < b1; b += 4 * RS) {
    double q[4][K];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) q[j][k] = parts[(long long)(b + j * RS) * K + k];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = red_op(ops.op[k], acc[k], q[j][k]);
  }
  for (; b < b1; b += RS)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = red_op(ops.op[k], acc[k], parts[(long long)b * K + k]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = red_op(ops.op[k], acc[k], __shfl_down(acc[k], off, 64));
  if (lane == 0)
    for (int k = 0; k < K; ++k) sm[k][wv] = acc[k];
  __syncthreads();
  if (wv == 0) {
    // the K trees side by side, so that their shuffle latencies overlap
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      v[k] = lane < RS / 64 ? sm[k][lane] : (ops.op[k] == 0 ? 0.0 : (ops.op[k] == 1 ? -INFINITY : INFINITY));
#pragma unroll
    for (int off = RS / 128; off > 0; off >>= 1)
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = red_op(ops.op[k], v[k], __shfl_down(v[k], off, 64));
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < K; ++k) out[p * K + k] = v[k];
  }
}

// the entries of one segment: thread tid owns primal entry NV t0 + tid (tid <
// NV ns), row entry NR t0 + tid (tid < NR ns), stage t0 + tid (tid < ns), and
// the last nd threads of the problem's first segment own its nd design
// entries (Seg::first holds nd there, 0 elsewhere)
struct SegView {
  long long t0;
  int ns, p, tid, nd;
  bool owns_d;
  __device__ SegView(const Seg* seg) {
    const Seg s = seg[blockIdx.x];
    t0 = s.t0;
    ns = s.t1 - s.t0;
    p = s.p;
    tid = threadIdx.x;
    nd = s.first;
    owns_d = tid >= BS - nd;
  }
  // primal entry of this thread (or -1)
  __device__ long long xi(long long nxs) const {
    if (tid < NV * ns) return NV * t0 + tid;
    if (owns_d) return nxs + (long long)p * nd + (tid - (BS - nd));
    return -1;
  }
  __device__ long long ci() const { return tid < NR * ns ? NR * t0 + tid : -1; }
  __device__ long long ti() const { return tid < ns ? t0 + tid : -1; }
};
// Lagrangian gradient J^T y of the stage variables (the objective's only
// term, on d, is added in k_grad_d).  One block per IPM segment stages the
// segment's records and multipliers, with one neighbour on each side, in LDS;
// one thread per (stage, variable) walks that variable's term list (J entries
// of its stage and of both neighbours times the rows' multipliers).
// dpart[g] = sum over segment g of b_t y_hyd(t) (the d column of J^T y).
constexpr int GBS = 256;  // >= NV * SEG threads
__global__ __launch_bounds__(GBS) void k_lag_grad(const double* __restrict__ rec, const int* __restrict__ gtab,
                                                   int gtab_n, const double* __restrict__ y,
                                                   const Seg* __restrict__ segs, const StageInfo* __restrict__ sinfo,
                                                   long long nst, int jd, double* __restrict__ g,
                                                   double* __restrict__ dpart) {
  __shared__ double cf[(SEG + 2) * REC];
  __shared__ double sy[(SEG + 2) * NR];
  __shared__ int tab[RT_MAX];
  __shared__ double dsum[SEG];
  const int tid = threadIdx.x;
  const Seg sg = segs[blockIdx.x];
  const long long t0 = sg.t0;
  const int ns = sg.t1 - sg.t0;
  const long long la = t0 > 0 ? t0 - 1 : 0, lb = sg.t1 + 1 < nst ? sg.t1 + 1 : nst;
  const int s0 = (int)(la - (t0 - 1));  // LDS slot of stage la (slot s holds stage t0 - 1 + s)
  const int ncf = (int)(lb - la) * REC, nsy = (int)(lb - la) * NR;
  LdsStage<GBS, (SEG + 2) * REC, double> scf;
  LdsStage<GBS, (SEG + 2) * NR, double> ssy;
  LdsStage<GBS, RT_MAX, int> stb;
  scf.load(rec + la * REC, ncf, tid);
  ssy.load(y + la * NR, nsy, tid);
  stb.load(gtab, gtab_n, tid);
  const int k = tid / SEG, ls = tid - k * SEG;
  const bool mine = k < NV && ls < ns;
  const StageInfo si = sinfo[t0 + min(ls, ns - 1)];  // loaded before the LDS writes as well
  scf.store(cf + s0 * REC, ncf, tid);
  ssy.store(sy + s0 * NR, nsy, tid);
  stb.store(tab, gtab_n, tid);
  __syncthreads();
  if (mine) {
    const long long t = t0 + ls;
    const bool has_dn = si.n > 0, has_up = si.n < si.N - 1;
    const int s = ls + 1;
    const int cbase = s * REC - RT_COFF, ybase = s * NR - RT_XOFF;
    const int* tl = tab + NV + 1;
    double a = 0.0;
    for (int q = tab[k]; q < tab[k + 1]; ++q) {
      const int c = tl[2 * q], yc = tl[2 * q + 1];
      const bool ok = !(((yc & RT_NBDN) && !has_dn) || ((yc & RT_NBUP) && !has_up));
      const double pr = cf[cbase + c] * sy[ybase + (yc & (RT_XDTERM - 1))];
      a += ok ? pr : 0.0;
    }
    g[t * NV + k] = a;
    if (k == 0) dsum[ls] = cf[s * REC + jd] * sy[s * NR + NR - 1];
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0;
    for (int l = 0; l < ns; ++l) a += dsum[l];  // fixed order
    dpart[blockIdx.x] = a;
  }
}

// g_d = sf * D_d + the problem's hydraulic-row terms (one block per problem,
// fixed order over its segments)
__global__ void k_grad_d(const double* __restrict__ dpart, const int* __restrict__ pseg, Obj ob,
                         const double* __restrict__ x, long long nxs, double* __restrict__ g) {
  const int pd = blockIdx.x;
  const double gf = obj_g(ob, nxs + pd, nxs, x[nxs + pd]);
  __shared__ double sm[BS];
  const int p = blockIdx.x;
  double a = 0.0;
  for (int i = pseg[p] + threadIdx.x; i < pseg[p + 1]; i += BS) a += dpart[i];
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[nxs + p] = gf + sm[0];
}

// the design entries of J^T y for npar > 1 (one 1024-thread block per problem):
// g_k = the objective's gradient + the hydraulic rows of section k, summed in a
// fixed order (thread i takes stages i, i + DGS, ...; a shuffle tree in each wave
// and across the waves)
constexpr int DGS = 1024;
__global__ __launch_bounds__(DGS) void k_grad_design(const double* __restrict__ rec, const double* __restrict__ y,
                                                     const long long* __restrict__ pstage,
                                                     const StageInfo* __restrict__ sinfo, int jd, Obj ob,
                                                     const double* __restrict__ x, long long nxs,
                                                     double* __restrict__ g) {
  __shared__ double sm[MAX_NPAR][DGS / 64];
  const int pb = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double a[MAX_NPAR] = {0, 0, 0, 0};
  for (long long t = pstage[pb] + threadIdx.x; t < pstage[pb + 1]; t += DGS) {
    const StageInfo si = sinfo[t];
    const int k = section_of(si.n, si.N, ob.npar);
    const double v = rec[t * REC + jd] * y[t * NR + NR - 1];
#pragma unroll
    for (int q = 0; q < MAX_NPAR; ++q) a[q] += q == k ? v : 0.0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < MAX_NPAR; ++q) a[q] += __shfl_down(a[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < MAX_NPAR; ++q) sm[q][wv] = a[q];
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int q = 0; q < MAX_NPAR; ++q) {
    a[q] = lane < DGS / 64 ? sm[q][lane] : 0.0;
#pragma unroll
    for (int off = DGS / 128; off > 0; off >>= 1) a[q] += __shfl_down(a[q], off, 64);
  }
#pragma unroll
  for (int q = 0; q < MAX_NPAR; ++q)
    if (lane == 0 && q < ob.npar) {
      const long long i = nxs + (long long)pb * ob.npar + q;
      g[i] = obj_g(ob, i, nxs, x[i]) + a[q];
    }
}

// ---- optimality-error partials per segment
// 0 max|g - zL + zU|, 1 max|vU - y_hyd|, 2 max|cE|, 3 max|c_hyd - s|, 4 min compl product,
// 5 max compl product, 6 sum|y|, 7 sum|z| (zL, zU, vU), 8 nonfinite count
__global__ void k_opt_parts(const Seg* __restrict__ seg, const double* __restrict__ x,
                            const double* __restrict__ zL, const double* __restrict__ zU,
                            const double* __restrict__ g, const double* __restrict__ y, const double* __restrict__ c,
                            const double* __restrict__ s, const double* __restrict__ vU, Bnd b, long long nxs,
                            double* __restrict__ out) {
  const SegView V(seg);
  Part<9> p;
  p.v[0] = p.v[1] = p.v[2] = p.v[3] = 0.0;
  p.v[4] = INFINITY;
  p.v[5] = -INFINITY;
  p.v[6] = p.v[7] = p.v[8] = 0.0;
  const long long i = V.xi(nxs);
  if (i >= 0) {
    const int k = lidx(i, nxs);
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
  const long long j = V.ci();
  if (j >= 0) {
    const double cj = c[j];
    if (!isfinite(cj)) p.v[8] += 1.0;
    p.v[6] += fabs(y[j]);
    if (j % NR != NR - 1) p.v[2] = fabs(cj);
  }
  const long long t = V.ti();
  if (t >= 0) {
    p.v[1] = fabs(vU[t] - y[t * NR + NR - 1]);
    p.v[3] = fabs(c[t * NR + NR - 1] - s[t]);
    const double pr = -s[t] * vU[t];
    p.v[4] = fmin(p.v[4], pr);
    p.v[5] = fmax(p.v[5], pr);
    p.v[7] += fabs(vU[t]);
  }
  block_reduce<9>(p, Ops<9>{{1, 1, 1, 1, 2, 1, 0, 0, 0}}, out);
}

// ---- barrier diagonals
// (the design entries also carry the operating cost's curvature)
__global__ void k_sigma(const double* __restrict__ x, const double* __restrict__ zL, const double* __restrict__ zU,
                        const double* __restrict__ s, const double* __restrict__ vU, Bnd b, Obj ob, long long nx,
                        long long nxs, long long nst, double* __restrict__ dx, double* __restrict__ ds) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) {
    const int k = lidx(i, nxs);
    double sg = 0.0;
    if (isfinite(b.lo[k])) sg += zL[i] / (x[i] - b.lo[k]);
    if (isfinite(b.hi[k])) sg += zU[i] / (b.hi[k] - x[i]);
    dx[i] = sg + obj_h(ob, i, nxs, x[i]);
  }
  if (i < nst) ds[i] = vU[i] / (-s[i]);
}

// barrier gradient of a primal entry (without J^T y)
// gf: the objective's gradient at this entry (0 for a stage entry)
__device__ __forceinline__ double barrier_grad(double xi, int k, const Bnd& b, double mu, double kd, double gf) {
  double v = (k == NV) ? gf : 0.0;
  const bool hl = isfinite(b.lo[k]), hu = isfinite(b.hi[k]);
  if (hl) v -= mu / (xi - b.lo[k]);
  if (hu) v += mu / (b.hi[k] - xi);
  if (hl && !hu) v += kd * mu;
  if (hu && !hl) v -= kd * mu;
  return v;
}

// ---- right-hand side of the slack-reduced primal-dual system (zero for
// problems no longer iterating)
__global__ void k_rhs(const Seg* __restrict__ seg, const PS* __restrict__ ps, const double* __restrict__ dwv,
                      const double* __restrict__ x, const double* __restrict__ g, const double* __restrict__ y,
                      const double* __restrict__ c, const double* __restrict__ s, const double* __restrict__ ds,
                      Bnd b, double kd, Obj ob, long long nxs, long long nks, double* __restrict__ rhs) {
  const SegView V(seg);
  const PS q = ps[V.p];
  const double mu = q.mu, dw = dwv[V.p];
  const long long i = V.xi(nxs);
  if (i >= 0) {
    const int k = lidx(i, nxs);
    // g holds grad f~ + J~^T y; remove grad f~ for d since barrier_grad adds it
    const double gf = obj_g(ob, i, nxs, x[i]);
    const double gl = (k == NV) ? g[i] - gf : g[i];
    rhs[kkt_of_primal(i, nxs, nks)] = q.active ? -(gl + barrier_grad(x[i], k, b, mu, kd, gf)) : 0.0;
  }
  const long long j = V.ci();
  if (j >= 0 && j % NR != NR - 1) rhs[kkt_of_row(j)] = q.active ? -c[j] : 0.0;
  const long long t = V.ti();
  if (t >= 0) {
    const double yh = y[t * NR + NR - 1];
    const double rs = mu / (-s[t]) - kd * mu - yh;
    const double rd = c[t * NR + NR - 1] - s[t];
    rhs[t * NK + NK - 1] = q.active ? -rd - rs / (ds[t] + dw) : 0.0;
  }
}

// ---- search direction pieces, fraction to the boundary and grad(phi)^T dx
// segment partials: 0 min alpha primal, 1 min alpha dual, 2 sum grad phi . d
__global__ void k_direction(const Seg* __restrict__ seg, const PS* __restrict__ ps, const double* __restrict__ dwv,
                            const double* __restrict__ x, const double* __restrict__ zL,
                            const double* __restrict__ zU, const double* __restrict__ y, const double* __restrict__ s,
                            const double* __restrict__ vU, const double* __restrict__ dss,
                            const double* __restrict__ sol, Bnd b, double kd, Obj ob, long long nxs, long long nks,
                            double* __restrict__ dx, double* __restrict__ dy, double* __restrict__ dzL,
                            double* __restrict__ dzU, double* __restrict__ dsl, double* __restrict__ dvU,
                            double* __restrict__ out) {
  const SegView V(seg);
  const PS q = ps[V.p];
  const double mu = q.mu, tau = q.tau, dw = dwv[V.p];
  Part<4> p;
  p.v[0] = 1.0;
  p.v[1] = 1.0;
  p.v[2] = 0.0;
  p.v[3] = 0.0;
  const long long i = V.xi(nxs);
  if (i >= 0) {
    const int k = lidx(i, nxs);
    const double d = sol[kkt_of_primal(i, nxs, nks)];
    dx[i] = d;
    // the problem's design-cost step sum_k c_k d theta_k (its owner threads only)
    if (i >= nxs) p.v[3] = ob.c[(i - nxs) % ob.npar] * d;
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
    p.v[2] += barrier_grad(xi, k, b, mu, kd, obj_g(ob, i, nxs, xi)) * d;
  }
  const long long j = V.ci();
  if (j >= 0) dy[j] = sol[kkt_of_row(j)];
  const long long t = V.ti();
  if (t >= 0) {
    const double si = -s[t];  // distance of the slack to its bound 0
    const double yh = y[t * NR + NR - 1];
    const double rs = mu / si - kd * mu - yh;
    const double dyh = sol[t * NK + NK - 1];
    const double d = (dyh - rs) / (dss[t] + dw);
    dsl[t] = d;
    const double dv = mu / si - vU[t] + vU[t] / si * d;
    dvU[t] = dv;
    if (d > 0.0) p.v[0] = fmin(p.v[0], tau * si / d);
    if (dv < 0.0) p.v[1] = fmin(p.v[1], -tau * vU[t] / dv);
    p.v[2] += (mu / si - kd * mu) * d;
  }
  block_reduce<4>(p, Ops<4>{{2, 2, 0, 0}}, out);
}

// trial point of the problems in the line search
__global__ void k_trial(const Seg* __restrict__ seg, const PS* __restrict__ ps, const double* __restrict__ x,
                        const double* __restrict__ dx, const double* __restrict__ s, const double* __restrict__ dsl,
                        long long nxs, double* __restrict__ xt, double* __restrict__ st) {
  const SegView V(seg);
  const PS q = ps[V.p];
  if (!q.search) return;
  const long long i = V.xi(nxs);
  if (i >= 0) xt[i] = x[i] + q.alpha * dx[i];
  const long long t = V.ti();
  if (t >= 0) st[t] = s[t] + q.alpha * dsl[t];
}

// first trial point of every active problem, at the step alpha_max that the
// direction reduction left on the device (aout[4 p]); queued before the host
// has read that reduction
__global__ void k_trial_first(const Seg* __restrict__ seg, const PS* __restrict__ ps,
                              const double* __restrict__ aout, const double* __restrict__ x,
                              const double* __restrict__ dx, const double* __restrict__ s,
                              const double* __restrict__ dsl, long long nxs, double* __restrict__ xt,
                              double* __restrict__ st) {
  const SegView V(seg);
  if (!ps[V.p].active) return;
  const double a = aout[4 * V.p];
  const long long i = V.xi(nxs);
  if (i >= 0) xt[i] = x[i] + a * dx[i];
  const long long t = V.ti();
  if (t >= 0) st[t] = s[t] + a * dsl[t];
}

// line-search partials at a point: 0 theta (1-norm), 1 barrier sum, 2 infeasible count
__global__ void k_ls_parts(const Seg* __restrict__ seg, const PS* __restrict__ ps, const double* __restrict__ xt,
                           const double* __restrict__ st, const double* __restrict__ c, Bnd b, double kd, Obj ob,
                           long long nxs, double* __restrict__ out) {
  const SegView V(seg);
  const double mu = ps[V.p].mu;
  Part<3> p;
  p.v[0] = p.v[1] = p.v[2] = 0.0;
  const long long i = V.xi(nxs);
  if (i >= 0) {
    const int k = lidx(i, nxs);
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
    if (i >= nxs && xt[i] > 0.0) p.v[1] += obj_fnl(ob, i, nxs, xt[i]);  // operating cost at this point
  }
  const long long j = V.ci();
  if (j >= 0) {
    if (j % NR != NR - 1) p.v[0] += fabs(c[j]);
    if (!isfinite(c[j])) p.v[2] += 1.0;
  }
  const long long t = V.ti();
  if (t >= 0) {
    const double si = -st[t];
    if (!(si > 0.0)) p.v[2] += 1.0;
    else p.v[1] += -mu * log(si) + kd * mu * si;
    p.v[0] += fabs(c[t * NR + NR - 1] - st[t]);
  }
  block_reduce<3>(p, Ops<3>{{0, 0, 0}}, out);
}

// accept the step of the problems whose trial point passed: primal and slack
// from the trial point, multipliers, bound multipliers with their own step and
// the safeguard
__global__ void k_accept(const Seg* __restrict__ seg, const PS* __restrict__ ps, double* __restrict__ x,
                         const double* __restrict__ xn, double* __restrict__ s, const double* __restrict__ sn,
                         double* __restrict__ y, const double* __restrict__ dy, double* __restrict__ zL,
                         const double* __restrict__ dzL, double* __restrict__ zU, const double* __restrict__ dzU,
                         double* __restrict__ vU, const double* __restrict__ dvU, Bnd b, double ksig,
                         long long nxs) {
  const SegView V(seg);
  const PS q = ps[V.p];
  if (!q.accept) return;
  const double a = q.alpha, az = q.alpha_z, mu = q.mu;
  const long long i = V.xi(nxs);
  if (i >= 0) {
    const int k = lidx(i, nxs);
    const double xi = xn[i];
    x[i] = xi;
    if (isfinite(b.lo[k])) {
      const double sl = xi - b.lo[k];
      const double z = zL[i] + az * dzL[i];
      zL[i] = fmax(fmin(z, ksig * mu / sl), mu / (ksig * sl));
    }
    if (isfinite(b.hi[k])) {
      const double su = b.hi[k] - xi;
      const double z = zU[i] + az * dzU[i];
      zU[i] = fmax(fmin(z, ksig * mu / su), mu / (ksig * su));
    }
  }
  const long long j = V.ci();
  if (j >= 0) y[j] += a * dy[j];
  const long long t = V.ti();
  if (t >= 0) {
    const double snt = sn[t];
    s[t] = snt;
    const double si = -snt;
    const double v = vU[t] + az * dvU[t];
    vU[t] = fmax(fmin(v, ksig * mu / si), mu / (ksig * si));
  }
}

// bound push and multiplier initialisation
__global__ void k_init_point(double* __restrict__ x, double* __restrict__ zL, double* __restrict__ zU, Bnd b,
                             double push, double frac, int warm, double mu, double zinit, long long nx,
                             long long nxs) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= nx) return;
  const int k = lidx(i, nxs);
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
__global__ void k_ls_rhs(const double* __restrict__ x, const double* __restrict__ zL, const double* __restrict__ zU,
                         const double* __restrict__ vU, Obj ob, long long nx, long long nxs, long long nks,
                         long long nst, double* __restrict__ rhs) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) rhs[kkt_of_primal(i, nxs, nks)] = -(obj_g(ob, i, nxs, x[i]) - zL[i] + zU[i]);
  if (i < nst) rhs[i * NK + NK - 1] = -vU[i];
}

__global__ void k_copy_duals(const double* __restrict__ sol, long long nc, double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nc) y[i] = sol[kkt_of_row(i)];
}

// per-segment max |y| (least-squares multiplier check)
__global__ void k_ymax_parts(const Seg* __restrict__ seg, const double* __restrict__ y, double* __restrict__ out) {
  const SegView V(seg);
  Part<1> p;
  const long long j = V.ci();
  p.v[0] = j >= 0 ? (isfinite(y[j]) ? fabs(y[j]) : INFINITY) : 0.0;
  block_reduce<1>(p, Ops<1>{{1}}, out);
}

__global__ void k_zero_y(const Seg* __restrict__ seg, const PS* __restrict__ ps, double* __restrict__ y) {
  const SegView V(seg);
  if (!ps[V.p].zero_y) return;
  const long long j = V.ci();
  if (j >= 0) y[j] = 0.0;
}

__global__ void k_fill(double* __restrict__ p, double v, long long n) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < n) p[i] = v;
}

// final iterate of the problems flagged "write": x = D * xt and y = y~ * cs
__global__ void k_output(const Seg* __restrict__ seg, const PS* __restrict__ ps, const double* __restrict__ xt,
                         const double* __restrict__ y, const double* __restrict__ cs, Scaling sc, long long nxs,
                         double* __restrict__ xout, double* __restrict__ yout) {
  const SegView V(seg);
  if (!ps[V.p].write) return;
  const long long i = V.xi(nxs);
  if (xout && i >= 0) xout[i] = xt[i] * (i >= nxs ? sc.Dd : sc.D[i % NV]);
  const long long j = V.ci();
  if (yout && j >= 0) yout[j] = y[j] * cs[j];
}

// unscale x = D * xt, y = y~ (multipliers of scaled rows) * cs
__global__ void k_unscale(const double* __restrict__ xt, Scaling sc, long long nx, long long nxs,
                          double* __restrict__ x) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) x[i] = xt[i] * (i >= nxs ? sc.Dd : sc.D[i % NV]);
}
__global__ void k_scale_x(const double* __restrict__ x, Scaling sc, long long nx, long long nxs,
                          double* __restrict__ xt) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i < nx) xt[i] = x[i] / (i >= nxs ? sc.Dd : sc.D[i % NV]);
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
         *rowmax = nullptr;
  PS* ps = nullptr;        // device [P] (in the handle's control block)
  PS* ps_h = nullptr;      // pinned [P] (its host copy)
  double* dw_h = nullptr;  // pinned [P]
  double* dc_h = nullptr;  // pinned [P]
  int* fm_h = nullptr;     // pinned [P]
  double* dd_h = nullptr;  // pinned [P]: the d entries of a primal vector
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
  double alpha_floor = 0x1p-52;
};

// host state of one problem
struct Prob {
  double mu = 0, tau = 0, dw = 0, dc = 0, dw_last = 0, theta_max = 0, theta_min = 0;
  double E0 = INFINITY, inf_pr = 0, inf_du = 0, compl0 = 0, xd = 0, dxd = 0;
  double alpha = 0, alpha_max = 0, alpha_z = 0, gdx = 0, th = 0, phi = 0, amin = 0;
  double n_all = 0, n_b = 0, nx_p = 0, nc_p = 0;
  double max_lin = 0;  // largest relative residual of this problem's Newton-system solves
  int status = ABS_ERR_MAXITER, it = 0, ncorr = 0, nls = 0, nfac = 0;
  bool active = true, need = false, searching = false, accepted = false, ftype = false;
  Filter filt;
};

}  // namespace

// ------------------------------------------------------------------ device-resident control
// With use_graph, the per-problem decisions of an iteration (convergence test
// and barrier update, inertia correction, refinement stop, step bounds, filter
// acceptance, step acceptance) are taken on the device by one thread per
// problem, with the same arithmetic and in the same order as the host
// decisions of the host-driven loop.  Each problem moves through the phases
// of an iteration; every launch of the iteration acts on the problems in its
// phase, so the launches of one iteration can be replayed as fixed HIP graphs
// and the host only reads a compact status once per replay pass.
namespace {

constexpr int PH_IDLE = 0;    // between iterations (or finished)
constexpr int PH_FACTOR = 1;  // a factorisation trial of the inertia correction is due
constexpr int PH_RES0 = 2;    // factorised with the right inertia: first residual due
constexpr int PH_REFINE = 3;  // refinement corrections due
constexpr int PH_DIR = 4;     // solution final: step pieces and bounds due
constexpr int PH_SEARCH = 5;  // line search: the trial point at alpha is due
constexpr int PH_ACCEPT = 6;  // trial accepted: the step is due

struct DevProb {
  double mu, tau, dw, dc, dw_last, theta_max, theta_min;
  double E0, inf_pr, inf_du, compl0, xd, dxd;
  double alpha, alpha_z, gdx, th, phi, amin;
  double n_all, n_b, nx_p, nc_p, max_lin, best;
  int status, it, ncorr, nls, nfac, nfilt, nref, phase, active, ftype;
};

// device pointers of the control state (passed by value)
struct GCtl {
  DevProb* dp;
  PS* ps;
  int* pact;
  double* dwv;
  double* dcv;
  int* fmask;
  int* rmask;  // problems whose refinement correction is due
  int* cmask;  // problems whose corrected iterate is kept
  double* filt;  // [P][fcap][2]
  int fcap;
  int2* stat;  // [P] (phase, active) for the host
  absorber_ipm_log_entry* log;  // [log_np][log_cap]
  int log_np, log_cap;
  int P;
};

__device__ __forceinline__ void ctl_store(const GCtl& g, int p, const DevProb& q) {
  g.dp[p] = q;
  g.stat[p] = make_int2(q.phase, q.active);
}

__device__ __forceinline__ void ctl_stop(const GCtl& g, int p, DevProb& q, int status) {
  q.status = status;
  q.active = 0;
  q.phase = PH_IDLE;
  g.pact[p] = 0;
  g.fmask[p] = 0;
  g.rmask[p] = 0;
  g.ps[p].active = 0;
  g.ps[p].search = 0;
  g.ps[p].accept = 0;
}

// convergence test on the reduced optimality-error parts and the monotone
// barrier update; starts the inertia correction with delta_w = delta_c = 0
__global__ void k_ctl_opt(GCtl g, const double* __restrict__ ov, Consts C, double tol, int max_iter) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  if (!q.active || q.phase != PH_IDLE) return;
  const double* o = ov + 9LL * p;
  const double dual = fmax(o[0], o[1]);
  const double primal = fmax(o[2], o[3]);
  const double sd = fmax(C.s_max, (o[6] + o[7]) / q.n_all) / C.s_max;
  const double sc = fmax(C.s_max, o[7] / q.n_b) / C.s_max;
  auto Emu = [&](double m) {
    const double comp = fmax(fabs(o[5] - m), fabs(o[4] - m));
    return fmax(fmax(dual / sd, primal), comp / sc);
  };
  q.E0 = Emu(0.0);
  q.inf_pr = primal;
  q.inf_du = dual;
  q.compl0 = fmax(fabs(o[4]), fabs(o[5]));
  int stop = 1;
  if (o[8] > 0 || !isfinite(q.E0)) q.status = ABS_ERR_NAN;
  else if (q.E0 <= tol) q.status = ABS_OK;
  else if (q.it >= max_iter) q.status = ABS_ERR_MAXITER;
  else stop = 0;
  if (stop) {
    ctl_stop(g, p, q, q.status);
    ctl_store(g, p, q);
    return;
  }
  while (Emu(q.mu) <= C.kappa_eps * q.mu) {
    const double mu_new = fmax(tol / 10.0, fmin(C.kappa_mu * q.mu, pow(q.mu, C.theta_mu)));
    if (mu_new >= q.mu) break;  // already at its floor tol / 10
    q.mu = mu_new;
    q.tau = fmax(C.tau_min, 1.0 - q.mu);
    q.nfilt = 0;
  }
  q.dw = 0.0;
  q.dc = 0.0;
  q.nfac = 0;
  q.phase = PH_FACTOR;
  g.ps[p].mu = q.mu;
  g.ps[p].tau = q.tau;
  g.dwv[p] = 0.0;
  g.dcv[p] = 0.0;
  g.fmask[p] = 1;
  ctl_store(g, p, q);
}

// inertia of the last factorisation: accept it or raise delta_w (and set delta_c)
__global__ void k_ctl_inertia(GCtl g, const DevScalars* __restrict__ scal, Consts C, double dw_max) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  if (!q.active || q.phase != PH_FACTOR) return;
  ++q.nfac;
  const DevScalars D = scal[p];
  if ((double)D.npos == q.nx_p && (double)D.nneg == q.nc_p && D.nzero == 0) {
    if (q.dw > 0.0) q.dw_last = q.dw;
    q.phase = PH_RES0;
    g.fmask[p] = 0;
    ctl_store(g, p, q);
    return;
  }
  ++q.ncorr;
  if (D.nzero > 0) q.dc = C.dc_bar * pow(q.mu, C.kappa_c);
  if (q.dw == 0.0) q.dw = q.dw_last == 0.0 ? C.dw_init : fmax(C.dw_min, C.kw_minus * q.dw_last);
  else q.dw = (q.dw_last == 0.0 ? C.kw_plus_bar : C.kw_plus) * q.dw;
  if (q.dw > dw_max) {
    ctl_stop(g, p, q, ABS_ERR_INERTIA);
  } else {
    g.dwv[p] = q.dw;
    g.dcv[p] = q.dc;
    g.fmask[p] = 1;
  }
  ctl_store(g, p, q);
}

// relative residual of each problem's own rows from the per-problem maxima
__device__ __forceinline__ double rel_of(const double* pres, int p) {
  const double r = pres[2 * p], b = pres[2 * p + 1];
  return b > 0.0 ? r / b : r;
}

// first residual of the fused solution: done at the target, else refine
__global__ void k_ctl_res0(GCtl g, const double* __restrict__ pres, double target) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  if (!q.active || q.phase != PH_RES0) return;
  const double rel = rel_of(pres, p);
  q.best = INFINITY;
  q.nref = 0;
  bool done = true;
  if (rel < q.best) {  // false for a residual that is not finite
    q.best = rel;
    done = rel <= target;
  }
  if (done) {
    q.max_lin = fmax(q.max_lin, q.best);
    q.phase = PH_DIR;
    g.rmask[p] = 0;
  } else {
    q.phase = PH_REFINE;
    g.rmask[p] = 1;
  }
  g.cmask[p] = 0;
  ctl_store(g, p, q);
}

// residual of the corrected iterate: keep it if it decreased; stop at the
// target, at no decrease, or after 10 corrections
__global__ void k_ctl_refine(GCtl g, const double* __restrict__ pres, double target) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  g.cmask[p] = 0;
  if (!q.active || q.phase != PH_REFINE) return;
  const double rel = rel_of(pres, p);
  ++q.nref;
  bool done;
  if (rel < q.best) {
    q.best = rel;
    g.cmask[p] = 1;
    done = rel <= target || q.nref >= 10;
  } else {
    done = true;
  }
  if (done) {
    q.max_lin = fmax(q.max_lin, q.best);
    q.phase = PH_DIR;
    g.rmask[p] = 0;
  }
  ctl_store(g, p, q);
}

// step bounds from the direction reduction; the line search starts at alpha_max
__global__ void k_ctl_dir(GCtl g, const double* __restrict__ dv4, const double* __restrict__ lv3, Consts C,
                          double phi_d) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  if (!q.active || q.phase != PH_DIR) return;
  const double* dv = dv4 + 4LL * p;
  const double* lv = lv3 + 3LL * p;
  q.alpha = dv[0];
  q.alpha_z = dv[1];
  q.gdx = dv[2];
  q.dxd = dv[3];
  q.th = lv[0];
  q.phi = phi_d * q.xd + lv[1];
  const double th = q.th, gdx = q.gdx;
  if (gdx < 0 && th <= q.theta_min)
    q.amin = C.gamma_alpha * fmin(fmin(C.gamma_theta, C.gamma_phi * th / (-gdx)),
                                  C.delta * pow(th, C.s_theta) / pow(-gdx, C.s_phi));
  else if (gdx < 0)
    q.amin = C.gamma_alpha * fmin(C.gamma_theta, C.gamma_phi * th / (-gdx));
  else
    q.amin = C.gamma_alpha * C.gamma_theta;
  q.nls = 0;
  q.phase = PH_SEARCH;
  g.ps[p].alpha = q.alpha;
  g.ps[p].alpha_z = q.alpha_z;
  g.ps[p].search = 1;
  g.ps[p].accept = 0;
  ctl_store(g, p, q);
}

// filter acceptance of the trial point (its reduced theta, barrier sum and
// infeasibility count in tv3); backtrack by one half otherwise
__global__ void k_ctl_ls(GCtl g, const double* __restrict__ tv3, Consts C, double phi_d) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  if (!q.active || q.phase != PH_SEARCH) return;
  const double* tv = tv3 + 3LL * p;
  ++q.nls;
  const double tht = tv[0];
  const double phit = tv[2] > 0 ? INFINITY : phi_d * (q.xd + q.alpha * q.dxd) + tv[1];
  const double th = q.th, phi = q.phi;
  bool okt = isfinite(phit) && isfinite(tht) && tht < q.theta_max;
  if (okt) {
    const double* f = g.filt + 2LL * g.fcap * p;
    for (int i = 0; i < q.nfilt; ++i)
      if (tht >= f[2 * i] && phit >= f[2 * i + 1]) {
        okt = false;
        break;
      }
  }
  bool acc = false, ftype = false;
  if (okt) {
    const double ma = q.alpha * q.gdx;
    const bool switching = ma < 0 && pow(-ma, C.s_phi) * pow(q.alpha, 1 - C.s_phi) > C.delta * pow(th, C.s_theta);
    if (th <= q.theta_min && switching) {
      if (phit <= phi + C.eta_phi * ma) {
        acc = true;
        ftype = true;
      }
    } else if (tht <= (1 - C.gamma_theta) * th || phit <= phi - C.gamma_phi * th) {
      acc = true;
    }
  }
  if (acc) {
    q.ftype = ftype;
    q.phase = PH_ACCEPT;
    g.ps[p].search = 0;
    g.ps[p].accept = 1;
  } else {
    q.alpha *= 0.5;
    if (q.alpha < fmax(q.amin, C.alpha_floor)) {
      ctl_stop(g, p, q, ABS_ERR_LS);
    } else {
      g.ps[p].alpha = q.alpha;
    }
  }
  ctl_store(g, p, q);
}

// after the accepted step: filter augmentation, the diameter, the log entry
__global__ void k_ctl_accept(GCtl g, Consts C, double Dd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  DevProb q = g.dp[p];
  if (!q.active || q.phase != PH_ACCEPT) return;
  if (!q.ftype && q.nfilt < g.fcap) {
    double* f = g.filt + 2LL * g.fcap * p + 2LL * q.nfilt;
    f[0] = (1 - C.gamma_theta) * q.th;
    f[1] = q.phi - C.gamma_phi * q.th;
    ++q.nfilt;
  }
  q.xd = q.xd + q.alpha * q.dxd;
  ++q.it;
  if (p < g.log_np && q.it - 1 < g.log_cap) {
    absorber_ipm_log_entry e;
    e.iteration = q.it;
    e.n_factorizations = q.nfac;
    e.n_trials = q.nls;
    e.pad = 0;
    e.mu = q.mu;
    e.theta = q.th;
    e.alpha = q.alpha;
    e.alpha_z = q.alpha_z;
    e.delta_w = q.dw;
    e.delta_c = q.dc;
    e.d = q.xd * Dd;
    e.E0 = q.E0;
    g.log[(long long)p * g.log_cap + q.it - 1] = e;
  }
  g.ps[p].accept = 0;
  q.phase = PH_IDLE;
  if (fabs(q.xd) > 1e20) ctl_stop(g, p, q, ABS_ERR_DIVERGE);
  ctl_store(g, p, q);
}

}  // namespace
#define GTRY(expr)           \
  do {                       \
    const int rc_ = (expr);  \
    if (rc_) return rc_;     \
  } while (0)
// ------------------------------------------------------------------ graph-replayed iterations
namespace {

// G_FAC_A and G_FAC_B are G_FAC without its factorisation, which is launched
// between them (with the per-launch timing events) when the factorisation is timed
enum { G_OPT = 0, G_FAC, G_FAC_A, G_FAC_B, G_REF, G_DIR, G_LS, G_ACC, G_COUNT };

// graphs of one iteration's launches and the device control state they act on
struct GraphState {
  hipStream_t st = nullptr;  // capture and replay stream (default priority)
  hipGraphExec_t ex[G_COUNT] = {};
  bool captured = false;
  // what the captured launches depend on besides the handle's fixed buffers
  double tol = 0, dw_max = 0;
  int max_iter = -1, timed = -1, fwpe = -1, fsplit = -1, swpe = -1, ebs = -1;
  char* dev = nullptr;
  size_t dev_bytes = 0;
  DevProb* dp = nullptr;
  double* filt = nullptr;
  int2* stat = nullptr;
  int* cmask = nullptr;
  absorber_ipm_log_entry* log = nullptr;
  int fcap = 0, log_np = 0, log_cap = 0;
  int2* stat_h = nullptr;  // pinned [P]
  ~GraphState() {
    for (auto& e : ex)
      if (e) (void)hipGraphExecDestroy(e);
    if (dev) (void)hipFree(dev);
    if (stat_h) (void)hipHostFree(stat_h);
    if (st) (void)hipStreamDestroy(st);
  }
};

}  // namespace

void free_ipm_graph(Handle& h) {
  delete static_cast<GraphState*>(h.ipm_graph);
  h.ipm_graph = nullptr;
}

hipStream_t ipm_graph_stream(Handle& h) {
  if (!h.ipm_graph) h.ipm_graph = new GraphState();
  GraphState& gs = *static_cast<GraphState*>(h.ipm_graph);
  if (!gs.st && hipStreamCreateWithFlags(&gs.st, hipStreamNonBlocking) != hipSuccess) gs.st = nullptr;
  return gs.st;
}

namespace {

// record the launches of body() on st into an executable graph
template <class F>
int capture_graph(hipStream_t st, hipGraphExec_t* out, F body) {
  if (*out) {
    (void)hipGraphExecDestroy(*out);
    *out = nullptr;
  }
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  const int rc = body();
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIP_TRY(e);
  const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_TRY(ei);
  return ABS_OK;
}

// The interior-point iterations with the per-problem decisions on the device:
// each iteration replays the graphs of its phases (evaluation and convergence
// test, factorisation trial with the first residual, direction with the first
// trial point, step) and reads the problems' phases once; a problem that needs
// another factorisation trial, refinement corrections or further trial points
// is finished by replaying the graphs of those phases.  Same arithmetic and
// order of decisions as the host-driven loop.
int graph_iterations(Handle& h, const absorber_ipm_options& o, const Consts& C, const Bnd& b, const Obj& ob,
                     Work& W, std::vector<Prob>& pr, hipStream_t st, int& nfact, int& replays) {
  GraphState& gs = *static_cast<GraphState*>(h.ipm_graph);
  const int P = h.P;
  const long long nx = h.nx, nst = h.nst, nkkt = h.nkkt;
  const long long nxs = nst * NV, nks = nst * NK;
  const int nseg = h.nseg;
  const unsigned gm = grid_for(std::max(nx, h.nc), BS);
  const unsigned gp = grid_for(P, 64);
  // ---- device control state
  const int fcap = o.max_iter + 1, log_np = std::min(P, 64), log_cap = std::max(o.max_iter, 1);
  auto al = [](size_t n) { return (n + 255) / 256 * 256; };
  const size_t b_dp = al(sizeof(DevProb) * P), b_filt = al(sizeof(double) * 2 * (size_t)fcap * P),
               b_stat = al(sizeof(int2) * P), b_cm = al(sizeof(int) * P),
               b_log = al(sizeof(absorber_ipm_log_entry) * (size_t)log_np * log_cap);
  const size_t need = b_dp + b_filt + b_stat + b_cm + b_log;
  if (need > gs.dev_bytes) {
    if (gs.dev) HIP_TRY(hipFree(gs.dev));
    gs.dev = nullptr;
    gs.dev_bytes = 0;
    HIP_TRY(hipMalloc((void**)&gs.dev, need));
    gs.dev_bytes = need;
    if (gs.stat_h) HIP_TRY(hipHostFree(gs.stat_h));
    gs.stat_h = nullptr;
    HIP_TRY(hipHostMalloc((void**)&gs.stat_h, sizeof(int2) * P, 0));
    gs.captured = false;
  }
  if (!gs.stat_h) HIP_TRY(hipHostMalloc((void**)&gs.stat_h, sizeof(int2) * P, 0));
  gs.dp = reinterpret_cast<DevProb*>(gs.dev);
  gs.filt = reinterpret_cast<double*>(gs.dev + b_dp);
  gs.stat = reinterpret_cast<int2*>(gs.dev + b_dp + b_filt);
  gs.cmask = reinterpret_cast<int*>(gs.dev + b_dp + b_filt + b_stat);
  gs.log = reinterpret_cast<absorber_ipm_log_entry*>(gs.dev + b_dp + b_filt + b_stat + b_cm);
  gs.fcap = fcap;
  gs.log_np = log_np;
  gs.log_cap = log_cap;
  {
    std::vector<DevProb> dp((size_t)P);
    for (int p = 0; p < P; ++p) {
      const Prob& q = pr[(size_t)p];
      DevProb d{};
      d.mu = q.mu;
      d.tau = q.tau;
      d.theta_max = q.theta_max;
      d.theta_min = q.theta_min;
      d.E0 = q.E0;
      d.xd = q.xd;
      d.n_all = q.n_all;
      d.n_b = q.n_b;
      d.nx_p = q.nx_p;
      d.nc_p = q.nc_p;
      d.status = q.status;
      d.active = q.active ? 1 : 0;
      d.phase = PH_IDLE;
      dp[(size_t)p] = d;
    }
    HIP_TRY(hipMemcpyAsync(gs.dp, dp.data(), sizeof(DevProb) * P, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  GCtl g{gs.dp, W.ps, h.pact, h.dwv, h.dcv, h.fmask, h.rmask, gs.cmask, gs.filt, fcap, gs.stat, gs.log,
         log_np, log_cap, P};
  const double phi_d = h.sf * h.sc.Dd;
  const int timed = (h.prof & 1) ? 1 : 0;
  // ---- capture (again when the options, the launch shapes or the timing changed)
  if (o.autotune && !h.tune.done) GTRY(autotune(h, W.xt, W.y, W.c, h.diagx, h.diags, W.rhs, st));
  if (!gs.captured || gs.tol != o.tol || gs.dw_max != o.delta_w_max || gs.max_iter != o.max_iter ||
      gs.timed != timed || gs.fwpe != h.tune.factor_wpe || gs.fsplit != h.tune.factor_split ||
      gs.swpe != h.tune.solve_wpe ||
      gs.ebs != h.tune.eval_bs) {
    gs.captured = false;
    const int prof = h.prof;
    h.prof = 0;  // per-launch event pairs are not recorded into graphs
    struct Restore {
      Handle& h;
      int prof;
      ~Restore() { h.prof = prof; }
    } restore{h, prof};
    double* out = h.redbuf + 7LL * nseg;  // direction [4P], current point [3P], trial point [3P]
    GTRY(capture_graph(st, &gs.ex[G_OPT], [&]() -> int {
      HIP_TRY(launch_eval(h, W.xt, 1, W.y, 1, W.c, st));
      hipLaunchKernelGGL(k_lag_grad, dim3(nseg), dim3(GBS), 0, st, h.rec, h.gtab, h.gtab_n, W.y, h.seg, h.sinfo,
                         nst, h.jac_d_index, W.g, W.dpart);
      if (h.npar == 1)
        hipLaunchKernelGGL(k_grad_d, dim3(P), dim3(BS), 0, st, W.dpart, h.pseg, ob, W.xt, nxs, W.g);
      else
        hipLaunchKernelGGL(k_grad_design, dim3(P), dim3(DGS), 0, st, h.rec, W.y, h.pstage, h.sinfo, h.jac_d_index,
                           ob, W.xt, nxs, W.g);
      hipLaunchKernelGGL(k_opt_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.xt, W.zL, W.zU, W.g, W.y, W.c, W.s,
                         W.vU, b, nxs, h.redbuf);
      hipLaunchKernelGGL(k_sigma, dim3(gm), dim3(BS), 0, st, W.xt, W.zL, W.zU, W.s, W.vU, b, ob, nx, nxs, nst, h.diagx,
                         h.diags);
      hipLaunchKernelGGL(k_seg_reduce<9>, dim3(P), dim3(RS), 0, st, h.redbuf, h.pseg,
                         Ops<9>{{1, 1, 1, 1, 2, 1, 0, 0, 0}}, h.redbuf + 9LL * nseg);
      hipLaunchKernelGGL(k_ctl_opt, dim3(gp), dim3(64), 0, st, g, h.redbuf + 9LL * nseg, C, o.tol, o.max_iter);
      HIP_TRY(hipGetLastError());
      return ABS_OK;
    }));
    auto fac_a = [&]() -> int {
      hipLaunchKernelGGL(k_rhs, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, h.dwv, W.xt, W.g, W.y, W.c, W.s, h.diags,
                         b, C.kappa_d, ob, nxs, nks, W.rhs);
      HIP_TRY(hipGetLastError());
      return ABS_OK;
    };
    auto fac_b = [&]() -> int {
      HIP_TRY(launch_schur(h, h.diagx, W.rhs, 1, W.sol, st, h.fmask));
      hipLaunchKernelGGL(k_ctl_inertia, dim3(gp), dim3(64), 0, st, g, h.scal, C, o.delta_w_max);
      HIP_TRY(launch_residual(h, h.diagx, h.diags, W.sol, W.rhs, h.kres, h.omega_d, st));
      HIP_TRY(launch_residual_pmax(h, st));
      hipLaunchKernelGGL(k_ctl_res0, dim3(gp), dim3(64), 0, st, g, h.pres, 1e-10);
      HIP_TRY(hipGetLastError());
      return ABS_OK;
    };
    GTRY(capture_graph(st, &gs.ex[G_FAC], [&]() -> int {
      GTRY(fac_a());
      HIP_TRY(launch_factor(h, h.diagx, h.diags, W.rhs, true, st));
      return fac_b();
    }));
    GTRY(capture_graph(st, &gs.ex[G_FAC_A], fac_a));
    GTRY(capture_graph(st, &gs.ex[G_FAC_B], fac_b));
    // W.sol holds every problem's best iterate, h.kcor the corrected candidate
    // of the refining ones (rmask); every step of a correction reads and
    // writes only the refining problems' rows, so the others' rows of kres and
    // kcor are neither cleared nor read
    GTRY(capture_graph(st, &gs.ex[G_REF], [&]() -> int {
      int* const pact = h.pact;
      h.pact = h.rmask;
      const hipError_t e = launch_solve(h, h.kres, st, -1, nullptr, 1, 0, false);
      h.pact = pact;
      HIP_TRY(e);
      HIP_TRY(launch_schur(h, h.diagx, h.kres, 2, h.kres, st, h.rmask));
      HIP_TRY(launch_axpy_rows(h, h.rmask, h.kcor, W.sol, h.kres, 1.0, st));
      // the residual of the corrected iterate only for the refining problems
      // (the others' rows and partials come out zero and k_ctl_refine skips them)
      h.pact = h.rmask;
      const hipError_t er = launch_residual(h, h.diagx, h.diags, h.kcor, W.rhs, h.kres, h.omega_d, st, false);
      h.pact = pact;
      HIP_TRY(er);
      HIP_TRY(launch_residual_pmax(h, st));
      hipLaunchKernelGGL(k_ctl_refine, dim3(gp), dim3(64), 0, st, g, h.pres, 1e-10);
      HIP_TRY(launch_copy_rows(h, gs.cmask, W.sol, h.kcor, st));
      HIP_TRY(hipGetLastError());
      return ABS_OK;
    }));
    auto trial = [&]() -> int {
      hipLaunchKernelGGL(k_trial, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.dx, W.s, W.ds, nxs, W.xtt,
                         W.st);
      HIP_TRY(launch_eval(h, W.xtt, 1, nullptr, 0, W.ct, st));
      hipLaunchKernelGGL(k_ls_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xtt, W.st, W.ct, b, C.kappa_d,
                         ob, nxs, h.redbuf);
      hipLaunchKernelGGL(k_seg_reduce<3>, dim3(P), dim3(RS), 0, st, h.redbuf, h.pseg, Ops<3>{{0, 0, 0}},
                         out + 7LL * P);
      hipLaunchKernelGGL(k_ctl_ls, dim3(gp), dim3(64), 0, st, g, out + 7LL * P, C, phi_d);
      HIP_TRY(hipGetLastError());
      return ABS_OK;
    };
    GTRY(capture_graph(st, &gs.ex[G_DIR], [&]() -> int {
      hipLaunchKernelGGL(k_direction, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, h.dwv, W.xt, W.zL, W.zU, W.y, W.s,
                         W.vU, h.diags, W.sol, b, C.kappa_d, ob, nxs, nks, W.dx, W.dy, W.dzL, W.dzU, W.ds, W.dvU,
                         h.redbuf);
      hipLaunchKernelGGL(k_ls_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.s, W.c, b, C.kappa_d, ob, nxs,
                         h.redbuf + 4LL * nseg);
      hipLaunchKernelGGL(k_seg_reduce<4>, dim3(P), dim3(RS), 0, st, h.redbuf, h.pseg, Ops<4>{{2, 2, 0, 0}}, out);
      hipLaunchKernelGGL(k_seg_reduce<3>, dim3(P), dim3(RS), 0, st, h.redbuf + 4LL * nseg, h.pseg,
                         Ops<3>{{0, 0, 0}}, out + 4LL * P);
      hipLaunchKernelGGL(k_ctl_dir, dim3(gp), dim3(64), 0, st, g, out, out + 4LL * P, C, phi_d);
      return trial();
    }));
    GTRY(capture_graph(st, &gs.ex[G_LS], trial));
    GTRY(capture_graph(st, &gs.ex[G_ACC], [&]() -> int {
      hipLaunchKernelGGL(k_accept, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.xtt, W.s, W.st, W.y, W.dy,
                         W.zL, W.dzL, W.zU, W.dzU, W.vU, W.dvU, b, C.kappa_sigma, nxs);
      hipLaunchKernelGGL(k_ctl_accept, dim3(gp), dim3(64), 0, st, g, C, h.sc.Dd);
      HIP_TRY(hipGetLastError());
      return ABS_OK;
    }));
    gs.captured = true;
    gs.tol = o.tol;
    gs.dw_max = o.delta_w_max;
    gs.max_iter = o.max_iter;
    gs.timed = timed;
    gs.fwpe = h.tune.factor_wpe;
    gs.fsplit = h.tune.factor_split;
    gs.swpe = h.tune.solve_wpe;
    gs.ebs = h.tune.eval_bs;
  }
  // ---- replay passes
  auto read_status = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(gs.stat_h, gs.stat, sizeof(int2) * P, hipMemcpyDeviceToHost, st));
    HIP_TRY(wait_stream(st));
    return ABS_OK;
  };
  // a factorisation trial; timed: the factorisation is launched between the two
  // halves of the graph, bracketed by the profiling events on the same stream
  auto replay = [&](int k) -> hipError_t {
    ++replays;
    return hipGraphLaunch(gs.ex[k], st);
  };
  auto factor_trial = [&]() -> int {
    ++nfact;
    if (!timed) {
      HIP_TRY(replay(G_FAC));
      return ABS_OK;
    }
    HIP_TRY(replay(G_FAC_A));
    HIP_TRY(launch_factor(h, h.diagx, h.diags, W.rhs, true, st));
    HIP_TRY(replay(G_FAC_B));
    return ABS_OK;
  };
  auto count_phase = [&](int lo, int hi) {
    int n = 0;
    for (int p = 0; p < P; ++p) n += gs.stat_h[p].y && gs.stat_h[p].x >= lo && gs.stat_h[p].x <= hi;
    return n;
  };
  for (int p = 0; p < P; ++p) gs.stat_h[p] = make_int2(PH_IDLE, pr[(size_t)p].active ? 1 : 0);
  HIP_TRY(hipMemcpyAsync(gs.stat, gs.stat_h, sizeof(int2) * P, hipMemcpyHostToDevice, st));
  for (int iter = 0;; ++iter) {
    // the usual iteration: one factorisation with the right inertia, no
    // refinement correction, the first trial point accepted
    HIP_TRY(replay(G_OPT));
    GTRY(factor_trial());
    HIP_TRY(replay(G_DIR));
    HIP_TRY(replay(G_ACC));
    GTRY(read_status());
    // the problems that need more finish the iteration phase by phase; each
    // replay advances every problem in that phase (a bounded number of times:
    // delta_w grows to its bound, at most 10 corrections, alpha halves to its floor)
    for (int pass = 0; count_phase(PH_FACTOR, PH_ACCEPT) > 0; ++pass) {
      if (pass > 100000) {
        set_error("ipm_solve: the iteration of a problem does not advance");
        return ABS_ERR_STATE;
      }
      bool accept = count_phase(PH_ACCEPT, PH_ACCEPT) > 0;
      if (count_phase(PH_FACTOR, PH_FACTOR)) {
        GTRY(factor_trial());
      } else if (count_phase(PH_REFINE, PH_REFINE)) {
        HIP_TRY(replay(G_REF));
      } else if (count_phase(PH_DIR, PH_DIR)) {
        HIP_TRY(replay(G_DIR));
        accept = true;
      } else if (count_phase(PH_SEARCH, PH_SEARCH)) {
        HIP_TRY(replay(G_LS));
        accept = true;
      }
      if (accept) HIP_TRY(replay(G_ACC));
      GTRY(read_status());
    }
    int n_active = 0;
    for (int p = 0; p < P; ++p) n_active += gs.stat_h[p].y;
    if (o.print_level > 0 && P > 1) fprintf(stderr, "batch iteration %4d: %d of %d problems active\n", iter, n_active, P);
    if (n_active == 0) break;
  }
  // ---- final state of every problem, and the iteration logs
  std::vector<DevProb> dp((size_t)P);
  HIP_TRY(hipMemcpyAsync(dp.data(), gs.dp, sizeof(DevProb) * P, hipMemcpyDeviceToHost, st));
  std::vector<absorber_ipm_log_entry> lg((size_t)log_np * log_cap);
  HIP_TRY(hipMemcpyAsync(lg.data(), gs.log, sizeof(absorber_ipm_log_entry) * lg.size(), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int p = 0; p < P; ++p) {
    Prob& q = pr[(size_t)p];
    if (!q.active) continue;  // not part of this solve
    const DevProb& d = dp[(size_t)p];
    q.status = d.status;
    q.it = d.it;
    q.ncorr = d.ncorr;
    q.E0 = d.E0;
    q.inf_pr = d.inf_pr;
    q.inf_du = d.inf_du;
    q.compl0 = d.compl0;
    q.xd = d.xd;
    q.max_lin = d.max_lin;
    q.active = false;
    if (p < log_np) {
      auto& L = h.ipm_log[(size_t)p];
      L.clear();
      for (int i = 0; i < std::min(d.it, log_cap); ++i) L.push_back(lg[(size_t)p * log_cap + i]);
    }
  }
  return ABS_OK;
}

}  // namespace

#undef GTRY

// per-problem results of the segment partials in h.redbuf -> h.redbuf_h[p * K + k]
template <int K>
static int seg_reduce(Handle& h, const Ops<K>& ops, hipStream_t st) {
  double* out = h.redbuf + (long long)h.nseg * K;
  hipLaunchKernelGGL(k_seg_reduce<K>, dim3(h.P), dim3(RS), 0, st, h.redbuf, h.pseg, ops, out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h.redbuf_h, out, sizeof(double) * h.P * K, hipMemcpyDeviceToHost, st));
  HIP_TRY(wait_stream(st));
  return ABS_OK;
}

int kkt_solve_refined(Handle& h, const double* rhs, double* sol, bool fused_first, double* rel, hipStream_t st,
                      bool first_residual_read, double* rel_p, double target) {
  if (!fused_first) {
    HIP_TRY(launch_solve(h, rhs, st));
    HIP_TRY(launch_schur(h, h.diagx, rhs, 2, sol, st));
  }
  // Each problem refines until its own relative residual ||r_p - K_p x_p||_inf /
  // ||r_p||_inf (its stage rows and its d row) is at most the target, or until
  // a correction no longer decreases it; then it keeps its best iterate and
  // later corrections skip it (its rows of the residual are cleared and its
  // chains solve nothing).  Corrections are applied out of place: xn = xb +
  // correction, where xb holds every problem's best iterate so far; a problem
  // whose residual grew takes its entries of xb back into xn.
  const int P = h.P;
  const bool per_problem = P > 1;
  std::vector<double> best((size_t)P, INFINITY);
  std::vector<char> refining((size_t)P, 1);
  if (per_problem) {
    // In a batch, sol holds every problem's best iterate and h.kcor the
    // corrected candidate of the refining ones; each step reads and writes only
    // the rows of the problems it concerns (residual, solve, Schur step and
    // update under the refining mask, the candidates that lowered their
    // residual copied into sol), so the other rows are neither cleared nor read.
    // The arithmetic of each problem is that of the single-problem loop below.
    int* const pact = h.pact;
    const bool pact_on = h.pact_on;
    for (int it = 0; it <= 10; ++it) {
      if (it > 0 || !first_residual_read) {  // else the caller has taken the first residual
        if (it > 0) {
          h.pact = h.rmask;  // the problems corrected in the previous step
          h.pact_on = true;
        }
        const hipError_t e = launch_residual(h, h.diagx, h.diags, it > 0 ? h.kcor : sol, rhs, h.kres,
                                             h.omega_d, st, it == 0);
        h.pact = pact;
        h.pact_on = pact_on;
        HIP_TRY(e);
      }
      HIP_TRY(launch_residual_pmax(h, st));
      HIP_TRY(hipMemcpyAsync(h.pres_h, h.pres, sizeof(double) * 2 * P, hipMemcpyDeviceToHost, st));
      HIP_TRY(wait_stream(st));
      // first half of the pinned mask: the candidates kept; second half: the
      // problems refining on (both copies of the last step have completed)
      int* const keep_h = h.rmask_h;
      int* const ref_h = h.rmask_h + P;
      bool any_keep = false, any_left = false;
      for (int p = 0; p < P; ++p) {
        keep_h[p] = 0;
        if (refining[(size_t)p]) {
          const double r = h.pres_h[2 * p], b = h.pres_h[2 * p + 1];
          const double relr = b > 0.0 ? r / b : r;
          if (relr < best[(size_t)p]) {
            best[(size_t)p] = relr;
            if (it > 0) {
              keep_h[p] = 1;
              any_keep = true;
            }
            if (relr <= target) refining[(size_t)p] = 0;
          } else {  // no decrease (or not finite): sol keeps its previous iterate
            refining[(size_t)p] = 0;
          }
        }
        ref_h[p] = refining[(size_t)p] ? 1 : 0;
        any_left = any_left || refining[(size_t)p];
      }
      if (any_keep) {
        HIP_TRY(hipMemcpyAsync(h.rmask, keep_h, sizeof(int) * P, hipMemcpyHostToDevice, st));
        HIP_TRY(launch_copy_rows(h, h.rmask, sol, h.kcor, st));
      }
      if (!any_left || it == 10) break;
      HIP_TRY(hipMemcpyAsync(h.rmask, ref_h, sizeof(int) * P, hipMemcpyHostToDevice, st));
      h.pact = h.rmask;
      h.pact_on = true;
      const hipError_t e = launch_solve(h, h.kres, st, -1, nullptr, 1, 0, false);
      h.pact = pact;
      h.pact_on = pact_on;
      HIP_TRY(e);
      HIP_TRY(launch_schur(h, h.diagx, h.kres, 2, h.kres, st, h.rmask));       // the correction
      HIP_TRY(launch_axpy_rows(h, h.rmask, h.kcor, sol, h.kres, 1.0, st));  // candidate = sol + correction
    }
    double worst = 0.0;
    for (int p = 0; p < P; ++p) {
      worst = std::max(worst, best[(size_t)p]);
      if (rel_p) rel_p[p] = best[(size_t)p];
    }
    if (rel) *rel = worst;
    return ABS_OK;
  }
  // One problem: corrections are applied out of place, xn = xb + correction,
  // where xb is the best iterate so far; if the residual grows, xb is kept.
  double* xb = sol;
  double* xn = sol;
  double* om = h.redbuf_h + h.red_cap - 4;  // four pinned doubles past the partials
  for (int it = 0; it <= 10; ++it) {
    if (it > 0 || !first_residual_read) {  // else the caller has read the first residual's norms into om
      HIP_TRY(launch_residual(h, h.diagx, h.diags, xn, rhs, h.kres, h.omega_d, st));
      HIP_TRY(hipMemcpyAsync(om, h.omega_d, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(wait_stream(st));
    }
    const double relr = om[3] > 0.0 ? om[2] / om[3] : om[2];
    if (relr < best[0]) {
      best[0] = relr;
      h.last_omega = fmax(om[0], om[1]);  // backward error of the kept iterate
      if (relr <= target) break;
    } else {  // no decrease (or not finite): the previous iterate is kept
      xn = xb;
      break;
    }
    if (it == 10) break;
    HIP_TRY(launch_solve(h, h.kres, st));
    HIP_TRY(launch_schur(h, h.diagx, h.kres, 2, h.kres, st));  // the correction, in place
    double* xnew = xn == sol ? h.kcor : sol;
    HIP_TRY(launch_axpy(xnew, xn, h.kres, 1.0, h.nkkt, st));  // xnew = xn + correction
    xb = xn;
    xn = xnew;
  }
  if (xn != sol) HIP_TRY(hipMemcpyAsync(sol, xn, sizeof(double) * h.nkkt, hipMemcpyDeviceToDevice, st));
  double worst = 0.0;
  for (int p = 0; p < P; ++p) {
    worst = std::max(worst, best[(size_t)p]);
    if (rel_p) rel_p[p] = best[(size_t)p];
  }
  if (rel) *rel = worst;
  return ABS_OK;
}

int ipm_solve(Handle& h, const absorber_ipm_options& o, const double* x0_dev, const double* y0_dev, double* xout,
              double* yout, absorber_ipm_result* res, const unsigned char* active0) {
  const auto t_start = std::chrono::steady_clock::now();
  const Consts C;
  hipStream_t st = h.stream;
  if (o.use_graph) {
    // graphs are captured on a stream of their own; the caller's work on the
    // default stream (its start point, multipliers) is complete first
    st = ipm_graph_stream(h);
    if (!st) {
      set_error("ipm_solve: could not create the graph stream");
      return ABS_ERR_HIP;
    }
    HIP_TRY(hipDeviceSynchronize());
  }
  const int P = h.P;
  const long long nx = h.nx, nc = h.nc, nst = h.nst, nkkt = h.nkkt;
  const long long nxs = nst * NV, nks = nst * NK;
  const int nseg = h.nseg;
  if (9LL * (nseg + P) > h.red_cap - 4) {
    set_error("ipm_solve: problem too large for the reduction buffer");
    return ABS_ERR_ARG;
  }
  Work W;
  {
    // the work vectors, carved from one device allocation kept by the handle
    double** bufs[] = {&W.xt, &W.xtt, &W.zL, &W.zU, &W.g, &W.dx, &W.dzL, &W.dzU,  // nx
                       &W.y, &W.c, &W.ct, &W.dy, &W.rowmax,                       // nc
                       &W.s, &W.st, &W.vU, &W.ds, &W.dvU, &W.dpart,               // nst
                       &W.rhs, &W.sol};                                           // nkkt
    const long long len[] = {nx, nx, nx, nx, nx, nx, nx, nx, nc, nc, nc, nc, nc,
                             nst, nst, nst, nst, nst, nst, nkkt, nkkt};
    static_assert(sizeof(bufs) / sizeof(bufs[0]) == sizeof(len) / sizeof(len[0]), "one length per buffer");
    size_t off[sizeof(len) / sizeof(len[0])], total = 0;
    for (size_t i = 0; i < sizeof(len) / sizeof(len[0]); ++i) {
      off[i] = total;
      total += ((size_t)std::max<long long>(len[i], 1) + 31) / 32 * 32;  // 256-byte aligned pieces
    }
    if (!h.ipm_work) {
      HIP_TRY(hipMalloc((void**)&h.ipm_work, total * sizeof(double)));
      h.ipm_work_bytes = total * sizeof(double);
    }
    if (!h.ipm_dd_h) HIP_TRY(hipHostMalloc((void**)&h.ipm_dd_h, sizeof(double) * (size_t)P * MAX_NPAR, 0));
    HIP_TRY(hipMemsetAsync(h.ipm_work, 0, h.ipm_work_bytes, st));
    for (size_t i = 0; i < sizeof(len) / sizeof(len[0]); ++i) *bufs[i] = h.ipm_work + off[i];
  }
  // per-problem scalars live in the handle's control block (one transfer for all of them)
  static_assert(sizeof(PS) <= CTL_SLOT, "solver scalars exceed the control block slot");
  W.ps = reinterpret_cast<PS*>(h.slot_area);
  W.ps_h = reinterpret_cast<PS*>(h.ctl_h + ctl_off_slot(P));
  W.dw_h = reinterpret_cast<double*>(h.ctl_h);
  W.dc_h = W.dw_h + P;
  W.fm_h = reinterpret_cast<int*>(h.ctl_h + ctl_off_fmask(P));
  int* pa_h = reinterpret_cast<int*>(h.ctl_h + ctl_off_pact(P));
  W.dd_h = h.ipm_dd_h;
  std::vector<Prob> pr((size_t)P);
  h.ipm_log.resize((size_t)P);
  for (int p = 0; p < P; ++p)
    if (!active0 || active0[p]) h.ipm_log[(size_t)p].clear();
  std::vector<double> rel_p((size_t)P, 0.0);
  // scalars, activity, regularisation and the refactorisation mask of every
  // problem -> device, in one transfer
  auto upload = [&]() -> int {
    // the previous upload's copy reads ctl_h when it runs: let it finish first
    if (h.ctl_ev_rec) HIP_TRY(hipEventSynchronize(h.ctl_ev));
    for (int p = 0; p < P; ++p) {
      const Prob& q = pr[(size_t)p];
      PS& d = W.ps_h[p];
      d.mu = q.mu;
      d.tau = q.tau;
      d.alpha = q.alpha;
      d.alpha_z = q.alpha_z;
      d.active = q.active;
      d.search = q.searching;
      d.accept = q.accepted;
      d.zero_y = 0;
      d.write = !active0 || active0[p];
      pa_h[p] = q.active;
      W.dw_h[p] = q.dw;
      W.dc_h[p] = q.dc;
      W.fm_h[p] = q.need ? 1 : 0;
    }
    HIP_TRY(hipMemcpyAsync(h.ctl, h.ctl_h, h.ctl_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(h.ctl_ev, st));
    h.ctl_ev_rec = true;
    return ABS_OK;
  };
  // the per-stage kernels skip problems that are done (or not asked for)
  struct PactGuard {
    Handle& h;
    ~PactGuard() { h.pact_on = false; }
  } pact_guard{h};
  // design entries of a primal vector -> W.dd_h[p] = sum_k c_k xt_theta_k (the
  // scaled design cost; the diameter itself with one design entry)
  auto read_d = [&](const double* v) -> int {
    HIP_TRY(hipMemcpyAsync(W.dd_h, v + nxs, sizeof(double) * P * h.npar, hipMemcpyDeviceToHost, st));
    HIP_TRY(wait_stream(st));
    if (h.npar > 1)
      for (int p = 0; p < P; ++p) {
        double a = 0.0;
        for (int k = 0; k < h.npar; ++k) a += h.cw[k] * W.dd_h[(size_t)p * h.npar + k];
        W.dd_h[p] = a;  // p <= p * npar: no entry still needed is overwritten
      }
    return ABS_OK;
  };
#define TRY(expr)            \
  do {                       \
    const int rc_ = (expr);  \
    if (rc_) return rc_;     \
  } while (0)

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
  const unsigned gx = grid_for(nx, BS), gc = grid_for(nc, BS), gst = grid_for(nst, BS);
  const unsigned gm = grid_for(std::max(nx, nc), BS);
  // ---- bound-pushed cold point and gradient-based row scaling there
  TRY(initial_point(h, W.xtt, st));
  hipLaunchKernelGGL(k_scale_x, dim3(gx), dim3(BS), 0, st, W.xtt, h.sc, nx, nxs, W.xt);
  hipLaunchKernelGGL(k_init_point, dim3(gx), dim3(BS), 0, st, W.xt, W.zL, W.zU, b, o.bound_push, o.bound_push, 0,
                     0.0, C.zinit, nx, nxs);
  HIP_TRY(launch_rowmax(h, W.xt, 1, W.rowmax, st));
  hipLaunchKernelGGL(k_rowscale, dim3(gc), dim3(BS), 0, st, W.rowmax, o.nlp_scaling_max_gradient, nc, h.cs);
  // gradient-based objective scaling at the cold point: f = sum_k c_k theta_k +
  // a_k theta_k^-4 has the gradient (c_k - 4 a_k theta_k^-5) D_d with respect to
  // the scaled design entries (c = 1 and a = 0 for problem (10))
  double gmax = 0.0;
  {
    const double th0 = zc[NV], t5 = th0 * th0 * th0 * th0 * th0;
    for (int p = 0; p < P; ++p)
      for (int k = 0; k < h.npar; ++k) {
        const double c = h.npar == 1 ? 1.0 : h.cw[k];
        const double a = h.has_op ? h.opa_h[(size_t)p * h.npar + k] : 0.0;
        gmax = std::max(gmax, a == 0.0 ? c : fabs(c - 4.0 * a / t5));
      }
  }
  h.sf = std::min(1.0, o.nlp_scaling_max_gradient / (gmax * h.sc.Dd));
  const double gf = h.sf * h.sc.Dd;  // gradient of f~ = sf * d with respect to xt_d
  Obj ob{};
  ob.npar = h.npar;
  ob.a = h.has_op ? h.opa : nullptr;
  ob.sf = h.sf;
  ob.Dd = h.sc.Dd;
  for (int k = 0; k < h.npar; ++k) {
    ob.c[k] = h.npar == 1 ? 1.0 : h.cw[k];
    ob.g[k] = h.npar == 1 ? gf : gf * h.cw[k];
  }
  const double mu0 = warm ? o.warm_mu_init : o.mu_init;
  for (auto& q : pr) {
    q.mu = mu0;
    q.tau = std::max(C.tau_min, 1.0 - mu0);
  }
  if (warm) {
    hipLaunchKernelGGL(k_scale_x, dim3(gx), dim3(BS), 0, st, x0_dev, h.sc, nx, nxs, W.xt);
    hipLaunchKernelGGL(k_init_point, dim3(gx), dim3(BS), 0, st, W.xt, W.zL, W.zU, b, o.warm_bound_push,
                       o.warm_bound_push, 1, mu0, C.zinit, nx, nxs);
  }
  HIP_TRY(launch_eval(h, W.xt, 1, nullptr, 0, W.c, st));
  hipLaunchKernelGGL(k_init_slack, dim3(gst), dim3(BS), 0, st, W.c, W.s, W.vU, warm ? o.warm_bound_push : o.bound_push,
                     warm ? 1 : 0, mu0, C.zinit, nst);
  hipLaunchKernelGGL(k_fill, dim3(gc), dim3(BS), 0, st, W.y, 0.0, nc);
  double rel = 0.0;
  int nfact = 0;
  TRY(upload());
  if (warm && y0_dev) {
    // multipliers of the unscaled rows -> multipliers of the scaled rows
    hipLaunchKernelGGL(k_mul, dim3(gc), dim3(BS), 0, st, y0_dev, h.cs, nc, 1, W.y);
  } else {
    // least-squares multipliers: [[I, J^T], [J, 0]] (slack block eliminated)
    HIP_TRY(launch_eval(h, W.xt, 1, W.y, 1, W.ct, st));
    hipLaunchKernelGGL(k_fill, dim3(gx), dim3(BS), 0, st, h.diagx, 0.0, nx);
    hipLaunchKernelGGL(k_fill, dim3(gst), dim3(BS), 0, st, h.diags, 0.0, nst);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(nkkt, BS)), dim3(BS), 0, st, W.rhs, 0.0, nkkt);
    hipLaunchKernelGGL(k_ls_rhs, dim3(grid_for(std::max(nx, nst), BS)), dim3(BS), 0, st, W.xt, W.zL, W.zU, W.vU, ob, nx,
                       nxs, nks, nst, W.rhs);
    for (auto& q : pr) {
      q.dw = 1.0;
      q.dc = 0.0;
    }
    TRY(upload());
    HIP_TRY(launch_factor(h, h.diagx, h.diags, W.rhs, false, st));
    ++nfact;
    HIP_TRY(launch_schur(h, h.diagx, W.rhs, 1, W.sol, st));
    TRY(kkt_solve_refined(h, W.rhs, W.sol, true, &rel, st));
    hipLaunchKernelGGL(k_copy_duals, dim3(gc), dim3(BS), 0, st, W.sol, nc, W.y);
    hipLaunchKernelGGL(k_ymax_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.y, h.redbuf);
    TRY(seg_reduce<1>(h, Ops<1>{{1}}, st));
    bool any = false;
    for (int p = 0; p < P; ++p) {
      W.ps_h[p].zero_y = !(h.redbuf_h[p] <= C.constr_mult_init_max);
      any = any || W.ps_h[p].zero_y;
    }
    if (any) {
      HIP_TRY(hipMemcpyAsync(W.ps, W.ps_h, sizeof(PS) * P, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_zero_y, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.y);
    }
  }
  TRY(read_d(W.xt));
  // ---- per-problem filter bounds from theta(x0) and multiplier counts
  hipLaunchKernelGGL(k_ls_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.s, W.c, b, C.kappa_d, ob, nxs,
                     h.redbuf);
  TRY(seg_reduce<3>(h, Ops<3>{{0, 0, 0}}, st));
  long long nbL1 = 0, nbU1 = 0;  // finite bounds per stage
  for (int k = 0; k < NV; ++k) {
    nbL1 += std::isfinite(b.lo[k]);
    nbU1 += std::isfinite(b.hi[k]);
  }
  for (int p = 0; p < P; ++p) {
    Prob& q = pr[(size_t)p];
    const double th0 = h.redbuf_h[p * 3 + 0];
    q.theta_max = C.theta_max_fact * std::max(1.0, th0);
    q.theta_min = C.theta_min_fact * std::max(1.0, th0);
    q.xd = W.dd_h[p];
    const double nsp = (double)(h.pstage_h[(size_t)p + 1] - h.pstage_h[(size_t)p]);
    q.nx_p = NV * nsp + h.npar;
    q.nc_p = NR * nsp;
    const double nbL = nbL1 * nsp + h.npar * std::isfinite(b.lo[NV]);
    const double nbU = nbU1 * nsp + h.npar * std::isfinite(b.hi[NV]);
    q.n_all = q.nc_p + nbL + nbU + nsp;
    q.n_b = nbL + nbU + nsp;
  }
  int n_active = P, iter = 0;
  if (active0) {
    n_active = 0;
    for (int p = 0; p < P; ++p) {
      pr[(size_t)p].active = active0[p] != 0;
      n_active += active0[p] != 0;
    }
  }
  TRY(upload());
  h.pact_on = true;
  int replays = 0;
  if (o.use_graph) TRY(graph_iterations(h, o, C, b, ob, W, pr, st, nfact, replays));
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  while (!o.use_graph) {
    const auto ph0 = now();
    int n_fac_it = 0, n_ls_it = 0;
    // ---- evaluation at (x_k, y_k): residuals, Jacobian, Hessian, Lagrangian gradient
    HIP_TRY(launch_eval(h, W.xt, 1, W.y, 1, W.c, st));
    hipLaunchKernelGGL(k_lag_grad, dim3(nseg), dim3(GBS), 0, st, h.rec, h.gtab, h.gtab_n, W.y, h.seg, h.sinfo, nst,
                       h.jac_d_index, W.g, W.dpart);
    if (h.npar == 1)
      hipLaunchKernelGGL(k_grad_d, dim3(P), dim3(BS), 0, st, W.dpart, h.pseg, ob, W.xt, nxs, W.g);
    else
      hipLaunchKernelGGL(k_grad_design, dim3(P), dim3(DGS), 0, st, h.rec, W.y, h.pstage, h.sinfo, h.jac_d_index, ob,
                         W.xt, nxs, W.g);
    hipLaunchKernelGGL(k_opt_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.xt, W.zL, W.zU, W.g, W.y, W.c, W.s, W.vU,
                       b, nxs, h.redbuf);
    // the barrier Hessian diagonals at x_k need no decision of the host: queue them now
    hipLaunchKernelGGL(k_sigma, dim3(gm), dim3(BS), 0, st, W.xt, W.zL, W.zU, W.s, W.vU, b, ob, nx, nxs, nst, h.diagx,
                       h.diags);
    TRY(seg_reduce<9>(h, Ops<9>{{1, 1, 1, 1, 2, 1, 0, 0, 0}}, st));
    for (int p = 0; p < P; ++p) {
      Prob& q = pr[(size_t)p];
      if (!q.active) continue;
      const double* ov = h.redbuf_h + p * 9;
      const double dual = std::max(ov[0], ov[1]);
      const double primal = std::max(ov[2], ov[3]);
      const double sd = std::max(C.s_max, (ov[6] + ov[7]) / q.n_all) / C.s_max;
      const double sc = std::max(C.s_max, ov[7] / q.n_b) / C.s_max;
      auto Emu = [&](double m) {
        const double comp = std::max(fabs(ov[5] - m), fabs(ov[4] - m));
        return std::max(std::max(dual / sd, primal), comp / sc);
      };
      q.E0 = Emu(0.0);
      q.inf_pr = primal;
      q.inf_du = dual;
      q.compl0 = std::max(fabs(ov[4]), fabs(ov[5]));
      int stop = 1;
      if (ov[8] > 0 || !std::isfinite(q.E0)) q.status = ABS_ERR_NAN;
      else if (q.E0 <= o.tol) q.status = ABS_OK;
      else if (q.it >= o.max_iter) q.status = ABS_ERR_MAXITER;
      else stop = 0;
      if (stop) {
        q.active = false;
        --n_active;
        continue;
      }
      // monotone barrier update (repeated while the barrier problem is solved)
      while (Emu(q.mu) <= C.kappa_eps * q.mu) {
        const double mu_new = std::max(o.tol / 10.0, std::min(C.kappa_mu * q.mu, pow(q.mu, C.theta_mu)));
        if (mu_new >= q.mu) break;  // already at its floor tol / 10: the update is done
        q.mu = mu_new;
        q.tau = std::max(C.tau_min, 1.0 - q.mu);
        q.filt.pts.clear();
      }
    }
    if (n_active == 0) break;
    const auto ph1 = now();
    // ---- search direction with inertia correction (each problem its own delta_w)
    for (auto& q : pr) {
      q.dw = 0.0;
      q.dc = 0.0;
      q.need = q.active;
      q.nfac = 0;
    }
    TRY(upload());
    for (bool first = true;; first = false) {
      if (!first) TRY(upload());
      hipLaunchKernelGGL(k_rhs, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, h.dwv, W.xt, W.g, W.y, W.c, W.s, h.diags,
                         b, C.kappa_d, ob, nxs, nks, W.rhs);
      if (o.autotune && !h.tune.done) TRY(autotune(h, W.xt, W.y, W.c, h.diagx, h.diags, W.rhs, st));
      HIP_TRY(launch_factor(h, h.diagx, h.diags, W.rhs, true, st));
      ++nfact;
      ++n_fac_it;
      HIP_TRY(launch_schur(h, h.diagx, W.rhs, 1, W.sol, st));
      // the first residual of this solve is queued with the inertia read (one round trip
      // for both; it is wasted only when the inertia asks for another factorisation)
      HIP_TRY(launch_residual(h, h.diagx, h.diags, W.sol, W.rhs, h.kres, h.omega_d, st));
      HIP_TRY(hipMemcpyAsync(h.redbuf_h + h.red_cap - 4, h.omega_d, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(h.scal_h, h.scal, sizeof(DevScalars) * P, hipMemcpyDeviceToHost, st));
      HIP_TRY(wait_stream(st));
      bool again = false;
      for (int p = 0; p < P; ++p) {
        Prob& q = pr[(size_t)p];
        if (!q.need) continue;
        ++q.nfac;
        const DevScalars& D = h.scal_h[p];
        if ((double)D.npos == q.nx_p && (double)D.nneg == q.nc_p && D.nzero == 0) {
          if (q.dw > 0.0) q.dw_last = q.dw;
          q.need = false;
          continue;
        }
        ++q.ncorr;
        if (D.nzero > 0) q.dc = C.dc_bar * pow(q.mu, C.kappa_c);
        if (q.dw == 0.0) q.dw = q.dw_last == 0.0 ? C.dw_init : std::max(C.dw_min, C.kw_minus * q.dw_last);
        else q.dw = (q.dw_last == 0.0 ? C.kw_plus_bar : C.kw_plus) * q.dw;
        if (q.dw > o.delta_w_max) {
          q.status = ABS_ERR_INERTIA;
          q.active = false;
          q.need = false;
          --n_active;
          continue;
        }
        again = true;
      }
      if (!again) break;
    }
    if (n_active == 0) break;
    const auto ph2 = now();
    TRY(upload());
    TRY(kkt_solve_refined(h, W.rhs, W.sol, true, &rel, st, true, rel_p.data()));
    for (int p = 0; p < P; ++p)
      if (pr[(size_t)p].active) pr[(size_t)p].max_lin = std::max(pr[(size_t)p].max_lin, rel_p[(size_t)p]);
    const auto ph3 = now();
    // ---- step pieces and fraction to the boundary
    // and, reduced together, theta and the barrier function at the current point
    hipLaunchKernelGGL(k_direction, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, h.dwv, W.xt, W.zL, W.zU, W.y, W.s,
                       W.vU, h.diags, W.sol, b, C.kappa_d, ob, nxs, nks, W.dx, W.dy, W.dzL, W.dzU, W.ds, W.dvU,
                       h.redbuf);
    hipLaunchKernelGGL(k_ls_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.s, W.c, b, C.kappa_d, ob, nxs,
                       h.redbuf + 4LL * nseg);
    {
      // per problem: [4] direction values, [3] the current point's theta/phi parts, then
      // [3] those of the first trial point (at alpha_max, queued without a round trip)
      double* out = h.redbuf + 7LL * nseg;
      hipLaunchKernelGGL(k_seg_reduce<4>, dim3(P), dim3(RS), 0, st, h.redbuf, h.pseg, Ops<4>{{2, 2, 0, 0}}, out);
      hipLaunchKernelGGL(k_seg_reduce<3>, dim3(P), dim3(RS), 0, st, h.redbuf + 4LL * nseg, h.pseg,
                         Ops<3>{{0, 0, 0}}, out + 4LL * P);
      hipLaunchKernelGGL(k_trial_first, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, out, W.xt, W.dx, W.s, W.ds, nxs,
                         W.xtt, W.st);
      HIP_TRY(launch_eval(h, W.xtt, 1, nullptr, 0, W.ct, st));
      hipLaunchKernelGGL(k_ls_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xtt, W.st, W.ct, b, C.kappa_d,
                         ob, nxs, h.redbuf);
      hipLaunchKernelGGL(k_seg_reduce<3>, dim3(P), dim3(RS), 0, st, h.redbuf, h.pseg, Ops<3>{{0, 0, 0}},
                         out + 7LL * P);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(h.redbuf_h, out, sizeof(double) * 10 * P, hipMemcpyDeviceToHost, st));
      HIP_TRY(wait_stream(st));
    }
    for (int p = 0; p < P; ++p) {
      Prob& q = pr[(size_t)p];
      const double* dv = h.redbuf_h + p * 4;
      const double* lv = h.redbuf_h + 4 * P + p * 3;
      q.alpha_max = dv[0];
      q.alpha_z = dv[1];
      q.gdx = dv[2];
      q.dxd = dv[3];
      if (!q.active) continue;
      q.th = lv[0];
      q.phi = h.sf * h.sc.Dd * q.xd + lv[1];
      const double th = q.th, gdx = q.gdx;
      if (gdx < 0 && th <= q.theta_min)
        q.amin = C.gamma_alpha * std::min({C.gamma_theta, C.gamma_phi * th / (-gdx),
                                           C.delta * pow(th, C.s_theta) / pow(-gdx, C.s_phi)});
      else if (gdx < 0)
        q.amin = C.gamma_alpha * std::min(C.gamma_theta, C.gamma_phi * th / (-gdx));
      else
        q.amin = C.gamma_alpha * C.gamma_theta;
      q.alpha = q.alpha_max;
      q.searching = true;
      q.accepted = false;
      q.nls = 0;
    }
    // ---- filter line search, all searching problems at once
    const auto ph4 = now();
    for (bool first = true;; first = false) {
      ++n_ls_it;
      if (!first) {  // the first trial (alpha_max) was evaluated with the direction
        TRY(upload());
        hipLaunchKernelGGL(k_trial, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.dx, W.s, W.ds, nxs, W.xtt,
                           W.st);
        HIP_TRY(launch_eval(h, W.xtt, 1, nullptr, 0, W.ct, st));
        hipLaunchKernelGGL(k_ls_parts, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xtt, W.st, W.ct, b, C.kappa_d,
                           ob, nxs, h.redbuf);
        TRY(seg_reduce<3>(h, Ops<3>{{0, 0, 0}}, st));
      }
      const double* tvs = first ? h.redbuf_h + 7 * P : h.redbuf_h;
      bool any = false;
      for (int p = 0; p < P; ++p) {
        Prob& q = pr[(size_t)p];
        if (!q.searching) continue;
        const double* tv = tvs + p * 3;
        ++q.nls;
        const double tht = tv[0];
        const double phit = tv[2] > 0 ? INFINITY : h.sf * h.sc.Dd * (q.xd + q.alpha * q.dxd) + tv[1];
        const double th = q.th, phi = q.phi;
        bool okt = std::isfinite(phit) && std::isfinite(tht) && tht < q.theta_max && q.filt.acceptable(tht, phit);
        bool acc = false, ftype = false;
        if (okt) {
          const double ma = q.alpha * q.gdx;
          const bool switching =
              ma < 0 && pow(-ma, C.s_phi) * pow(q.alpha, 1 - C.s_phi) > C.delta * pow(th, C.s_theta);
          if (th <= q.theta_min && switching) {
            if (phit <= phi + C.eta_phi * ma) {
              acc = true;
              ftype = true;
            }
          } else if (tht <= (1 - C.gamma_theta) * th || phit <= phi - C.gamma_phi * th) {
            acc = true;
          }
        }
        if (acc) {
          q.searching = false;
          q.accepted = true;
          q.ftype = ftype;
          continue;
        }
        q.alpha *= 0.5;
        // below the minimum step (or below double resolution when that bound underflows)
        if (q.alpha < std::max(q.amin, C.alpha_floor)) {
          q.searching = false;
          q.status = ABS_ERR_LS;
          q.active = false;
          --n_active;
          continue;
        }
        any = true;
      }
      if (!any) break;
    }
    // ---- accept
    for (int p = 0; p < P; ++p) {
      Prob& q = pr[(size_t)p];
      if (!q.accepted) continue;
      if (!q.ftype) q.filt.pts.push_back({(1 - C.gamma_theta) * q.th, q.phi - C.gamma_phi * q.th});
      q.xd = q.xd + q.alpha * q.dxd;
      ++q.it;
      absorber_ipm_log_entry e{};
      e.iteration = q.it;
      e.n_factorizations = q.nfac;
      e.n_trials = q.nls;
      e.mu = q.mu;
      e.theta = q.th;
      e.alpha = q.alpha;
      e.alpha_z = q.alpha_z;
      e.delta_w = q.dw;
      e.delta_c = q.dc;
      e.d = q.xd * h.sc.Dd;
      e.E0 = q.E0;
      h.ipm_log[(size_t)p].push_back(e);
    }
    TRY(upload());
    hipLaunchKernelGGL(k_accept, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.xtt, W.s, W.st, W.y, W.dy, W.zL,
                       W.dzL, W.zU, W.dzU, W.vU, W.dvU, b, C.kappa_sigma, nxs);
    ++iter;
    for (int p = 0; p < P; ++p) {
      Prob& q = pr[(size_t)p];
      if (q.accepted && P == 1 && o.print_level > 0)
        fprintf(stderr, "it %4d mu %9.2e th %9.2e a %9.2e az %9.2e ls %2d dw %8.1e d %.10f E0 %9.2e res %8.1e\n",
                q.it, q.mu, q.th, q.alpha, q.alpha_z, q.nls, q.dw, q.xd * h.sc.Dd, q.E0, rel);
      q.accepted = false;
      if (q.active && fabs(q.xd) > 1e20) {
        q.status = ABS_ERR_DIVERGE;
        q.active = false;
        --n_active;
      }
    }
    if (P > 1 && o.print_level > 0) fprintf(stderr, "batch iteration %4d: %d of %d problems active\n", iter, n_active, P);
    if (o.print_level > 1) {
      const auto ph5 = now();
      fprintf(stderr,
              "  phases [ms] eval+opt %.1f  factor(x%d) %.1f  refine %.1f  direction %.1f  line search(x%d) %.1f\n",
              ms(ph0, ph1), n_fac_it, ms(ph1, ph2), ms(ph2, ph3), ms(ph3, ph4), n_ls_it, ms(ph4, ph5));
    }
    if (n_active == 0) break;
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (xout || yout) {
    TRY(upload());
    hipLaunchKernelGGL(k_output, dim3(nseg), dim3(BS), 0, st, h.seg, W.ps, W.xt, W.y, h.cs, h.sc, nxs, xout, yout);
  }
#undef TRY
  HIP_TRY(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  int first_err = ABS_OK;
  for (int p = 0; p < P; ++p) {
    if (active0 && !active0[p]) continue;
    const Prob& q = pr[(size_t)p];
    if (q.status != ABS_OK && first_err == ABS_OK) first_err = q.status;
    if (!res) continue;
    absorber_ipm_result& r = res[p];
    r.status = q.status;
    r.iterations = q.it;
    r.E0 = q.E0;
    r.inf_pr = q.inf_pr;
    r.inf_du = q.inf_du;
    r.compl_ = q.compl0;
    r.d = q.xd * h.sc.Dd;
    r.seconds = secs;
    r.n_inertia_corrections = q.ncorr;
    r.n_factorizations = nfact;
    r.max_lin_resid = q.max_lin;
    r.feasibility_restarts = 0;
    r.graph_replays = replays;
  }
  return first_err;
}

// Solve; then, with o.feasibility_restart, solve the problems that stopped
// without converging once more from their simulated states (process
// simulation of every scenario, d at its hydraulic minimum times 1 + 1e-3,
// warm-start options).  The results of a restarted problem count both runs.
int solve_with_restart(Handle& h, const absorber_ipm_options& o, const double* x0_dev, const double* y0_dev,
                       double* xout, double* yout, absorber_ipm_result* res) {
  const int P = h.P;
  std::vector<absorber_ipm_result> r1((size_t)P);
  int rc = ipm_solve(h, o, x0_dev, y0_dev, xout, yout, r1.data(), nullptr);
  if (rc < 0 && rc > ABS_ERR_INERTIA) return rc;  // argument, device or allocation error
  std::vector<unsigned char> redo((size_t)P, 0);
  bool any = false;
  for (int p = 0; p < P; ++p) {
    const int s = r1[(size_t)p].status;
    redo[(size_t)p] = o.feasibility_restart && (s == ABS_ERR_LS || s == ABS_ERR_INERTIA || s == ABS_ERR_MAXITER ||
                                                 s == ABS_ERR_DIVERGE || s == ABS_ERR_NAN);
    any = any || redo[(size_t)p];
  }
  if (any) {
    double* xs = nullptr;
    HIP_TRY(hipMalloc((void**)&xs, sizeof(double) * (size_t)h.nx));
    std::vector<int> conv((size_t)P);
    int it = 0;
    int rs = initial_point(h, xs, h.stream);
    if (!rs) rs = simulate(h, xs, redo.data(), 1e-10, 100, conv.data(), &it);
    if (!rs) rs = set_hydraulic_diameters(h, xs, 1e-3, h.stream);
    if (!rs) {
      absorber_ipm_options ow = o;
      ow.warm_start = 1;
      std::vector<absorber_ipm_result> r2 = r1;
      const int rc2 = ipm_solve(h, ow, xs, nullptr, xout, yout, r2.data(), redo.data());
      if (rc2 < 0 && rc2 > ABS_ERR_INERTIA) rs = rc2;  // argument, device or allocation error of the restart
      for (int p = 0; p < P && !rs; ++p)
        if (redo[(size_t)p]) {
          r2[(size_t)p].iterations += r1[(size_t)p].iterations;
          r2[(size_t)p].n_inertia_corrections += r1[(size_t)p].n_inertia_corrections;
          r2[(size_t)p].graph_replays += r1[(size_t)p].graph_replays;
          r2[(size_t)p].feasibility_restarts = 1;
          r1[(size_t)p] = r2[(size_t)p];
        }
    }
    (void)hipFree(xs);
    if (rs) return rs;
  }
  rc = ABS_OK;
  for (int p = 0; p < P; ++p) {
    if (r1[(size_t)p].status != ABS_OK && rc == ABS_OK) rc = r1[(size_t)p].status;
    if (res) res[p] = r1[(size_t)p];
  }
  return rc;
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
  o->feasibility_restart = 1;
  o->autotune = 1;
  o->delta_w_max = 1e40;
}

static int check_options(const absorber_ipm_options* opts, absorber_ipm_options* o, const char* who) {
  if (opts) *o = *opts;
  else absorber_ipm_default_options(o);
  if (!(o->tol > 0) || o->max_iter < 0 || !(o->delta_w_max > 0)) {
    set_error(std::string(who) + ": bad options");
    return ABS_ERR_ARG;
  }
  return ABS_OK;
}

int absorber_ipm_solve(absorber_t* H, const absorber_ipm_options* opts, const double* x0_dev,
                       const double* lambda0_dev, double* x_out_dev, double* lambda_out_dev,
                       absorber_ipm_result* result) {
  if (!H) {
    set_error("absorber_ipm_solve: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_ipm_solve: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  absorber_ipm_options o;
  const int rc = check_options(opts, &o, "absorber_ipm_solve");
  if (rc) return rc;
  return solve_with_restart(H->h, o, x0_dev, lambda0_dev, x_out_dev, lambda_out_dev, result);
}

int absorber_batch_solve(absorber_t* H, const absorber_ipm_options* opts, const double* x0_dev,
                         const double* lambda0_dev, double* x_out_dev, double* lambda_out_dev,
                         absorber_ipm_result* results) {
  if (!H || !results) {
    set_error("absorber_batch_solve: bad argument");
    return ABS_ERR_ARG;
  }
  absorber_ipm_options o;
  const int rc = check_options(opts, &o, "absorber_batch_solve");
  if (rc) return rc;
  return solve_with_restart(H->h, o, x0_dev, lambda0_dev, x_out_dev, lambda_out_dev, results);
}

int absorber_tuning_get(const absorber_t* H, absorber_tuning* out) {
  if (!H || !out) {
    set_error("absorber_tuning_get: bad argument");
    return ABS_ERR_ARG;
  }
  const Tune& t = H->h.tune;
  out->tuned = t.done;
  out->factor_waves_per_simd = t.factor_wpe;
  out->factor_row_split = t.factor_split;
  out->solve_waves_per_simd = t.solve_wpe;
  out->eval_block = t.eval_bs;
  for (int i = 0; i < 3; ++i) {
    out->factor_ms[0][i] = t.ms_factor[0][i];
    out->factor_ms[1][i] = t.ms_factor[1][i];
    out->solve_ms[i] = t.ms_solve[i];
    out->eval_ms[i] = t.ms_eval[i];
  }
  return ABS_OK;
}

int absorber_tuning_set(absorber_t* H, const absorber_tuning* in) {
  if (!H || !in || (in->factor_waves_per_simd != 2 && in->factor_waves_per_simd != 3) || in->factor_row_split < 0 ||
      in->factor_row_split > 2 || in->solve_waves_per_simd < 2 || in->solve_waves_per_simd > 4 ||
      (in->eval_block != 64 && in->eval_block != 128 && in->eval_block != 256)) {
    set_error("absorber_tuning_set: bad argument");
    return ABS_ERR_ARG;
  }
  Tune& t = H->h.tune;
  t.factor_wpe = in->factor_waves_per_simd;
  t.factor_split = in->factor_row_split;
  t.solve_wpe = in->solve_waves_per_simd;
  t.eval_bs = in->eval_block;
  t.done = true;
  return ABS_OK;
}

int absorber_ipm_log_get(const absorber_t* H, int32_t problem, int32_t max_entries, absorber_ipm_log_entry* out,
                         int32_t* n_out) {
  if (!H || problem < 0 || problem >= H->h.P || max_entries < 0 || (max_entries > 0 && !out)) {
    set_error("absorber_ipm_log_get: bad argument");
    return ABS_ERR_ARG;
  }
  const Handle& h = H->h;
  const std::vector<absorber_ipm_log_entry>* log =
      (size_t)problem < h.ipm_log.size() ? &h.ipm_log[(size_t)problem] : nullptr;
  const int n = log ? (int)log->size() : 0;
  for (int i = 0; i < n && i < max_entries; ++i) out[i] = (*log)[(size_t)i];
  if (n_out) *n_out = n;
  return ABS_OK;
}

int absorber_kkt_solve(absorber_t* H, const double* rhs_dev, double* sol_dev, double* rel_resid_host, void* stream) {
  if (!H || !rhs_dev || !sol_dev) {
    set_error("absorber_kkt_solve: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  if (h.P != 1) {
    set_error("absorber_kkt_solve: single-problem handles only");
    return ABS_ERR_ARG;
  }
  if (!h.factored) {
    set_error("absorber_kkt_solve: no factorisation (call absorber_kkt_factor first)");
    return ABS_ERR_STATE;
  }
  double rel = 0.0;
  const int rc = kkt_solve_refined(h, rhs_dev, sol_dev, false, &rel, (hipStream_t)stream);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  if (rel_resid_host) *rel_resid_host = rel;
  return ABS_OK;
}

}  // extern "C"
