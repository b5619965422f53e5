// HIP kernels for gfx950: stage evaluation (SIMD over scenario x stage), the
// residual of the bordered KKT system, and the launch-shape autotuner.  The
// block LDL^T, the stored-factor solve and the Schur complement on the shared
// diameter are in factor.hip.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <functional>

#include "internal.h"

namespace absorber {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// ---------------------------------------------------------------- evaluation
struct RecSink {
  double* rec;
  const double* cs;  // 22 row scales of this stage
  const double* D;   // 21 variable scales
  double Dd;
  int no = 0, nu = 0, nd = 0;
  __device__ void operator()(int r, int blk, int col, double v) {
    const double s = cs[r] * v;
    if (blk == BLK_OWN) rec[REC_OWN + no++] = s * D[col];
    else if (blk == BLK_D) rec[REC_OWN + no++] = s * Dd;
    else if (blk == BLK_UP) rec[REC_UP + nu++] = s * D[col];
    else rec[REC_DOWN + nd++] = s * D[col];
  }
};

struct CooSink {
  double* vals;
  int k = 0;
  __device__ void operator()(int, int, int, double v) { vals[k++] = v; }
};

struct RowMaxSink {
  double* m;  // 22
  const double* D;
  double Dd;
  __device__ void operator()(int r, int blk, int col, double v) {
    const double a = fabs(v) * (blk == BLK_D ? Dd : D[col]);
    if (a > m[r]) m[r] = a;
  }
};

__device__ __forceinline__ void load_stage(const double* __restrict__ x, const Scaling& sc, int scaled,
                                           long long t, double* z) {
  const double* p = x + t * NV;
#pragma unroll
  for (int k = 0; k < NV; ++k) z[k] = scaled ? p[k] * sc.D[k] : p[k];
}

__device__ __forceinline__ void load_inflow(const double* __restrict__ x, const Scaling& sc, int scaled,
                                            long long t, int n, int N, const double* feed, Inflow& f) {
  if (n < N - 1) {
    const double* p = x + (t + 1) * NV;
    f.L_up = scaled ? p[IL] * sc.D[IL] : p[IL];
    for (int i = 0; i < 9; ++i) f.x_up[i] = scaled ? p[i] * sc.D[i] : p[i];
    f.T_up = scaled ? p[IT] * sc.D[IT] : p[IT];
  } else {
    f.L_up = feed[6];
    for (int i = 0; i < 9; ++i) f.x_up[i] = feed[7 + i];
    f.T_up = feed[16];
  }
  if (n > 0) {
    const double* p = x + (t - 1) * NV;
    f.V_dn = scaled ? p[IV] * sc.D[IV] : p[IV];
    for (int j = 0; j < 4; ++j) f.y_dn[j] = scaled ? p[IY + j] * sc.D[IY + j] : p[IY + j];
    f.T_dn = scaled ? p[IT] * sc.D[IT] : p[IT];
  } else {
    f.V_dn = feed[0];
    for (int j = 0; j < 4; ++j) f.y_dn[j] = feed[1 + j];
    f.T_dn = feed[5];
  }
}

// One thread per stage: residuals (scaled by cs) and, if full, the scaled stage
// record: Jacobian blocks and the Lagrangian Hessian block.
__global__ __launch_bounds__(256) void k_eval(const double* __restrict__ x, Scaling sc, int scaled, const double* __restrict__ y,
                       const double* __restrict__ cs, const double* __restrict__ feeds, ModelParams p,
                       const StageInfo* __restrict__ sinfo, long long nst, const int* __restrict__ pact, int full,
                       int npar, double* __restrict__ cout, double* __restrict__ rec) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nst) return;
  const StageInfo si = sinfo[t];
  if (pact && !pact[si.p]) return;  // problem not being worked on
  const int n = si.n, N = si.N;
  const double* feed = feeds + (long long)si.w * NF;
  double z[NV];
  load_stage(x, sc, scaled, t, z);
  Inflow f;
  load_inflow(x, sc, scaled, t, n, N, feed, f);
  // the diameter of this stage's section
  const long long xd = nst * NV + (long long)si.p * npar + section_of(n, N, npar);
  const double d = scaled ? x[xd] * sc.Dd : x[xd];
  const double P = stage_pressure(p, feed[17], n, N);
  double csr[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) csr[r] = cs ? cs[t * NR + r] : 1.0;
  double c[NR];
  stage_residuals(p, z, f, P, d, c);
#pragma unroll
  for (int r = 0; r < NR; ++r) cout[t * NR + r] = csr[r] * c[r];
  if (!full) return;
  double* R = rec + t * REC;
  RecSink sink{R, csr, sc.D, sc.Dd};
  stage_jacobian(p, z, f, P, d, n < N - 1, n > 0, sink);
  double lam[NR], lamd[NR], lamu[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    lam[r] = y ? y[t * NR + r] * csr[r] : 0.0;
    lamd[r] = (y && n > 0) ? y[(t - 1) * NR + r] * (cs ? cs[(t - 1) * NR + r] : 1.0) : 0.0;
    lamu[r] = (y && n < N - 1) ? y[(t + 1) * NR + r] * (cs ? cs[(t + 1) * NR + r] : 1.0) : 0.0;
  }
  double H[NH];
  stage_hessian(p, z, P, n > 0 ? lamd : nullptr, lam, n < N - 1 ? lamu : nullptr, H);
  HessPos pos[NH];
  hess_positions(pos);
#pragma unroll
  for (int e = 0; e < NH; ++e) R[REC_H + e] = H[e] * sc.D[pos[e].r] * sc.D[pos[e].c];
  R[REC_WDD] = hess_dd(p, lam[NR - 1]) * sc.Dd * sc.Dd;
}

// maximum |d c~_r / d xt| over the whole row (for gradient-based row scaling)
__global__ __launch_bounds__(128) void k_rowmax(const double* __restrict__ x, Scaling sc, int scaled, const double* __restrict__ feeds,
                         ModelParams p, const StageInfo* __restrict__ sinfo, long long nst, int npar,
                         double* __restrict__ rowmax) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nst) return;
  const StageInfo si = sinfo[t];
  const int n = si.n, N = si.N;
  const double* feed = feeds + (long long)si.w * NF;
  double z[NV];
  load_stage(x, sc, scaled, t, z);
  Inflow f;
  load_inflow(x, sc, scaled, t, n, N, feed, f);
  const long long xd = nst * NV + (long long)si.p * npar + section_of(n, N, npar);
  const double d = scaled ? x[xd] * sc.Dd : x[xd];
  double m[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) m[r] = 0.0;
  RowMaxSink sink{m, sc.D, sc.Dd};
  stage_jacobian(p, z, f, stage_pressure(p, feed[17], n, N), d, n < N - 1, n > 0, sink);
#pragma unroll
  for (int r = 0; r < NR; ++r) rowmax[t * NR + r] = m[r];
}

// unscaled Jacobian values in the compact structure order of the public ABI
__global__ __launch_bounds__(128) void k_jac_coo(const double* __restrict__ x, const double* __restrict__ feeds, ModelParams p, int N,
                          int S, double* __restrict__ vals) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int w = (int)(t / N), n = (int)(t % N);
  const double* feed = feeds + (long long)w * NF;
  Scaling sc{};
  double z[NV];
  load_stage(x, sc, 0, t, z);
  Inflow f;
  load_inflow(x, sc, 0, t, n, N, feed, f);
  const long long nx = (long long)N * S * NV;
  const long long per_scen = (long long)N * NJO + (long long)(N - 1) * (NJU + NJD);
  const long long off = (long long)w * per_scen + (long long)n * (NJO + NJU) + (long long)(n > 0 ? n - 1 : 0) * NJD;
  CooSink sink{vals + off};
  stage_jacobian(p, z, f, stage_pressure(p, feed[17], n, N), x[nx], n < N - 1, n > 0, sink);
}

// unscaled Lagrangian Hessian block values (48 per stage) of the public ABI
__global__ __launch_bounds__(128) void k_hess_coo(const double* __restrict__ x, const double* __restrict__ lam,
                           const double* __restrict__ feeds, ModelParams p, int N, int S, double* __restrict__ vals) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int w = (int)(t / N), n = (int)(t % N);
  const double* feed = feeds + (long long)w * NF;
  Scaling sc{};
  double z[NV];
  load_stage(x, sc, 0, t, z);
  double H[NH];
  stage_hessian(p, z, stage_pressure(p, feed[17], n, N), n > 0 ? lam + (t - 1) * NR : nullptr, lam + t * NR,
                n < N - 1 ? lam + (t + 1) * NR : nullptr, H);
#pragma unroll
  for (int e = 0; e < NH; ++e) vals[t * NH + e] = H[e];
}

// (d,d) Hessian entry: fixed-order sum over all hydraulic rows (one block)
__global__ void k_hess_dd(const double* __restrict__ lam, ModelParams p, long long nst, double* __restrict__ out) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (long long t = threadIdx.x; t < nst; t += blockDim.x) acc += hess_dd(p, lam[t * NR + NR - 1]);
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// the cold-start point: x0's stage vector in every stage, its diameter for every problem
struct TileX0 {
  double v[NV + 1];
};
// ndes: design entries (problems x sections)
__global__ void k_tile_x0(TileX0 x0, long long nst, long long ndes, double* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nst * NV) x[i] = x0.v[i % NV];
  else if (i < nst * NV + ndes) x[i] = x0.v[NV];
}

// z = y + a x (z may be y)
__global__ void k_axpy(double* z, const double* y, const double* __restrict__ x, double a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = y[i] + a * x[i];
}

// Residual of the bordered KKT system, res = rhs - K sol, and the componentwise
// backward error max_i |res_i| / (sum_j |K_ij sol_j| + |rhs_i|).  One block per
// IPM segment (at most SEG consecutive stages of one problem), one thread per
// (stage, row).  The block stages the segment's records and unknowns, plus one
// neighbour on each side, in LDS and each thread walks its row's term list
// (K_ij from a record or the diagonal, times an unknown of its stage, of a
// neighbour or d).  Threads are assigned rows in decreasing term count, so
// that the lanes of a wave walk lists of similar length.
// part[2 g] = sum over segment g of b_t . sol_hyd(t) and part[2 g + 1] its
// magnitude (for the d row); omb[3 g .. 3 g + 2] = the segment's largest
// backward error, largest |res_i| and largest |rhs_i|.
constexpr int RBS = ((NK * SEG + WAVE - 1) / WAVE) * WAVE;  // threads per block
constexpr int RDG = 24;                                      // diagonal coefficients per stage in LDS

__global__ __launch_bounds__(RBS) void k_residual(
    const double* __restrict__ rec, const int* __restrict__ rtab, int rtab_n, const double* __restrict__ diagx,
    const double* __restrict__ diags, const double* __restrict__ dwv, const double* __restrict__ dcv,
    const double* __restrict__ sol, const double* __restrict__ rhs, const Seg* __restrict__ segs,
    const StageInfo* __restrict__ sinfo, long long nst, const int* __restrict__ pact, long long nks, int jd,
    int npar, int zero_masked, double* __restrict__ res, double* __restrict__ part, double* __restrict__ omb) {
  __shared__ double cf[(SEG + 2) * REC + SEG * RDG];  // records of stages t0-1 .. t1, then diagonals
  __shared__ double sx[(SEG + 2) * NK];               // unknowns of the same stages
  __shared__ int tab[RT_MAX];
  __shared__ double dsum[2 * SEG];
  __shared__ double wred[3][RBS / WAVE];
  const int tid = threadIdx.x;
  const Seg sg = segs[blockIdx.x];
  const long long t0 = sg.t0;
  const int ns = sg.t1 - sg.t0;
  if (pact && !pact[sg.p]) {  // problem not being worked on: zero residual (rows on request)
    if (zero_masked)
      for (long long i = t0 * NK + tid; i < (long long)sg.t1 * NK; i += RBS) res[i] = 0.0;
    if (tid == 0) {
      part[2 * blockIdx.x] = 0.0;
      part[2 * blockIdx.x + 1] = 0.0;
      omb[3 * blockIdx.x] = 0.0;
      omb[3 * blockIdx.x + 1] = 0.0;
      omb[3 * blockIdx.x + 2] = 0.0;
    }
    return;
  }
  const double dw = dwv[sg.p], dc = dcv[sg.p];
  const long long la = t0 > 0 ? t0 - 1 : 0, lb = sg.t1 + 1 < nst ? sg.t1 + 1 : nst;
  const int s0 = (int)(la - (t0 - 1));  // LDS slot of stage la (slot s holds stage t0 - 1 + s)
  const int ncf = (int)(lb - la) * REC, nsx = (int)(lb - la) * NK;
  LdsStage<RBS, (SEG + 2) * REC, double> scf;
  LdsStage<RBS, (SEG + 2) * NK, double> ssx;
  LdsStage<RBS, RT_MAX, int> stb;
  scf.load(rec + la * REC, ncf, tid);
  ssx.load(sol + la * NK, nsx, tid);
  stb.load(rtab, rtab_n, tid);
  // every other load of the block goes out before the first LDS write too: the
  // diagonal coefficients (one per thread) and each (stage, row) thread's
  // stage data, diameter, row index and right-hand side
  // (indices clamped to the segment, so that no load waits behind a branch)
  static_assert(SEG * RDG <= RBS, "one diagonal coefficient per thread");
  const int dl = min(tid / RDG, ns - 1), dk = tid % RDG;
  double dgx = diagx[(t0 + dl) * NV + min(dk, NV - 1)], dgs = diags[t0 + dl];
  const int j = tid / SEG, ls = tid - j * SEG;
  const bool mine = j < NK && ls < ns;
  const long long tm = t0 + min(ls, ns - 1);
  const StageInfo si = sinfo[tm];
  const int row = rtab[min(j, NK - 1)];
  // the loads above complete together here (kept out of the selects below)
  __asm__ volatile("" : "+v"(dgx), "+v"(dgs));
  const double xd = sol[nks + (long long)sg.p * npar + section_of(si.n, si.N, npar)];  // its section's diameter
  const double r = rhs[tm * NK + row];
  const double dhyd = -(1.0 / (dgs + dw) + dc);
  const double dgv = dk < NV ? dgx + dw : (dk == NV ? -dc : (dk == NV + 1 ? dhyd : 0.0));
  scf.store(cf + s0 * REC, ncf, tid);
  ssx.store(sx + s0 * NK, nsx, tid);
  stb.store(tab, rtab_n, tid);
  if (tid < ns * RDG) cf[(SEG + 2) * REC + tid] = dgv;
  if (tid < 2 * SEG) dsum[tid] = 0.0;
  __syncthreads();
  double om = 0.0, rmax = 0.0, bmax = 0.0;
  if (mine) {
    const long long t = t0 + ls;
    const bool has_dn = si.n > 0, has_up = si.n < si.N - 1;
    const int s = ls + 1;
    const int cbase = s * REC - RT_COFF, dbase = (SEG + 2) * REC + ls * RDG - RT_DIAG, xbase = s * NK - RT_XOFF;
    const int* tl = tab + 2 * NK + 1;
    double y = 0.0, ya = 0.0;
    for (int q = tab[NK + j]; q < tab[NK + j + 1]; ++q) {
      const int c = tl[2 * q], xc = tl[2 * q + 1];
      const double cv = cf[c >= RT_DIAG ? dbase + c : cbase + c];
      const double xv = (xc & RT_XDTERM) ? xd : sx[xbase + (xc & (RT_XDTERM - 1))];
      // a neighbour that is not in the chain contributes nothing
      const bool ok = !(((xc & RT_NBDN) && !has_dn) || ((xc & RT_NBUP) && !has_up));
      const double pr = ok ? cv * xv : 0.0;
      y += pr;
      ya += fabs(pr);
    }
    const double rr = r - y;
    res[t * NK + row] = rr;
    const double den = ya + fabs(r);
    om = den > 0.0 ? fabs(rr) / den : (rr == 0.0 ? 0.0 : INFINITY);
    rmax = fabs(rr);
    bmax = fabs(r);
    if (!isfinite(rr)) om = rmax = INFINITY;  // maxima below ignore NaN: report it as infinite
    if (!isfinite(r)) bmax = INFINITY;
    if (row == NK - 1) {  // this stage's share of the d row: b . sol_hyd
      const double pr = cf[s * REC + jd] * sx[s * NK + NK - 1];
      dsum[2 * ls] = pr;
      dsum[2 * ls + 1] = fabs(pr);
    }
  }
  om = wave_reduce(1, om);
  rmax = wave_reduce(1, rmax);
  bmax = wave_reduce(1, bmax);
  if ((tid & (WAVE - 1)) == WAVE - 1) {
    wred[0][tid / WAVE] = om;
    wred[1][tid / WAVE] = rmax;
    wred[2][tid / WAVE] = bmax;
  }
  __syncthreads();
  if (tid < 3) {
    double m = 0.0;
    for (int i = 0; i < RBS / WAVE; ++i) m = fmax(m, wred[tid][i]);
    omb[3 * blockIdx.x + tid] = m;
  }
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int l = 0; l < ns; ++l) {  // fixed order
      a += dsum[2 * l];
      b += dsum[2 * l + 1];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// d row of each problem's residual (one block per problem, fixed order over
// its segments): res_d = rhs_d - sum b u_hyd - kdd u_d; omd[p] = its backward error
__global__ void k_residual_d(const double* __restrict__ part, const int* __restrict__ pseg,
                             const DevScalars* __restrict__ scv, const double* __restrict__ sol,
                             const double* __restrict__ rhs, long long nkk, const int* __restrict__ pact,
                             double* __restrict__ res, double* __restrict__ omd) {
  __shared__ double s1[256], s2[256];
  const int pb = blockIdx.x;
  if (pact && !pact[pb]) {
    if (threadIdx.x == 0) {
      res[nkk + pb] = 0.0;
      omd[3 * pb] = omd[3 * pb + 1] = omd[3 * pb + 2] = 0.0;
    }
    return;
  }
  double a = 0, b = 0;
  for (int g = pseg[pb] + threadIdx.x; g < pseg[pb + 1]; g += blockDim.x) {
    a += part[2 * g];
    b += part[2 * g + 1];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long long i = nkk + pb;
    const double kdd = scv[pb].kdd;
    const double ku = s1[0] + kdd * sol[i];
    const double ka = s2[0] + fabs(kdd * sol[i]);
    const double rr = rhs[i] - ku;
    res[i] = rr;
    const double den = ka + fabs(rhs[i]);
    const bool fin = isfinite(rr);
    omd[3 * pb] = !fin ? INFINITY : (den > 0.0 ? fabs(rr) / den : (rr == 0.0 ? 0.0 : INFINITY));
    omd[3 * pb + 1] = fin ? fabs(rr) : INFINITY;
    omd[3 * pb + 2] = isfinite(rhs[i]) ? fabs(rhs[i]) : INFINITY;
  }
}

// Design rows of each problem's residual for npar > 1 (one 1024-thread block per
// problem, fixed-order sums per section over its stages: thread i takes stages
// i, i + DBS, ..., then a shuffle tree in each wave and across the waves):
// res_k = rhs_k - sum over the section's stages of b u_hyd - K_dd,k u_k (K_dd
// diagonal from the Schur data); omd[3 p .. 3 p + 2] = the largest backward
// error, |res| and |rhs| of its rows.
constexpr int DBS = 1024;
__global__ __launch_bounds__(DBS) void k_residual_design(
    const double* __restrict__ rec, const long long* __restrict__ pstage, const StageInfo* __restrict__ sinfo,
    const double* __restrict__ dsc, const double* __restrict__ sol, const double* __restrict__ rhs, long long nks,
    int jd, int npar, const int* __restrict__ pact, double* __restrict__ res, double* __restrict__ omd) {
  __shared__ double sm[2 * MAX_NPAR][DBS / 64];
  const int pb = blockIdx.x;
  const long long d0 = nks + (long long)pb * npar;
  if (pact && !pact[pb]) {
    if (threadIdx.x < npar) res[d0 + threadIdx.x] = 0.0;
    if (threadIdx.x == 0) omd[3 * pb] = omd[3 * pb + 1] = omd[3 * pb + 2] = 0.0;
    return;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double a[2 * MAX_NPAR] = {0, 0, 0, 0, 0, 0, 0, 0};  // sums of b u and of |b u| per section
  for (long long t = pstage[pb] + threadIdx.x; t < pstage[pb + 1]; t += DBS) {
    const StageInfo si = sinfo[t];
    const int k = section_of(si.n, si.N, npar);
    const double pr = rec[t * REC + jd] * sol[t * NK + NK - 1];
#pragma unroll
    for (int q = 0; q < MAX_NPAR; ++q) {
      a[q] += q == k ? pr : 0.0;
      a[MAX_NPAR + q] += q == k ? fabs(pr) : 0.0;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < 2 * MAX_NPAR; ++q) a[q] += __shfl_down(a[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 2 * MAX_NPAR; ++q) sm[q][wv] = a[q];
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int q = 0; q < 2 * MAX_NPAR; ++q) {
    a[q] = lane < DBS / 64 ? sm[q][lane] : 0.0;
#pragma unroll
    for (int off = DBS / 128; off > 0; off >>= 1) a[q] += __shfl_down(a[q], off, 64);
  }
  if (lane == 0) {
    const double* D = dsc + (long long)pb * DSC;
    const double* kdiag = D + MAX_NPAR * MAX_NPAR + 2 * MAX_NPAR;
    double om = 0.0, rm = 0.0, bm = 0.0;
#pragma unroll
    for (int k = 0; k < MAX_NPAR; ++k) {
      if (k >= npar) break;
      const long long i = d0 + k;
      const double ku = a[k] + kdiag[k] * sol[i];
      const double ka = a[MAX_NPAR + k] + fabs(kdiag[k] * sol[i]);
      const double rr = rhs[i] - ku;
      res[i] = rr;
      const double den = ka + fabs(rhs[i]);
      const bool fin = isfinite(rr);
      om = fmax(om, !fin ? INFINITY : (den > 0.0 ? fabs(rr) / den : (rr == 0.0 ? 0.0 : INFINITY)));
      rm = fmax(rm, fin ? fabs(rr) : INFINITY);
      bm = fmax(bm, isfinite(rhs[i]) ? fabs(rhs[i]) : INFINITY);
    }
    omd[3 * pb] = om;
    omd[3 * pb + 1] = rm;
    omd[3 * pb + 2] = bm;
  }
}

// out[0] = largest backward error over the segments, out[1] over the problems'
// d rows, out[2] = largest |res_i| and out[3] = largest |rhs_i| over both.  One
// block of MAX_BS threads, four segments' loads in flight per thread, then a
// shuffle tree in each wave and across the waves (maxima: order-free).
constexpr int MAX_BS = 1024;
__global__ __launch_bounds__(MAX_BS) void k_residual_max(const double* __restrict__ omb, int G,
                                                         const double* __restrict__ omd, int P,
                                                         double* __restrict__ out) {
  __shared__ double sm[4][MAX_BS / 64];
  double m[4] = {0, 0, 0, 0};  // a, b, r, q
  int i = threadIdx.x;
  for (; i + 3 * MAX_BS < G; i += 4 * MAX_BS) {
    double v[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) v[j][k] = omb[3LL * (i + j * MAX_BS) + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      m[0] = fmax(m[0], v[j][0]);
      m[2] = fmax(m[2], v[j][1]);
      m[3] = fmax(m[3], v[j][2]);
    }
  }
  for (; i < G; i += MAX_BS) {
    m[0] = fmax(m[0], omb[3LL * i]);
    m[2] = fmax(m[2], omb[3LL * i + 1]);
    m[3] = fmax(m[3], omb[3LL * i + 2]);
  }
  for (int p = threadIdx.x; p < P; p += MAX_BS) {
    m[1] = fmax(m[1], omd[3 * p]);
    m[2] = fmax(m[2], omd[3 * p + 1]);
    m[3] = fmax(m[3], omd[3 * p + 2]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) m[k] = wave_reduce(1, m[k]);
  if (lane == 63)
    for (int k = 0; k < 4; ++k) sm[k][wv] = m[k];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double v = wave_reduce(1, lane < MAX_BS / 64 ? sm[k][lane] : 0.0);
      if (lane == 63) out[k] = v;
    }
  }
}

// per problem (one block each): the largest |res_i| and |rhs_i| over its
// segments' partials and its d row
__global__ __launch_bounds__(256) void k_residual_pmax(const double* __restrict__ omb, const int* __restrict__ pseg,
                                                       const double* __restrict__ omd, double* __restrict__ out) {
  __shared__ double sm[2][4];
  const int p = blockIdx.x;
  double r = 0.0, q = 0.0;
  for (int g = pseg[p] + (int)threadIdx.x; g < pseg[p + 1]; g += 256) {
    r = fmax(r, omb[3LL * g + 1]);
    q = fmax(q, omb[3LL * g + 2]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    r = fmax(r, __shfl_down(r, off, 64));
    q = fmax(q, __shfl_down(q, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = r;
    sm[1][threadIdx.x >> 6] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    r = fmax(omd[3 * p + 1], fmax(fmax(sm[0][0], sm[0][1]), fmax(sm[0][2], sm[0][3])));
    q = fmax(omd[3 * p + 2], fmax(fmax(sm[1][0], sm[1][1]), fmax(sm[1][2], sm[1][3])));
    out[2 * p] = r;
    out[2 * p + 1] = q;
  }
}

// res_i = 0 on the stage rows and the d row of the problems with mask 0
__global__ void k_copy_rows(const int* __restrict__ mask, const StageInfo* __restrict__ sinfo, long long nks, int P,
                            int npar, double* __restrict__ dst, const double* __restrict__ src) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nks) {
    if (mask[sinfo[i / NK].p]) dst[i] = src[i];
  } else if (i < nks + (long long)P * npar) {
    if (mask[(i - nks) / npar]) dst[i] = src[i];
  }
}

// z = y + a x on the rows of the problems in mask (stage rows and design rows)
__global__ void k_axpy_rows(const int* __restrict__ mask, const StageInfo* __restrict__ sinfo, long long nks, int P,
                            int npar, double* z, const double* y, const double* __restrict__ x, double a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nks) {
    if (mask[sinfo[i / NK].p]) z[i] = y[i] + a * x[i];
  } else if (i < nks + (long long)P * npar) {
    if (mask[(i - nks) / npar]) z[i] = y[i] + a * x[i];
  }
}

inline unsigned grid_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------- launch wrappers
hipError_t launch_eval(Handle& h, const double* x, int scaled, const double* y, int full, double* c_out,
                       hipStream_t st) {
  return launch_eval_ext(h, x, scaled, h.sc, h.cs, y, full, c_out, st);
}

hipError_t launch_eval_ext(Handle& h, const double* x, int scaled, const Scaling& sc, const double* cs,
                           const double* y, int full, double* c_out, hipStream_t st) {
  prof_begin(h, 2, st);
  const int bs = h.tune.eval_bs;
  hipLaunchKernelGGL(k_eval, dim3(grid_for(h.nst, bs)), dim3(bs), 0, st, x, sc, scaled, y, cs, h.feeds, h.mp,
                     h.sinfo, h.nst, h.pact_on ? h.pact : nullptr, full, h.npar, c_out, h.rec);
  prof_end(h, 2, st);
  return hipGetLastError();
}

hipError_t launch_rowmax(Handle& h, const double* x, int scaled, double* rowmax, hipStream_t st) {
  hipLaunchKernelGGL(k_rowmax, dim3(grid_for(h.nst, 128)), dim3(128), 0, st, x, h.sc, scaled, h.feeds, h.mp, h.sinfo,
                     h.nst, h.npar, rowmax);
  return hipGetLastError();
}

hipError_t launch_jac_coo(Handle& h, const double* x, double* vals, hipStream_t st) {
  const long long nst = (long long)h.N * h.S;
  hipLaunchKernelGGL(k_jac_coo, dim3(grid_for(nst, 128)), dim3(128), 0, st, x, h.feeds, h.mp, h.N, h.S, vals);
  return hipGetLastError();
}

hipError_t launch_hess_coo(Handle& h, const double* x, const double* lam, double* vals, hipStream_t st) {
  const long long nst = (long long)h.N * h.S;
  hipLaunchKernelGGL(k_hess_coo, dim3(grid_for(nst, 128)), dim3(128), 0, st, x, lam, h.feeds, h.mp, h.N, h.S,
                     vals);
  hipLaunchKernelGGL(k_hess_dd, dim3(1), dim3(256), 0, st, lam, h.mp, nst, vals + nst * NH);
  return hipGetLastError();
}

// Launch-shape tuning by measurement on the handle's own data: the occupancy
// target (waves per SIMD: 2, 3 or 4, which sets the register budget) of the
// factorisation and of the stored-factor solve, and the block size of the
// stage evaluation.  Each candidate runs twice on the current records (the
// launches are idempotent) and the fastest median is kept.
static float time_launch(hipStream_t st, hipEvent_t e0, hipEvent_t e1, const std::function<void()>& f) {
  float best = 1e30f;
  for (int r = 0; r < 2; ++r) {
    (void)hipEventRecord(e0, st);
    f();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = fminf(best, ms);
  }
  return best;
}

int autotune(Handle& h, const double* x, const double* y, double* c, const double* diagx, const double* diags,
             const double* rhs, hipStream_t st) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int prof = h.prof;
  h.prof = 0;
  const int bss[3] = {64, 128, 256};
  for (int i = 0; i < 3; ++i) {
    h.tune.eval_bs = bss[i];
    h.tune.ms_eval[i] = time_launch(st, e0, e1, [&] { (void)launch_eval(h, x, 1, y, 1, c, st); });
  }
  // The chain kernels are timed on at most TUNE_CHAINS chains (four rounds of the
  // wave slots at 3 waves/SIMD): enough for the steady state, and the tuning of a
  // large batch then costs a fraction of one factorisation per candidate.
  constexpr int TUNE_CHAINS = 4 * 3 * 4 * 256;
  // block LDL^T launch shapes: occupancy target x row split of the trailing update
  const int wpes[3] = {2, 3, 4};
  int best_w = 1, best_s = 0;
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 3; ++k) {
      h.tune.factor_wpe = wpes[i];
      h.tune.factor_split = k;
      h.tune.ms_factor[i][k] =
          time_launch(st, e0, e1, [&] { (void)launch_factor(h, diagx, diags, rhs, false, st, TUNE_CHAINS); });
      if (h.tune.ms_factor[i][k] < h.tune.ms_factor[best_w][best_s]) {
        best_w = i;
        best_s = k;
      }
    }
  for (int i = 0; i < 3; ++i) {
    h.tune.solve_wpe = wpes[i];
    h.tune.ms_solve[i] = time_launch(st, e0, e1, [&] { (void)launch_solve(h, rhs, st, TUNE_CHAINS); });
  }
  auto argmin = [](const float* v) { return v[0] <= v[1] ? (v[0] <= v[2] ? 0 : 2) : (v[1] <= v[2] ? 1 : 2); };
  h.tune.eval_bs = bss[argmin(h.tune.ms_eval)];
  h.tune.factor_wpe = wpes[best_w];
  h.tune.factor_split = best_s;
  h.tune.solve_wpe = wpes[argmin(h.tune.ms_solve)];
  h.tune.done = true;
  h.prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  return ABS_OK;
}

hipError_t launch_residual(Handle& h, const double* diagx, const double* diags, const double* sol,
                           const double* rhs, double* res, double* omega_out, hipStream_t st, bool zero_masked) {
  const long long nks = h.nst * NK;
  const int* pa = h.pact_on ? h.pact : nullptr;
  const int nb = h.nseg;
  double* part = h.kden;            // 2 per segment
  double* omb = h.kden + 2LL * nb;  // 3 per segment
  double* omd = omb + 3LL * nb;     // 3 per problem
  prof_begin(h, 3, st);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(RBS), 0, st, h.rec, h.rtab, h.rtab_n, diagx, diags, h.dwv, h.dcv, sol,
                     rhs, h.seg, h.sinfo, h.nst, pa, nks, h.jac_d_index, h.npar, zero_masked ? 1 : 0, res, part, omb);
  prof_end(h, 3, st);
  if (h.npar == 1)
    hipLaunchKernelGGL(k_residual_d, dim3(h.P), dim3(256), 0, st, part, h.pseg, h.scal, sol, rhs, nks, pa, res, omd);
  else
    hipLaunchKernelGGL(k_residual_design, dim3(h.P), dim3(DBS), 0, st, h.rec, h.pstage, h.sinfo, h.dsc, sol, rhs,
                       nks, h.jac_d_index, h.npar, pa, res, omd);
  hipLaunchKernelGGL(k_residual_max, dim3(1), dim3(MAX_BS), 0, st, omb, nb, omd, h.P, omega_out);
  return hipGetLastError();
}

hipError_t launch_residual_pmax(Handle& h, hipStream_t st) {
  const int nb = h.nseg;
  const double* omb = h.kden + 2LL * nb;
  const double* omd = omb + 3LL * nb;
  hipLaunchKernelGGL(k_residual_pmax, dim3(h.P), dim3(256), 0, st, omb, h.pseg, omd, h.pres);
  return hipGetLastError();
}

hipError_t launch_copy_rows(Handle& h, const int* mask, double* dst, const double* src, hipStream_t st) {
  const long long nks = h.nst * NK;
  hipLaunchKernelGGL(k_copy_rows, dim3(grid_for(h.nkkt, 256)), dim3(256), 0, st, mask, h.sinfo, nks, h.P, h.npar,
                     dst, src);
  return hipGetLastError();
}

hipError_t launch_tile_x0(Handle& h, double* x, hipStream_t st) {
  TileX0 a;
  for (int k = 0; k <= NV; ++k) a.v[k] = h.x0[k];
  hipLaunchKernelGGL(k_tile_x0, dim3(grid_for(h.nx, 256)), dim3(256), 0, st, a, h.nst, (long long)h.P * h.npar, x);
  return hipGetLastError();
}

hipError_t launch_axpy(double* z, const double* y, const double* x, double a, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, st, z, y, x, a, n);
  return hipGetLastError();
}

hipError_t launch_axpy_rows(Handle& h, const int* mask, double* z, const double* y, const double* x, double a,
                            hipStream_t st) {
  const long long nks = h.nst * NK;
  hipLaunchKernelGGL(k_axpy_rows, dim3(grid_for(h.nkkt, 256)), dim3(256), 0, st, mask, h.sinfo, nks, h.P, h.npar, z,
                     y, x, a);
  return hipGetLastError();
}

}  // namespace absorber
