// HIP kernels for gfx950: stage evaluation (SIMD over scenario x stage), the
// per-scenario block LDL^T of the primal-dual KKT system (one wavefront per
// scenario), the Schur complement on the shared diameter and the residual of
// the bordered system.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace absorber {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// deterministic wave sum (xor butterfly: every lane ends with the same bits)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 1; m < WAVE; m <<= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

// wave arg-max of non-negative values (ties -> lowest lane); returns the max and its lane
__device__ __forceinline__ double wave_argmax(double v, int& idx) {
  if (!(v == v)) v = INFINITY;  // a NaN must not make the result lane-dependent
  int i = lane_id();
#pragma unroll
  for (int m = 1; m < WAVE; m <<= 1) {
    const double ov = __shfl_xor(v, m, WAVE);
    const int oi = __shfl_xor(i, m, WAVE);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  idx = i;
  return v;
}

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

// One thread per (scenario, stage): residuals (scaled by cs) and, if full, the
// scaled stage record: Jacobian blocks and the Lagrangian Hessian block.
__global__ void k_eval(const double* __restrict__ x, Scaling sc, int scaled, const double* __restrict__ y,
                       const double* __restrict__ cs, const double* __restrict__ feeds, ModelParams p, int N,
                       int S, int full, double* __restrict__ cout, double* __restrict__ rec) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int w = (int)(t / N), n = (int)(t % N);
  const double* feed = feeds + (long long)w * NF;
  double z[NV];
  load_stage(x, sc, scaled, t, z);
  Inflow f;
  load_inflow(x, sc, scaled, t, n, N, feed, f);
  const long long nx = (long long)N * S * NV;
  const double d = scaled ? x[nx] * sc.Dd : x[nx];
  const double P = feed[17];
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
__global__ void k_rowmax(const double* __restrict__ x, Scaling sc, int scaled, const double* __restrict__ feeds,
                         ModelParams p, int N, int S, double* __restrict__ rowmax) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int w = (int)(t / N), n = (int)(t % N);
  const double* feed = feeds + (long long)w * NF;
  double z[NV];
  load_stage(x, sc, scaled, t, z);
  Inflow f;
  load_inflow(x, sc, scaled, t, n, N, feed, f);
  const long long nx = (long long)N * S * NV;
  const double d = scaled ? x[nx] * sc.Dd : x[nx];
  double m[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) m[r] = 0.0;
  RowMaxSink sink{m, sc.D, sc.Dd};
  stage_jacobian(p, z, f, feed[17], d, n < N - 1, n > 0, sink);
#pragma unroll
  for (int r = 0; r < NR; ++r) rowmax[t * NR + r] = m[r];
}

// unscaled Jacobian values in the compact structure order of the public ABI
__global__ void k_jac_coo(const double* __restrict__ x, const double* __restrict__ feeds, ModelParams p, int N,
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
  stage_jacobian(p, z, f, feed[17], x[nx], n < N - 1, n > 0, sink);
}

// unscaled Lagrangian Hessian block values (48 per stage) of the public ABI
__global__ void k_hess_coo(const double* __restrict__ x, const double* __restrict__ lam,
                           const double* __restrict__ feeds, ModelParams p, int N, int S, double* __restrict__ vals) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int w = (int)(t / N), n = (int)(t % N);
  const double* feed = feeds + (long long)w * NF;
  Scaling sc{};
  double z[NV];
  load_stage(x, sc, 0, t, z);
  double H[NH];
  stage_hessian(p, z, feed[17], n > 0 ? lam + (t - 1) * NR : nullptr, lam + t * NR,
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

// ---------------------------------------------------------------- block LDL^T
// Frontal matrix of stage n held one column per lane: lane j owns column j,
// v[i] is row i.  Columns/rows 0-42 are the stage's KKT unknowns, 43-58 the
// coupling unknowns of stage n+1, 59 the right-hand side r, 60 the border b
// (both carried as symmetric extra rows and columns).  Eliminating the 43 own
// pivots leaves in rows/cols 43-60 the contribution to stage n+1's block and
// right-hand sides.
struct WaveLDS {
  double src[NSRC];
  double cb0[WAVE];
  double cb1[WAVE];
  double xr[WAVE];
  double xb[WAVE];
};

__device__ __forceinline__ void bcast_col(const double (&v)[FR], int k, double* buf) {
  if (lane_id() == k) {
#pragma unroll
    for (int i = 0; i < FR; ++i) buf[i] = v[i];
  }
  __syncthreads();
}

__device__ __forceinline__ bool row_active(uint64_t act, int i, int p0, int p1) {
  return i < NK ? ((((act >> i) & 1ull) != 0ull) && i != p0 && i != p1) : true;
}

template <int WITH_RHS>
__global__ __launch_bounds__(WAVE) void k_factor(const double* __restrict__ rec, const int* __restrict__ gather,
                                                 const double* __restrict__ rhs, const double* __restrict__ diagx,
                                                 const double* __restrict__ diags, double dw, double dc, int N, int S,
                                                 int jd, double* __restrict__ slots, double* __restrict__ solr,
                                                 double* __restrict__ solb, int* __restrict__ inert,
                                                 double* __restrict__ part) {
  __shared__ WaveLDS L;
  const int w = blockIdx.x;
  if (w >= S) return;
  const int lane = lane_id();
  const double alpha = (1.0 + sqrt(17.0)) * 0.125;
  for (int i = lane; i < NC * (NC + 2); i += WAVE) L.src[SRC_CTB + i] = 0.0;
  if (lane == 0) L.src[SRC_ZERO] = 0.0;
  long long npos = 0, nneg = 0, nzero = 0;
  double v[FR];
  for (int n = 0; n < N; ++n) {
    const long long t = (long long)w * N + n;
    const double* R = rec + t * REC;
    for (int i = lane; i < REC; i += WAVE) L.src[SRC_REC + i] = R[i];
    if (lane < NJD) L.src[SRC_DOWN1 + lane] = (n < N - 1) ? rec[(t + 1) * REC + REC_DOWN + lane] : 0.0;
    if (lane < NK) L.src[SRC_RHS + lane] = WITH_RHS ? rhs[t * NK + lane] : 0.0;
    if (lane < NV) L.src[SRC_DIAGX + lane] = diagx[t * NV + lane] + dw;
    if (lane == 0) {
      L.src[SRC_BRD] = R[jd];
      L.src[SRC_DC] = -dc;
      L.src[SRC_DHYD] = -(1.0 / (diags[t] + dw) + dc);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FR; ++i) {
      const int g = gather[i * WAVE + lane];
      v[i] = L.src[g & 1023] + L.src[(g >> 10) & 1023] + L.src[(g >> 20) & 1023];
    }
    __syncthreads();
    double* sb = slots + t * NK * SLOT;
    uint64_t act = (1ull << NK) - 1ull;
    int slot = 0;
    while (act) {
      const int k = __builtin_ctzll(act);
      bcast_col(v, k, L.cb0);
      const double ck = lane < FR ? L.cb0[lane] : 0.0;
      const double akk = fabs(L.cb0[k]);
      int r;
      const bool oa = lane < NK && ((act >> lane) & 1ull) && lane != k;
      const double lam = wave_argmax(oa ? fabs(ck) : 0.0, r);
      int ptype;  // 1: 1x1 at k, 2: 1x1 at r, 3: 2x2 (k, r)
      if (akk >= alpha * lam || lam == 0.0) {
        ptype = 1;
      } else {
        bcast_col(v, r, L.cb1);
        const double cr = lane < FR ? L.cb1[lane] : 0.0;
        int r2;
        const bool ob = lane < NK && ((act >> lane) & 1ull) && lane != r;
        const double sig = wave_argmax(ob ? fabs(cr) : 0.0, r2);
        if (akk * sig >= alpha * lam * lam) ptype = 1;
        else if (fabs(L.cb1[r]) >= alpha * sig) ptype = 2;
        else ptype = 3;
      }
      if (ptype != 3) {
        const int p = ptype == 1 ? k : r;
        const double* buf = ptype == 1 ? L.cb0 : L.cb1;
        const double d = buf[p];
        const double cj = lane < FR ? buf[lane] : 0.0;
        const bool ra = lane < FR && row_active(act, lane, p, -1);
        // store the pivot column (rows still active, the pivot row cleared)
        double sv;
        if (lane < FR) sv = ra ? cj : 0.0;
        else if (lane == FR) sv = (double)(p + 64 * (d == 0.0 ? 0 : 1));
        else if (lane == FR + 1) sv = d;
        else sv = 0.0;
        sb[slot * SLOT + lane] = sv;
        if (d == 0.0) {
          ++nzero;
        } else {
          if (d > 0.0) ++npos; else ++nneg;
          const double t1 = ra ? cj / d : 0.0;
#pragma unroll
          for (int i = 0; i < FR; ++i)
            if (row_active(act, i, p, -1)) v[i] -= buf[i] * t1;
        }
        act &= ~(1ull << p);
        slot += 1;
      } else {
        const double e11 = L.cb0[k], e12 = L.cb0[r], e22 = L.cb1[r];
        const double det = e11 * e22 - e12 * e12;
        const double c0 = lane < FR ? L.cb0[lane] : 0.0;
        const double c1 = lane < FR ? L.cb1[lane] : 0.0;
        const bool ra = lane < FR && row_active(act, lane, k, r);
        double s0, s1;
        if (lane < FR) {
          s0 = ra ? c0 : 0.0;
          s1 = ra ? c1 : 0.0;
        } else if (lane == FR) {
          s0 = (double)(k + 64 * 2);
          s1 = (double)(r + 64 * 3);
        } else if (lane == FR + 1) {
          s0 = e11;
          s1 = e22;
        } else {
          s0 = e12;
          s1 = e12;
        }
        sb[slot * SLOT + lane] = s0;
        sb[(slot + 1) * SLOT + lane] = s1;
        if (det < 0.0) {
          ++npos;
          ++nneg;
        } else if (det > 0.0) {
          if (e11 + e22 > 0.0) npos += 2; else nneg += 2;
        } else {
          nzero += 2;
        }
        const double i11 = e22 / det, i12 = -e12 / det, i22 = e11 / det;
        const double t1 = ra ? i11 * c0 + i12 * c1 : 0.0;
        const double t2 = ra ? i12 * c0 + i22 * c1 : 0.0;
#pragma unroll
        for (int i = 0; i < FR; ++i)
          if (row_active(act, i, k, r)) v[i] -= L.cb0[i] * t1 + L.cb1[i] * t2;
        act &= ~((1ull << k) | (1ull << r));
        slot += 2;
      }
      __syncthreads();
    }
    // contribution block to stage n+1 (rows/cols 43..60 of the coupling lanes)
    if (lane >= NK && lane < NK + NC) {
      const int a = lane - NK;
#pragma unroll
      for (int b = 0; b < NC + 2; ++b) L.src[SRC_CTB + a * (NC + 2) + b] = v[NK + b];
    }
    __syncthreads();
  }
  // ---------------- backward substitution over the stages, top to bottom
  double xr = 0.0, xb = 0.0, sigb = 0.0, sigr = 0.0, wdd = 0.0;
  for (int n = N - 1; n >= 0; --n) {
    const long long t = (long long)w * N + n;
    const double* sb = slots + t * NK * SLOT;
    if (lane < NK) {
      xr = 0.0;
      xb = 0.0;
    }
    for (int s = NK - 1; s >= 0; --s) {
      const double c = sb[s * SLOT + lane];
      const int code = (int)__shfl(c, FR, WAVE);
      const int type = code >> 6, p = code & 63;
      const double cr = lane < FR_R ? c : 0.0;
      if (type == 1 || type == 0) {
        const double yr = __shfl(c, FR_R, WAVE), yb = __shfl(c, FR_B, WAVE);
        const double d = __shfl(c, FR + 1, WAVE);
        const double pr = wave_sum(cr * xr), pb = wave_sum(cr * xb);
        if (lane == p) {
          xr = type ? (yr - pr) / d : 0.0;
          xb = type ? (yb - pb) / d : 0.0;
        }
      } else {  // type 3: second column of a 2x2 pair, its first column is slot s-1
        const double c0 = sb[(s - 1) * SLOT + lane];
        const int code0 = (int)__shfl(c0, FR, WAVE);
        const int pk = code0 & 63;
        const double e11 = __shfl(c0, FR + 1, WAVE), e12 = __shfl(c0, FR + 2, WAVE);
        const double e22 = __shfl(c, FR + 1, WAVE);
        const double c0r = lane < FR_R ? c0 : 0.0;
        const double ykr = __shfl(c0, FR_R, WAVE) - wave_sum(c0r * xr);
        const double ykb = __shfl(c0, FR_B, WAVE) - wave_sum(c0r * xb);
        const double yrr = __shfl(c, FR_R, WAVE) - wave_sum(cr * xr);
        const double yrb = __shfl(c, FR_B, WAVE) - wave_sum(cr * xb);
        const double det = e11 * e22 - e12 * e12;
        if (lane == pk) {
          xr = (e22 * ykr - e12 * yrr) / det;
          xb = (e22 * ykb - e12 * yrb) / det;
        }
        if (lane == p) {
          xr = (e11 * yrr - e12 * ykr) / det;
          xb = (e11 * yrb - e12 * ykb) / det;
        }
        s -= 1;
      }
    }
    if (lane < NK) {
      solr[t * NK + lane] = xr;
      solb[t * NK + lane] = xb;
    }
    if (lane == NK - 1) {
      const double b = rec[t * REC + jd];
      sigb += b * xb;
      sigr += b * xr;
      wdd += rec[t * REC + REC_WDD];
    }
    // coupling values for stage n-1: this stage's solution at its 16 coupling indices
    L.xr[lane] = xr;
    L.xb[lane] = xb;
    __syncthreads();
    if (lane >= NK && lane < NK + NC) {
      const int src = coupling_index(lane - NK);
      xr = L.xr[src];
      xb = L.xb[src];
    }
    __syncthreads();
  }
  if (lane == NK - 1) {
    part[(long long)w * 4 + 0] = sigb;
    part[(long long)w * 4 + 1] = sigr;
    part[(long long)w * 4 + 2] = wdd;
    part[(long long)w * 4 + 3] = 0.0;
  }
  if (lane == 0) {
    inert[w * 4 + 0] = (int)npos;
    inert[w * 4 + 1] = (int)nneg;
    inert[w * 4 + 2] = (int)nzero;
    inert[w * 4 + 3] = 0;
  }
}

// Forward and backward substitution with stored pivot columns: solr <- K_w^{-1} rhs.
__global__ __launch_bounds__(WAVE) void k_solve(const double* __restrict__ rec, const double* __restrict__ slots,
                                                const double* __restrict__ rhs, int N, int S, int jd,
                                                double* __restrict__ solr, double* __restrict__ part) {
  __shared__ double sh[2 * WAVE];
  const int w = blockIdx.x;
  if (w >= S) return;
  const int lane = lane_id();
  double ctb = 0.0;  // contribution carried by coupling lane 43+a to stage n+1's index R[a]
  for (int n = 0; n < N; ++n) {
    const long long t = (long long)w * N + n;
    const double* sb = slots + t * NK * SLOT;
    // right-hand side of this stage plus the contribution of the stage below
    sh[lane] = 0.0;
    __syncthreads();
    if (lane >= NK && lane < NK + NC) sh[coupling_index(lane - NK)] = ctb;
    __syncthreads();
    double r = (lane < NK ? rhs[t * NK + lane] + sh[lane] : 0.0);
    for (int s = 0; s < NK; ++s) {
      const double c = sb[s * SLOT + lane];
      const int code = (int)__shfl(c, FR, WAVE);
      const int type = code >> 6, p = code & 63;
      const double cr = lane < FR_R ? c : 0.0;
      if (type == 1) {
        const double d = __shfl(c, FR + 1, WAVE);
        const double yp = __shfl(r, p, WAVE);
        if (lane == p) solr[t * NK + p] = yp;  // forward value, consumed by the backward sweep
        r -= cr * (yp / d);
      } else if (type == 0) {
        const double yp = __shfl(r, p, WAVE);
        if (lane == p) solr[t * NK + p] = yp;
      } else if (type == 2) {
        const double c1 = sb[(s + 1) * SLOT + lane];
        const int q = ((int)__shfl(c1, FR, WAVE)) & 63;
        const double e11 = __shfl(c, FR + 1, WAVE), e12 = __shfl(c, FR + 2, WAVE);
        const double e22 = __shfl(c1, FR + 1, WAVE);
        const double yk = __shfl(r, p, WAVE), yq = __shfl(r, q, WAVE);
        if (lane == p) solr[t * NK + p] = yk;
        if (lane == q) solr[t * NK + q] = yq;
        const double det = e11 * e22 - e12 * e12;
        const double t1 = (e22 * yk - e12 * yq) / det, t2 = (e11 * yq - e12 * yk) / det;
        const double c1r = lane < FR_R ? c1 : 0.0;
        r -= cr * t1 + c1r * t2;
        s += 1;
      }
    }
    ctb = (lane >= NK && lane < NK + NC) ? r : 0.0;
    __syncthreads();
  }
  // backward sweep
  double x = 0.0, sig = 0.0;
  for (int n = N - 1; n >= 0; --n) {
    const long long t = (long long)w * N + n;
    const double* sb = slots + t * NK * SLOT;
    if (lane < NK) x = 0.0;
    for (int s = NK - 1; s >= 0; --s) {
      const double c = sb[s * SLOT + lane];
      const int code = (int)__shfl(c, FR, WAVE);
      const int type = code >> 6, p = code & 63;
      const double cr = lane < FR_R ? c : 0.0;
      if (type == 1 || type == 0) {
        const double d = __shfl(c, FR + 1, WAVE);
        const double pr = wave_sum(cr * x);
        const double yp = solr[t * NK + p];
        if (lane == p) x = type ? (yp - pr) / d : 0.0;
      } else {
        const double c0 = sb[(s - 1) * SLOT + lane];
        const int pk = ((int)__shfl(c0, FR, WAVE)) & 63;
        const double e11 = __shfl(c0, FR + 1, WAVE), e12 = __shfl(c0, FR + 2, WAVE);
        const double e22 = __shfl(c, FR + 1, WAVE);
        const double c0r = lane < FR_R ? c0 : 0.0;
        const double yk = solr[t * NK + pk] - wave_sum(c0r * x);
        const double yq = solr[t * NK + p] - wave_sum(cr * x);
        const double det = e11 * e22 - e12 * e12;
        if (lane == pk) x = (e22 * yk - e12 * yq) / det;
        if (lane == p) x = (e11 * yq - e12 * yk) / det;
        s -= 1;
      }
    }
    __syncthreads();
    if (lane < NK) solr[t * NK + lane] = x;
    if (lane == NK - 1) sig += rec[t * REC + jd] * x;
    sh[lane] = x;
    __syncthreads();
    if (lane >= NK && lane < NK + NC) x = sh[coupling_index(lane - NK)];
    __syncthreads();
  }
  if (lane == NK - 1) part[(long long)w * 4 + 1] = sig;
}

// Schur complement on d.  Fixed-order reduction of the per-scenario partials:
// sigma_b = sum b^T K^{-1} b, sigma_r = sum b^T K^{-1} r, W_dd and the inertia.
__global__ void k_schur(const double* __restrict__ part, const int* __restrict__ inert, int S,
                        const double* __restrict__ diagd, double dw, const double* __restrict__ rd, int mode,
                        DevScalars* __restrict__ out) {
  // mode 0: factor only; 1: factor with a right-hand side; 2: right-hand side only
  __shared__ double sb[256], sr[256], sw[256];
  __shared__ long long ip[256], in_[256], iz[256];
  double ab = 0, ar = 0, aw = 0;
  long long p = 0, q = 0, z = 0;
  for (int w = threadIdx.x; w < S; w += blockDim.x) {
    ab += part[w * 4 + 0];
    ar += part[w * 4 + 1];
    aw += part[w * 4 + 2];
    p += inert[w * 4 + 0];
    q += inert[w * 4 + 1];
    z += inert[w * 4 + 2];
  }
  sb[threadIdx.x] = ab;
  sr[threadIdx.x] = ar;
  sw[threadIdx.x] = aw;
  ip[threadIdx.x] = p;
  in_[threadIdx.x] = q;
  iz[threadIdx.x] = z;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sb[threadIdx.x] += sb[threadIdx.x + s];
      sr[threadIdx.x] += sr[threadIdx.x + s];
      sw[threadIdx.x] += sw[threadIdx.x + s];
      ip[threadIdx.x] += ip[threadIdx.x + s];
      in_[threadIdx.x] += in_[threadIdx.x + s];
      iz[threadIdx.x] += iz[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (mode != 2) {
      out->sig_b = sb[0];
      out->wdd = sw[0];
      out->kdd = sw[0] + *diagd + dw;
      out->sd = out->kdd - sb[0];
      long long np = ip[0], nn = in_[0], nz = iz[0];
      if (out->sd > 0.0) ++np;
      else if (out->sd < 0.0) ++nn;
      else ++nz;
      out->npos = np;
      out->nneg = nn;
      out->nzero = nz;
    }
    if (mode != 0) {
      out->sig_r = sr[0];
      out->rd = *rd;
      out->dd = (*rd - sr[0]) / out->sd;
    }
  }
}

// sol = solr - solb * dd (scenario part), sol[last] = dd
__global__ void k_combine(const double* __restrict__ solr, const double* __restrict__ solb,
                          const DevScalars* __restrict__ sc, long long nk, double* __restrict__ sol) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double dd = sc->dd;
  if (i < nk) sol[i] = solr[i] - solb[i] * dd;
  if (i == nk) sol[nk] = dd;
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// Residual of the bordered KKT system for the rows of stage (w, n):
// res = rhs - K sol; part of the d row (b * sol_hyd) in dpart; per-stage
// componentwise backward error max_i |res_i| / (|K||sol| + |rhs|)_i in omg.
__global__ void k_residual(const double* __restrict__ rec, const int* __restrict__ jtab,
                           const double* __restrict__ diagx, const double* __restrict__ diags, double dw, double dc,
                           const double* __restrict__ sol, const double* __restrict__ rhs, int N, int S, int jd,
                           double* __restrict__ res, double* __restrict__ dpart, double* __restrict__ dabs,
                           double* __restrict__ omg) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * S) return;
  const int n = (int)(t % N);
  const long long nkk = (long long)N * S * NK;
  const double* R = rec + t * REC;
  const double* u = sol + t * NK;
  double ku[NK], ka[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    ku[k] = 0.0;
    ka[k] = 0.0;
  }
  // own Jacobian block (rows: duals, cols: primals) and the d entry
  for (int e = 0; e < NJO; ++e) {
    const int rc = jtab[e];
    const int r = rc & 255, col = (rc >> 8) & 255, blk = rc >> 16;
    const double j = R[REC_OWN + e];
    const int dr = r < NE ? NV + r : NK - 1;
    if (blk == BLK_D) {
      ku[dr] += j * sol[nkk];
      ka[dr] += fabs(j * sol[nkk]);
      continue;
    }
    ku[dr] += j * u[col];
    ka[dr] += fabs(j * u[col]);
    ku[col] += j * u[dr];
    ka[col] += fabs(j * u[dr]);
  }
  if (n < N - 1) {  // this stage's rows against stage n+1's primals
    for (int e = 0; e < NJU; ++e) {
      const int rc = jtab[NJO + e];
      const int r = rc & 255, col = (rc >> 8) & 255;
      const double j = R[REC_UP + e];
      ku[NV + r] += j * u[NK + col];
      ka[NV + r] += fabs(j * u[NK + col]);
    }
    const double* R1 = R + REC;  // stage n+1's rows against this stage's primals
    for (int e = 0; e < NJD; ++e) {
      const int rc = jtab[NJO + NJU + e];
      const int r = rc & 255, col = (rc >> 8) & 255;
      const double j = R1[REC_DOWN + e];
      ku[col] += j * u[NK + NV + r];
      ka[col] += fabs(j * u[NK + NV + r]);
    }
  }
  if (n > 0) {
    for (int e = 0; e < NJD; ++e) {  // this stage's rows against stage n-1's primals
      const int rc = jtab[NJO + NJU + e];
      const int r = rc & 255, col = (rc >> 8) & 255;
      const double j = R[REC_DOWN + e];
      ku[NV + r] += j * u[-NK + col];
      ka[NV + r] += fabs(j * u[-NK + col]);
    }
    const double* R0 = R - REC;  // stage n-1's rows against this stage's primals
    for (int e = 0; e < NJU; ++e) {
      const int rc = jtab[NJO + e];
      const int r = rc & 255, col = (rc >> 8) & 255;
      const double j = R0[REC_UP + e];
      ku[col] += j * u[-NK + NV + r];
      ka[col] += fabs(j * u[-NK + NV + r]);
    }
  }
  // Hessian block
  HessPos pos[NH];
  hess_positions(pos);
  for (int e = 0; e < NH; ++e) {
    const int a = pos[e].r, b = pos[e].c;
    const double hv = R[REC_H + e];
    ku[a] += hv * u[b];
    ka[a] += fabs(hv * u[b]);
    if (a != b) {
      ku[b] += hv * u[a];
      ka[b] += fabs(hv * u[a]);
    }
  }
  for (int k = 0; k < NV; ++k) {
    const double dg = diagx[t * NV + k] + dw;
    ku[k] += dg * u[k];
    ka[k] += fabs(dg * u[k]);
  }
  for (int r = 0; r < NE; ++r) {
    ku[NV + r] -= dc * u[NV + r];
    ka[NV + r] += fabs(dc * u[NV + r]);
  }
  {
    const double dh = -(1.0 / (diags[t] + dw) + dc);
    ku[NK - 1] += dh * u[NK - 1];
    ka[NK - 1] += fabs(dh * u[NK - 1]);
  }
  double om = 0.0;
  for (int k = 0; k < NK; ++k) {
    const double rr = rhs[t * NK + k] - ku[k];
    res[t * NK + k] = rr;
    const double den = ka[k] + fabs(rhs[t * NK + k]);
    const double o = den > 0.0 ? fabs(rr) / den : (rr == 0.0 ? 0.0 : INFINITY);
    om = fmax(om, o);
  }
  omg[t] = om;
  dpart[t] = R[jd] * u[NK - 1];
  dabs[t] = fabs(R[jd] * u[NK - 1]);
}

// d row of the residual: res_d = rhs_d - sum b u_hyd - kdd u_d (one block, fixed order)
__global__ void k_residual_d(const double* __restrict__ dpart, const double* __restrict__ dabs, long long nst,
                             const DevScalars* __restrict__ sc, const double* __restrict__ sol,
                             const double* __restrict__ rhs, long long nkk, double* __restrict__ res,
                             double* __restrict__ omg_d) {
  __shared__ double s1[256], s2[256];
  double a = 0, b = 0;
  for (long long t = threadIdx.x; t < nst; t += blockDim.x) {
    a += dpart[t];
    b += dabs[t];
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
    const double ku = s1[0] + sc->kdd * sol[nkk];
    const double ka = s2[0] + fabs(sc->kdd * sol[nkk]);
    const double rr = rhs[nkk] - ku;
    res[nkk] = rr;
    const double den = ka + fabs(rhs[nkk]);
    *omg_d = den > 0.0 ? fabs(rr) / den : (rr == 0.0 ? 0.0 : INFINITY);
  }
}

__global__ void k_max_reduce(const double* __restrict__ v, long long n, double* __restrict__ out) {
  __shared__ double sm[256];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) a = fmax(a, v[i]);
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
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
  const long long nst = (long long)h.N * h.S;
  prof_begin(h, st);
  hipLaunchKernelGGL(k_eval, dim3(grid_for(nst, 128)), dim3(128), 0, st, x, sc, scaled, y, cs, h.feeds, h.mp, h.N,
                     h.S, full, c_out, h.rec);
  prof_end(h, 2, st);
  return hipGetLastError();
}

hipError_t launch_rowmax(Handle& h, const double* x, int scaled, double* rowmax, hipStream_t st) {
  const long long nst = (long long)h.N * h.S;
  hipLaunchKernelGGL(k_rowmax, dim3(grid_for(nst, 128)), dim3(128), 0, st, x, h.sc, scaled, h.feeds, h.mp, h.N,
                     h.S, rowmax);
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

hipError_t launch_factor(Handle& h, const double* diagx, const double* diags, double dw, double dc,
                         const double* rhs, hipStream_t st) {
  prof_begin(h, st);
  if (rhs)
    hipLaunchKernelGGL(k_factor<1>, dim3(h.S), dim3(WAVE), 0, st, h.rec, h.gather, rhs, diagx, diags, dw, dc, h.N,
                       h.S, h.jac_d_index, h.slots, h.solr, h.solb, h.inert, h.part);
  else
    hipLaunchKernelGGL(k_factor<0>, dim3(h.S), dim3(WAVE), 0, st, h.rec, h.gather, rhs, diagx, diags, dw, dc, h.N,
                       h.S, h.jac_d_index, h.slots, h.solr, h.solb, h.inert, h.part);
  prof_end(h, 0, st);
  h.fdw = dw;
  h.fdc = dc;
  h.factored = true;
  ++h.n_factor;
  return hipGetLastError();
}

hipError_t launch_solve(Handle& h, const double* rhs, hipStream_t st) {
  prof_begin(h, st);
  hipLaunchKernelGGL(k_solve, dim3(h.S), dim3(WAVE), 0, st, h.rec, h.slots, rhs, h.N, h.S, h.jac_d_index, h.solr,
                     h.part);
  prof_end(h, 1, st);
  ++h.n_solve;
  return hipGetLastError();
}

hipError_t launch_schur(Handle& h, const double* diagd, double dw, const double* rd, int mode, double* sol,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_schur, dim3(1), dim3(256), 0, st, h.part, h.inert, h.S, diagd, dw, rd, mode, h.scal);
  if (mode != 0 && sol) {
    const long long nk = (long long)h.N * h.S * NK;
    hipLaunchKernelGGL(k_combine, dim3(grid_for(nk + 1, 256)), dim3(256), 0, st, h.solr, h.solb, h.scal, nk, sol);
  }
  return hipGetLastError();
}

hipError_t launch_residual(Handle& h, const double* diagx, const double* diags, double dw, double dc,
                           const double* sol, const double* rhs, double* res, double* omega_out, hipStream_t st) {
  const long long nst = (long long)h.N * h.S;
  const long long nkk = nst * NK;
  double* dpart = h.kden;
  double* dabs = h.kden + nst;
  double* omg = h.kden + 2 * nst;
  prof_begin(h, st);
  hipLaunchKernelGGL(k_residual, dim3(grid_for(nst, 64)), dim3(64), 0, st, h.rec, h.jtab, diagx, diags, dw, dc, sol,
                     rhs, h.N, h.S, h.jac_d_index, res, dpart, dabs, omg);
  prof_end(h, 3, st);
  hipLaunchKernelGGL(k_residual_d, dim3(1), dim3(256), 0, st, dpart, dabs, nst, h.scal, sol, rhs, nkk, res,
                     omega_out + 1);
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, st, omg, nst, omega_out);
  return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, st, y, x, a, n);
  return hipGetLastError();
}

}  // namespace absorber
