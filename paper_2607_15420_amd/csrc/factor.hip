// HIP kernels for gfx950: the per-scenario block LDL^T of the primal-dual KKT
// system (one wavefront per scenario chain, Bunch-Kaufman pivoting inside each
// stage), the solve with the stored factor and the Schur complement on the
// shared diameter.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace absorber {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

inline unsigned grid_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- block LDL^T
// Frontal matrix of stage n held one column per lane: lane j owns column j,
// v[i] is row i.  Columns/rows 0-42 are the stage's KKT unknowns, 43-58 the
// coupling unknowns of stage n+1, 59 the right-hand side r, 60 the border b
// (both carried as symmetric extra rows and columns).  Eliminating the 43 own
// pivots leaves in rows/cols 43-60 the contribution to stage n+1's block and
// right-hand sides.  The candidate pivot row is selected from the registers
// (by symmetry it is the candidate column) by one indexed register move inside
// a phase's window of rows, or by a uniform switch, single entries
// reach every lane through v_readlane, and the pivot column of each rank-1
// update is broadcast through LDS (every lane reads the same address).
constexpr int TAIL = SLOT - NK;  // rows 43-63 of a stored pivot column: coupling, r, b, code, d, 1/d
constexpr int STG = TAIL + 1;     // LDS stride of one staged tail
struct WaveLDS {
  double bc[WAVE];  // pivot row of the current elimination step (first: reachable by immediate offsets)
  union {
    double src[NSRC];     // assembly sources (elimination)
    double stg[NK * STG];  // tails of the stage's pivot columns (backward sweep)
  };
  double xr[WAVE];
  double xb[WAVE];
};

// value of lane l (l uniform) broadcast to the wave
__device__ __forceinline__ double rdl(double v, int l) {
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  return __hiloint2double(hi, lo);
}

// register p of this lane for a uniform p in [LO, NK): the cases below LO are
// left out, so the registers of rows already eliminated are dead in later phases
template <int LO>
__device__ __forceinline__ double rowsel(const double (&v)[FR], int p) {
  switch (p) {
#define ABS_CASE(i) \
  case i:           \
    return (i) >= LO ? v[i] : 0.0;
    ABS_CASE(0) ABS_CASE(1) ABS_CASE(2) ABS_CASE(3) ABS_CASE(4) ABS_CASE(5) ABS_CASE(6) ABS_CASE(7)
    ABS_CASE(8) ABS_CASE(9) ABS_CASE(10) ABS_CASE(11) ABS_CASE(12) ABS_CASE(13) ABS_CASE(14) ABS_CASE(15)
    ABS_CASE(16) ABS_CASE(17) ABS_CASE(18) ABS_CASE(19) ABS_CASE(20) ABS_CASE(21) ABS_CASE(22) ABS_CASE(23)
    ABS_CASE(24) ABS_CASE(25) ABS_CASE(26) ABS_CASE(27) ABS_CASE(28) ABS_CASE(29) ABS_CASE(30) ABS_CASE(31)
    ABS_CASE(32) ABS_CASE(33) ABS_CASE(34) ABS_CASE(35) ABS_CASE(36) ABS_CASE(37) ABS_CASE(38) ABS_CASE(39)
    ABS_CASE(40) ABS_CASE(41) ABS_CASE(42)
#undef ABS_CASE
    default:
      return 0.0;
  }
}

// register p of this lane for a uniform p in [LO, LO + W), W = 8 or 16: one
// indexed register move (s_set_gpr_idx) out of the tuple of rows LO..LO+W-1,
// which the compiler forms from the frontal registers themselves (no copies).
// A phase whose lowest remaining pivot stays inside such a window selects it
// this way instead of through the branch tree above.
typedef double dvec8 __attribute__((ext_vector_type(8)));
typedef double dvec16 __attribute__((ext_vector_type(16)));
template <int LO, int W>
__device__ __forceinline__ double rowsel_win(const double (&v)[FR], int p) {
  static_assert(W == 8 || W == 16, "window of 8 or 16 rows");
  static_assert(LO + W <= FR, "window inside the frontal matrix");
  if constexpr (W == 8) {
    dvec8 t;
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = v[LO + i];
    return t[(p - LO) & 7];
  } else {
    dvec16 t;
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[LO + i];
    return t[(p - LO) & 15];
  }
}

// Wave maximum of a non-negative double and its lane.  The key is the high
// word of the value (sign, exponent, 20 mantissa bits) with its 6 lowest bits
// replaced by 63 - lane (ties go to the lowest lane); keys are max-reduced with
// DPP row shifts and row broadcasts and lane 63 ends with the maximum.  The
// returned value keeps 14 mantissa bits (relative truncation below 2^-14),
// which is all the pivot tests compare.
#define ABS_DPP_MAX_U32(k, ctrl, rm, bm)                                                          \
  do {                                                                                           \
    const unsigned o_ = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(k), ctrl, rm, bm, false); \
    (k) = o_ > (k) ? o_ : (k);                                                                   \
  } while (0)

__device__ __forceinline__ double wave_max_lane(double a, int lane, int& idx) {
  unsigned key = ((unsigned)__double2hiint(a) & ~63u) | (unsigned)(63 - lane);
  ABS_DPP_MAX_U32(key, 0x111, 0xf, 0xf);  // row_shr:1
  ABS_DPP_MAX_U32(key, 0x112, 0xf, 0xf);  // row_shr:2
  ABS_DPP_MAX_U32(key, 0x114, 0xf, 0xf);  // row_shr:4
  ABS_DPP_MAX_U32(key, 0x118, 0xf, 0xf);  // row_shr:8
  ABS_DPP_MAX_U32(key, 0x142, 0xa, 0xf);  // row_bcast:15
  ABS_DPP_MAX_U32(key, 0x143, 0xc, 0xf);  // row_bcast:31
  const unsigned m = (unsigned)__builtin_amdgcn_readlane((int)key, 63);
  idx = 63 - (int)(m & 63u);
  return __hiloint2double((int)(m & ~63u), 0);
}

// Rank-1 update of rows 8*C0..60: v[i] -= bc[i] * tt, software pipelined (the
// next QN entries of the broadcast pivot column are read while QN rows update).
template <int C0>
__device__ __forceinline__ void rank1_rows(double (&v)[FR], const double* bc, double tt) {
  constexpr int QN = 4;
  constexpr int NQ = (FR + QN - 1) / QN;
  double qa[QN], qb[QN];
#pragma unroll
  for (int j = 0; j < QN; ++j) qa[j] = bc[8 * C0 + j];
#pragma unroll
  for (int c = 8 * C0 / QN; c < NQ; ++c) {
    if (c < NQ - 1) {
#pragma unroll
      for (int j = 0; j < QN; ++j) qb[j] = bc[QN * (c + 1) + j];
    }
#pragma unroll
    for (int j = 0; j < QN; ++j)
      if (QN * c + j < FR) v[QN * c + j] = fma(-qa[j], tt, v[QN * c + j]);
#pragma unroll
    for (int j = 0; j < QN; ++j) qa[j] = qb[j];
  }
}

// Pivots of one stage taken while the lowest remaining pivot is below LIMIT
// (Bunch-Kaufman inside the stage); stores one pivot column per slot (rows
// still active, code, d or 2x2 block, 1/d).  The matrix is symmetric, so the
// pivot candidates' columns are read as rows (register p of every lane): the
// lowest remaining pivot with an indexed move when the phase's window of
// possible pivots spans at most 16 rows, the second Bunch-Kaufman candidate
// (any active row) with a uniform switch.  The rank-1 updates start at row 8*C0.
template <int C0, int LIMIT>
__device__ __forceinline__ void eliminate_phase(double (&v)[FR], double* __restrict__ sb, double* bc,
                                                uint64_t& act, int& slot, int& npos, int& nneg,
                                                int& nzero) {
  int lane = lane_id();
  __asm__ volatile("" : "+v"(lane));
  const double alpha = (1.0 + sqrt(17.0)) * 0.125;
  while (act && __builtin_ctzll(act) < LIMIT) {
    const int k = __builtin_ctzll(act);
    const bool own_act = lane < NK && ((act >> lane) & 1ull);
    // F[k][lane] = F[lane][k]; k stays below LIMIT (and NK) in this phase
    constexpr int KW = (LIMIT < NK ? LIMIT : NK) - 8 * C0;
    const double rowk = KW <= 8 ? rowsel_win<8 * C0, 8>(v, k)
                        : KW <= 16 ? rowsel_win<8 * C0, 16>(v, k)
                                   : rowsel<8 * C0>(v, k);
    const double dkk = rdl(rowk, k);
    // 1/d for the usual 1x1 pivot at k, started before the search so that the
    // two dependency chains overlap
    const double dinv_k = dkk == 0.0 ? 0.0 : 1.0 / dkk;
    const double akk = fabs(dkk);
    int r;
    const double lam = wave_max_lane(own_act && lane != k ? fabs(rowk) : 0.0, lane, r);
    int ptype = 1;  // 1: 1x1 at k, 2: 1x1 at r, 3: 2x2 (k, r)
    double rowr = 0.0;
    if (!(akk >= alpha * lam) && lam > 0.0) {
      rowr = rowsel<8 * C0>(v, r);
      int r2;
      const double sig = wave_max_lane(own_act && lane != r ? fabs(rowr) : 0.0, lane, r2);
      if (akk * sig >= alpha * lam * lam) ptype = 1;
      else if (fabs(rdl(rowr, r)) >= alpha * sig) ptype = 2;
      else ptype = 3;
    }
    const bool in_col = lane < FR && (lane >= NK || ((act >> lane) & 1ull));
    const bool two = ptype == 3;
    const int p0 = ptype == 2 ? r : k;
    const int p1 = two ? r : p0;
    const double rk = ptype == 2 ? rowr : rowk;  // F[p0][lane]
    const double rr = two ? rowr : 0.0;          // F[p1][lane]
    const bool ca = in_col && lane != p0 && lane != p1;
    double t1 = 0.0, t2 = 0.0;
    bool zero = false;
    if (!two) {
      double d = dkk, dinv = dinv_k;
      if (ptype == 2) {
        d = rdl(rk, p0);
        dinv = d == 0.0 ? 0.0 : 1.0 / d;
      }
      // stored column: the active entries, then the pivot code, d and 1/d (selects,
      // not branches: the code is uniform and formed before the lane selects)
      const double code = (double)(p0 + 64 * (d == 0.0 ? 0 : 1));
      double sv = ca ? rk : 0.0;
      sv = lane == FR ? code : sv;
      sv = lane == FR + 1 ? d : sv;
      sv = lane > FR + 1 ? dinv : sv;
      sb[slot * SLOT + lane] = sv;
      slot += 1;
      if (d == 0.0) {
        ++nzero;
        zero = true;
      } else {
        const int pos = d > 0.0 ? 1 : 0;  // branch-free: keeps the counters in registers
        npos += pos;
        nneg += 1 - pos;
        t1 = ca ? rk * dinv : 0.0;
      }
    } else {
      const double e11 = rdl(rk, p0), e12 = rdl(rk, p1), e22 = rdl(rr, p1);
      const double det = e11 * e22 - e12 * e12;
      double s0 = ca ? rk : 0.0, s1 = ca ? rr : 0.0;
      if (lane == FR) {
        s0 = (double)(p0 + 64 * 2);
        s1 = (double)(p1 + 64 * 3);
      } else if (lane == FR + 1) {
        s0 = e11;
        s1 = e22;
      } else if (lane == FR + 2) {
        s0 = e12;
        s1 = e12;
      }
      sb[slot * SLOT + lane] = s0;
      sb[(slot + 1) * SLOT + lane] = s1;
      slot += 2;
      if (det < 0.0) {
        ++npos;
        ++nneg;
      } else if (det > 0.0) {
        const int pos = e11 + e22 > 0.0 ? 2 : 0;
        npos += pos;
        nneg += 2 - pos;
      } else {
        nzero += 2;
        zero = true;
      }
      if (!zero) {
        const double idet = 1.0 / det;
        const double i11 = e22 * idet, i12 = -e12 * idet, i22 = e11 * idet;
        t1 = ca ? i11 * rk + i12 * rr : 0.0;
        t2 = ca ? i12 * rk + i22 * rr : 0.0;
      }
    }
    act &= ~((1ull << p0) | (1ull << p1));
    if (zero) continue;
    // The pivot row reaches every lane through LDS (all lanes read the same
    // address, a broadcast).  Rows below 8*C0 are never updated: all their
    // pivots were eliminated before this phase and they are never read again.
    // Eliminated rows above (and p0/p1 themselves) are updated too, harmlessly.
    // A 2x2 pivot is applied as two rank-1 passes (c1 t1^T, then c2 t2^T).
    for (int pass = 0; pass < (two ? 2 : 1); ++pass) {
      const double tt = pass ? t2 : t1;
      bc[lane] = pass ? rr : rk;
      __syncthreads();
      rank1_rows<C0>(v, bc, tt);
      __syncthreads();
    }
  }
}


// Eliminate the 43 own pivots of one stage.  The lowest remaining pivot only
// grows, so the stage runs in phases whose rank-1 updates skip the leading rows
// once all their pivots are gone (those rows are never read again).  The row
// split is the tile shape of the trailing update, chosen by the autotuner:
//   SPLIT 0: three phases, updates from rows 0, 16, 32;
//   SPLIT 1: two phases, updates from rows 0, 24;
//   SPLIT 2: six phases, updates from rows 0, 8, 16, 24, 32, 40.
template <int SPLIT>
__device__ __forceinline__ void eliminate_stage(double (&v)[FR], double* __restrict__ sb, double* bc,
                                                int& npos, int& nneg, int& nzero) {
  uint64_t act = (1ull << NK) - 1ull;
  int slot = 0;
  if (SPLIT == 0) {
    eliminate_phase<0, 16>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<2, 32>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<4, 64>(v, sb, bc, act, slot, npos, nneg, nzero);
  } else if (SPLIT == 1) {
    eliminate_phase<0, 24>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<3, 64>(v, sb, bc, act, slot, npos, nneg, nzero);
  } else {
    eliminate_phase<0, 8>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<1, 16>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<2, 24>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<3, 32>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<4, 40>(v, sb, bc, act, slot, npos, nneg, nzero);
    eliminate_phase<5, 64>(v, sb, bc, act, slot, npos, nneg, nzero);
  }
}

// Backward sweep of one stage for two right-hand sides.  The stage's pivot
// columns are gathered into registers in pivot order (lane s holds slot s;
// reg[q] = its entry at the row eliminated q-th), so that each step is a
// static-register update.  The tails of the 43 columns (coupling rows, the
// forward values of r and b, the pivot code and d) are first staged in LDS
// with coalesced loads (three columns per load) and read back one column per
// lane.  The solutions of the stage above (LDS, by stage-local index; read at
// the 16 coupling indices) are applied first.
// On return lane s holds the solution of pivot s in xr_s/xb_s and p_s its index.
__device__ __forceinline__ void backward_stage(const double* __restrict__ sb, double* stg, const double* xcr,
                                               const double* xcb, bool two, double& xr_s, double& xb_s,
                                               int& p_s) {
  int lane = lane_id();
  __asm__ volatile("" : "+v"(lane));
  {
    const int sj = lane / TAIL, e = lane - sj * TAIL;  // column sj of each group of three, row NK + e
#pragma unroll
    for (int c = 0; c < (NK + 2) / 3; ++c) {
      const int s = 3 * c + sj;
      if (sj < 3 && s < NK) stg[s * STG + e] = sb[s * SLOT + NK + e];
    }
  }
  __syncthreads();
  const int ls = lane < NK ? lane : 0;
  const double* tl = stg + ls * STG;  // this lane's column tail
  double zr = tl[FR_R - NK], zb = tl[FR_B - NK];  // forward values of r and b by slot
  const double code_l = tl[FR - NK];
  const double a_l = tl[FR + 1 - NK];  // d, or e11 / e22 of a 2x2 pair
  const double b_l = tl[FR + 2 - NK];  // 1/d, or e12
  p_s = ((int)code_l) & 63;
  // Slot s's entry at the row eliminated q-th is zero unless q > s (and is only
  // read by lanes s < q), so only those lanes load it: the gathers touch half
  // the cache lines of a full 43 x 43 gather.
  double reg[NK];
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    const int pq = ((int)rdl(code_l, q)) & 63;
    reg[q] = 0.0;
    if (lane < q) reg[q] = sb[lane * SLOT + pq];
    if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const double c = tl[a];
    zr = fma(-c, xcr[coupling_index(a)], zr);
    if (two) zb = fma(-c, xcb[coupling_index(a)], zb);
  }
  // Slot s's entries at its own row and at the rows eliminated before it were
  // not loaded (reg = 0), so a lane's z stops changing once its own slot has been
  // solved: a 1x1 slot's solution is its final z times 1/d, formed for every lane
  // after the loop.  Pivot types are wave masks, tested on the scalar unit.
  const int type_l = lane < NK ? (((int)code_l) >> 6) : 1;  // 0 zero pivot, 1 1x1, 2/3 first/second of 2x2
  const uint64_t m_second = __ballot(lane < NK && type_l == 3);
  const uint64_t m_zero = __ballot(lane < NK && type_l == 0);
  double pr = 0.0, pb = 0.0;  // solutions of the 2x2 pairs
  bool skip = false;
#pragma unroll
  for (int s = NK - 1; s >= 0; --s) {
    if (skip) {
      skip = false;
      continue;
    }
    if (s > 0 && ((m_second >> s) & 1ull)) {
      const int s0 = s > 0 ? s - 1 : 0;
      const double e11 = rdl(a_l, s0), e12 = rdl(b_l, s0), e22 = rdl(a_l, s);
      const double idet = 1.0 / (e11 * e22 - e12 * e12);
      const double zk = rdl(zr, s0), zq = rdl(zr, s);
      const double xk = (e22 * zk - e12 * zq) * idet, xq = (e11 * zq - e12 * zk) * idet;
      zr = fma(-reg[s0], xk, fma(-reg[s], xq, zr));
      if (lane == s0) pr = xk;
      if (lane == s) pr = xq;
      if (two) {
        const double wk = rdl(zb, s0), wq = rdl(zb, s);
        const double yk = (e22 * wk - e12 * wq) * idet, yq = (e11 * wq - e12 * wk) * idet;
        zb = fma(-reg[s0], yk, fma(-reg[s], yq, zb));
        if (lane == s0) pb = yk;
        if (lane == s) pb = yq;
      }
      skip = true;
    } else {
      const bool zero = (m_zero >> s) & 1ull;
      const double x = zero ? 0.0 : rdl(zr * b_l, s);  // lane s: z_s / d_s
      zr = fma(-reg[s], x, zr);
      if (two) {
        const double y = zero ? 0.0 : rdl(zb * b_l, s);
        zb = fma(-reg[s], y, zb);
      }
    }
  }
  const bool pair = type_l >= 2;
  xr_s = pair ? pr : (type_l == 0 ? 0.0 : zr * b_l);
  xb_s = pair ? pb : (type_l == 0 ? 0.0 : zb * b_l);
}

// Sum over the wave of a double, fixed order (DPP row shifts and row
// broadcasts on the two halves; lane 63 ends with the total), returned to
// every lane.
#define ABS_DPP_ADD_F64(v, ctrl, rm)                                                     \
  do {                                                                                  \
    const int lo_ = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, rm, 0xf, false); \
    const int hi_ = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, rm, 0xf, false); \
    (v) += __hiloint2double(hi_, lo_);                                                  \
  } while (0)

__device__ __forceinline__ double wave_total(double v) {
  ABS_DPP_ADD_F64(v, 0x111, 0xf);  // row_shr:1
  ABS_DPP_ADD_F64(v, 0x112, 0xf);  // row_shr:2
  ABS_DPP_ADD_F64(v, 0x114, 0xf);  // row_shr:4
  ABS_DPP_ADD_F64(v, 0x118, 0xf);  // row_shr:8
  ABS_DPP_ADD_F64(v, 0x142, 0xa);  // row_bcast:15
  ABS_DPP_ADD_F64(v, 0x143, 0xc);  // row_bcast:31
  return rdl(v, 63);
}

// Backward sweep of one stage for R right-hand sides with rows on lanes:
// lane i loads row i of every stored pivot column (coalesced), and pivot s
// (descending) takes x = dinv_s (y_s - sum_i F_s[i] x_i) with one wave sum per
// right-hand side.  Rows eliminated before s are zero in column s and rows not
// yet solved hold x = 0, so the sums run over all lanes.  ys[r]: lane s holds
// the forward value of slot s; xc[r]: solution of the stage above by
// stage-local index (read at the 16 coupling indices).  On return lane i < 43
// holds the solution of row i in xl[r].
template <int R>
__device__ __forceinline__ void backward_rows(const double* __restrict__ sb, int lim, const double (&ys)[R],
                                              const double* const (&xc)[R], double (&xl)[R]) {
  const int lane = lane_id();
  double col[NK];
#pragma unroll
  for (int q = 0; q < NK; ++q) col[q] = q < lim ? sb[q * SLOT + lane] : 0.0;
  const bool cpl = lane >= NK && lane < NK + NC;
  const int ci = coupling_index(cpl ? lane - NK : 0);
#pragma unroll
  for (int r = 0; r < R; ++r) xl[r] = cpl ? xc[r][ci] : 0.0;
  bool skip = false;
#pragma unroll
  for (int s = NK - 1; s >= 0; --s) {
    if (skip) {
      skip = false;
      continue;
    }
    const int code = (int)rdl(col[s], FR);
    const int type = code >> 6, p = code & 63;
    if (s > 0 && type == 3) {  // second slot of a 2x2 pivot: solve the pair (s-1, s)
      const int s0 = s > 0 ? s - 1 : 0;
      const int pa = ((int)rdl(col[s0], FR)) & 63;
      const double e11 = rdl(col[s0], FR + 1), e12 = rdl(col[s0], FR + 2), e22 = rdl(col[s], FR + 1);
      const double idet = 1.0 / (e11 * e22 - e12 * e12);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double za = rdl(ys[r], s0) - wave_total(col[s0] * xl[r]);
        const double zb = rdl(ys[r], s) - wave_total(col[s] * xl[r]);
        const double xa = (e22 * za - e12 * zb) * idet, xb = (e11 * zb - e12 * za) * idet;
        if (lane == pa) xl[r] = xa;
        if (lane == p) xl[r] = xb;
      }
      skip = true;
    } else {
      const double dinv = rdl(col[s], FR + 2);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double dot = wave_total(col[s] * xl[r]);
        const double x = type ? (rdl(ys[r], s) - dot) * dinv : 0.0;
        if (lane == p) xl[r] = x;
      }
    }
  }
}

template <int SPLIT, int WPE>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(WPE))) void k_factor(
    const double* __restrict__ rec, const int* __restrict__ gather, const double* __restrict__ rhs,
    const double* __restrict__ diagx, const double* __restrict__ diags, const double* __restrict__ dwv,
    const double* __restrict__ dcv, const int* __restrict__ chain0, const int* __restrict__ chain_p,
    const int* __restrict__ fmask, const int* __restrict__ chmask, int W, int jd, int npar, double* __restrict__ slots, int* __restrict__ lines,
    double* __restrict__ solr, double* __restrict__ solb, int* __restrict__ inert, double* __restrict__ part) {
  __shared__ WaveLDS L;
  const int w = blockIdx.x;
  if (w >= W) return;
  const int pw = chain_p[w];
  if (fmask && !fmask[pw]) return;  // this problem keeps its factorisation
  if (chmask && !chmask[w]) {       // chain left out: zero solutions and partial sums
    for (long long i = (long long)chain0[w] * NK + threadIdx.x; i < (long long)chain0[w + 1] * NK; i += WAVE) {
      solr[i] = 0.0;
      solb[i] = 0.0;
    }
    if (threadIdx.x < 4) {
      part[(long long)w * 4 + threadIdx.x] = 0.0;
      inert[w * 4 + threadIdx.x] = 0;
    }
    return;
  }
  const long long t0 = chain0[w];
  const int N = chain0[w + 1] - (int)t0;
  const double dw = dwv[pw], dc = dcv[pw];
  const int lane = lane_id();
  for (int i = lane; i < NC * (NC + 2); i += WAVE) L.src[SRC_CTB + i] = 0.0;
  if (lane == 0) L.src[SRC_ZERO] = 0.0;
  int npos = 0, nneg = 0, nzero = 0;
  for (int n = 0; n < N; ++n) {
    const long long t = t0 + n;
    const double* R = rec + t * REC;
    double v[FR];
    // the stage's inputs: every load is issued before the first LDS write, so
    // that they cost one memory round trip (indices clamped, entries past the
    // ends reread and not written)
    // (the lane index is re-read here so that the compiler forms the per-lane
    // offsets in each stage instead of keeping them live, or spilled, across it)
    int ln = lane_id();
    __asm__ volatile("" : "+v"(ln));
    constexpr int NREC = (REC + WAVE - 1) / WAVE;
    double rv[NREC];
#pragma unroll
    for (int m = 0; m < NREC; ++m) rv[m] = R[min(ln + WAVE * m, REC - 1)];
    const double dn = rec[(n < N - 1 ? t + 1 : t) * REC + REC_DOWN + min(ln, NJD - 1)];
    const double dx = diagx[t * NV + min(ln, NV - 1)];
    const double ds = diags[t], brd = R[jd];
    const double rh = rhs ? rhs[t * NK + min(ln, NK - 1)] : 0.0;
#pragma unroll
    for (int m = 0; m < NREC; ++m)
      if (lane + WAVE * m < REC) L.src[SRC_REC + lane + WAVE * m] = rv[m];
    if (lane < NJD) L.src[SRC_DOWN1 + lane] = n < N - 1 ? dn : 0.0;
    if (lane < NK) L.src[SRC_RHS + lane] = rh;
    if (lane < NV) L.src[SRC_DIAGX + lane] = dx + dw;
    if (lane == 0) {
      // the fused border: the diameter of the stage's section (section 0 when
      // there are several; the other sections' borders are solved afterwards)
      L.src[SRC_BRD] = section_of(n, N, npar) == 0 ? brd : 0.0;
      L.src[SRC_DC] = -dc;
      L.src[SRC_DHYD] = -(1.0 / (ds + dw) + dc);
    }
    __syncthreads();
    // keep the table loads inside the stage loop (hoisting them would pin ~120
    // registers); the pointer keeps its global address space, so the loads are
    // global loads, issued eight at a time one chunk ahead of their LDS gathers
    typedef const __attribute__((address_space(1))) int gint;
    gint* gt = (gint*)gather;
    __asm__ volatile("" : "+s"(gt));
    int ga[8], gb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) ga[j] = gt[j * WAVE + lane];
#pragma unroll
    for (int i0 = 0; i0 < FR; i0 += 8) {
      if (i0 + 8 < FR) {
#pragma unroll
        for (int j = 0; j < 8; ++j) gb[j] = i0 + 8 + j < FR ? gt[(i0 + 8 + j) * WAVE + lane] : 0;
      }
      // only the rows that have them read a second and third source (the
      // others add exact zeros in the table's layout)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (i0 + j >= FR) continue;
        double a = L.src[ga[j] & 1023];
        if ((GATHER2 >> (i0 + j)) & 1ull) a += L.src[(ga[j] >> 10) & 1023];
        if ((GATHER3 >> (i0 + j)) & 1ull) a += L.src[(ga[j] >> 20) & 1023];
        v[i0 + j] = a;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) ga[j] = gb[j];
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    eliminate_stage<SPLIT>(v, slots + t * NK * SLOT, L.bc, npos, nneg, nzero);
    // contribution block to stage n+1 (rows/cols 43..60 of the coupling lanes)
    if (lane >= NK && lane < NK + NC) {
      const int a = lane - NK;
#pragma unroll
      for (int b = 0; b < NC + 2; ++b) L.src[SRC_CTB + a * (NC + 2) + b] = v[NK + b];
    }
    __syncthreads();
  }
  // ---------------- backward substitution over the stages, top to bottom
  L.xr[lane] = 0.0;  // solution of the stage above (none above the top stage)
  L.xb[lane] = 0.0;
  __syncthreads();
  double sigb = 0.0, sigr = 0.0, wdd = 0.0;
  for (int n = N - 1; n >= 0; --n) {
    const long long t = t0 + n;
    const double* sb = slots + t * NK * SLOT;
    double xr_s, xb_s;
    int p_s;
    backward_stage(sb, L.stg, L.xr, L.xb, true, xr_s, xb_s, p_s);
    // For the stored-factor solve: the entries of pivot column q at rows 0-15
    // (one 128-byte line) are all zero once every one of those rows has been
    // eliminated, i.e. for q at or past the last slot whose pivot lies there
    // (the pivot's own entry is stored as zero).  That slot, and the one for
    // rows 16-31, bound the columns whose line must be read.
    {
      const uint64_t in0 = __ballot(lane < NK && p_s < 16);
      const uint64_t in1 = __ballot(lane < NK && p_s >= 16 && p_s < 32);
      if (lane == 0) {
        lines[2 * t] = in0 ? 63 - __builtin_clzll(in0) : 0;
        lines[2 * t + 1] = in1 ? 63 - __builtin_clzll(in1) : 0;
      }
    }
    __syncthreads();
    if (lane < NK) {
      solr[t * NK + p_s] = xr_s;
      solb[t * NK + p_s] = xb_s;
      L.xr[p_s] = xr_s;
      L.xb[p_s] = xb_s;
    }
    __syncthreads();
    if (lane == NK - 1) {
      const double b = rec[t * REC + jd];
      sigb += b * L.xb[NK - 1];
      sigr += b * L.xr[NK - 1];
      wdd += rec[t * REC + REC_WDD];
    }
  }
  if (lane == NK - 1) {
    part[(long long)w * 4 + 0] = sigb;
    part[(long long)w * 4 + 1] = sigr;
    part[(long long)w * 4 + 2] = wdd;
    part[(long long)w * 4 + 3] = 0.0;
  }
  if (lane == 0) {
    inert[w * 4 + 0] = npos;
    inert[w * 4 + 1] = nneg;
    inert[w * 4 + 2] = nzero;
    inert[w * 4 + 3] = 0;
  }
}

// Forward and backward substitution with stored pivot columns for R right-hand
// sides at once (each stage's pivot columns are read once for all of them):
// solr[j] <- K_w^{-1} rhs[j], rhs[j] = rhs + j * stride, solr[j] likewise.
// With one right-hand side the border dot b . x goes to part (Schur on d).
template <int WPE, int R>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(WPE))) void k_solve(const double* __restrict__ rec, const double* __restrict__ slots, const int* __restrict__ lines,
                                                const double* __restrict__ rhs, const int* __restrict__ chain0,
                                                const int* __restrict__ chain_p, const int* __restrict__ pact,
                                                const int* __restrict__ chmask, int W, int jd, long long stride,
                                                int zero_masked, double* __restrict__ solr, double* __restrict__ part) {
  __shared__ double sh[R][WAVE];
  const int w = blockIdx.x;
  if (w >= W) return;
  const bool left_out = chmask && !chmask[w];
  if (left_out || (pact && !pact[chain_p[w]])) {  // not worked on: zero solution (rows on request)
    if (R == 1 && threadIdx.x == 0) part[(long long)w * 4 + 1] = 0.0;
    if (left_out || zero_masked)
      for (int j = 0; j < R; ++j)
        for (long long i = (long long)chain0[w] * NK + threadIdx.x; i < (long long)chain0[w + 1] * NK; i += WAVE)
          solr[j * stride + i] = 0.0;
    return;
  }
  const long long t0 = chain0[w];
  const int N = chain0[w + 1] - (int)t0;
  const int lane = lane_id();
  double ctb[R];  // contribution carried by coupling lane 43+a to stage n+1's index R[a]
#pragma unroll
  for (int j = 0; j < R; ++j) ctb[j] = 0.0;
  for (int n = 0; n < N; ++n) {
    const long long t = t0 + n;
    const double* sb = slots + t * NK * SLOT;
#pragma unroll
    for (int j = 0; j < R; ++j) sh[j][lane] = 0.0;
    __syncthreads();
    if (lane >= NK && lane < NK + NC)
#pragma unroll
      for (int j = 0; j < R; ++j) sh[j][coupling_index(lane - NK)] = ctb[j];
    __syncthreads();
    double r[R], ys[R];  // lane s keeps the forward value of slot s
#pragma unroll
    for (int j = 0; j < R; ++j) {
      r[j] = lane < NK ? rhs[j * stride + t * NK + lane] + sh[j][lane] : 0.0;
      ys[j] = 0.0;
    }
    // the stage's 43 pivot columns, all loads in flight at once (lane = row);
    // the lines of rows 0-15 and 16-31 only in the columns that can have
    // nonzeros there (the others are zero)
    const int l0 = lines[2 * t], l1 = lines[2 * t + 1];
    const int lim = lane < 16 ? l0 : lane < 32 ? l1 : NK;
    double col[NK];
#pragma unroll
    for (int q = 0; q < NK; ++q) col[q] = q < lim ? sb[q * SLOT + lane] : 0.0;
    bool skip = false;
#pragma unroll
    for (int q = 0; q < NK; ++q) {
      if (skip) {  // second slot of a 2x2 pivot, applied with the first
        skip = false;
        continue;
      }
      const double c = col[q];
      const int code = (int)rdl(c, FR);
      const int type = code >> 6, p = code & 63;
      const double cr = lane < FR_R ? c : 0.0;
      if (q + 1 < NK && type == 2) {
        const double cn = col[q + 1 < NK ? q + 1 : q];
        const int pq = ((int)rdl(cn, FR)) & 63;
        const double e11 = rdl(c, FR + 1), e12 = rdl(c, FR + 2), e22 = rdl(cn, FR + 1);
        const double idet = 1.0 / (e11 * e22 - e12 * e12);
        const double c1r = lane < FR_R ? cn : 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const double yk = rdl(r[j], p), yq = rdl(r[j], pq);
          if (lane == q) ys[j] = yk;
          if (lane == q + 1) ys[j] = yq;
          const double t1 = (e22 * yk - e12 * yq) * idet, t2 = (e11 * yq - e12 * yk) * idet;
          r[j] = fma(-cr, t1, fma(-c1r, t2, r[j]));
        }
        skip = true;
        continue;
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const double yp = rdl(r[j], p);
        if (lane == q) ys[j] = yp;
        if (type == 1) r[j] = fma(-cr, yp * rdl(c, FR + 2), r[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (lane < NK) solr[j * stride + t * NK + lane] = ys[j];  // forward values in slot order
      ctb[j] = (lane >= NK && lane < NK + NC) ? r[j] : 0.0;
    }
    __syncthreads();
  }
  // backward sweep
#pragma unroll
  for (int j = 0; j < R; ++j) sh[j][lane] = 0.0;
  __syncthreads();
  double sig = 0.0;
  for (int n = N - 1; n >= 0; --n) {
    const long long t = t0 + n;
    const double* sb = slots + t * NK * SLOT;
    double y[R];
    const double* xc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      y[j] = lane < NK ? solr[j * stride + t * NK + lane] : 0.0;
      xc[j] = sh[j];
    }
    double x[R];
    const int l0 = lines[2 * t], l1 = lines[2 * t + 1];
    const int lim = lane < 16 ? l0 : lane < 32 ? l1 : NK;
    backward_rows<R>(sb, lim, y, xc, x);
    __syncthreads();
    if (lane < NK)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        solr[j * stride + t * NK + lane] = x[j];
        sh[j][lane] = x[j];
      }
    __syncthreads();
    if (R == 1 && lane == NK - 1) sig += rec[t * REC + jd] * sh[0][NK - 1];
  }
  if (R == 1 && lane == NK - 1) part[(long long)w * 4 + 1] = sig;
}

// Schur complement on d.  Fixed-order reduction of the per-scenario partials:
// sigma_b = sum b^T K^{-1} b, sigma_r = sum b^T K^{-1} r, W_dd and the inertia.
// One block per problem: sums over the problem's chains (fixed order), then
// S_d = k_dd - sigma_b with k_dd = sum W_dd + Sigma_d + delta_w, the inertia
// (Haynsworth: the chains' counts plus the sign of S_d) and
// dd = (r_d - sigma_r) / S_d.
constexpr int SCHUR_BS = 1024;
__global__ __launch_bounds__(SCHUR_BS) void k_schur(const double* __restrict__ part, const int* __restrict__ inert,
                                                    const int* __restrict__ pchain, const double* __restrict__ diagd,
                                                    const double* __restrict__ dwv, const double* __restrict__ rd,
                                                    int mode, const int* __restrict__ pmask,
                                                    DevScalars* __restrict__ outv) {
  // mode 0: factor only; 1: factor with a right-hand side; 2: right-hand side only
  // The six sums (three of them integer counts, exact in double) run in a fixed
  // order: thread i takes chains i, i + SCHUR_BS, ... four at a time, then a
  // DPP tree inside each wave and across the waves.
  __shared__ double sm[6][SCHUR_BS / 64];
  const int pb = blockIdx.x;
  if (pmask && !pmask[pb]) return;  // this problem keeps its scalars
  const int w0 = pchain[pb], w1 = pchain[pb + 1];
  DevScalars* out = outv + pb;
  double a[6] = {0, 0, 0, 0, 0, 0};
  int w = w0 + (int)threadIdx.x;
  for (; w + 3 * SCHUR_BS < w1; w += 4 * SCHUR_BS) {
    double q[4][6];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long c = (long long)(w + j * SCHUR_BS) * 4;
      q[j][0] = part[c];
      q[j][1] = part[c + 1];
      q[j][2] = part[c + 2];
      q[j][3] = inert[c];
      q[j][4] = inert[c + 1];
      q[j][5] = inert[c + 2];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] += q[j][k];
  }
  for (; w < w1; w += SCHUR_BS) {
    const long long c = (long long)w * 4;
    a[0] += part[c];
    a[1] += part[c + 1];
    a[2] += part[c + 2];
    a[3] += inert[c];
    a[4] += inert[c + 1];
    a[5] += inert[c + 2];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) a[k] = wave_reduce(0, a[k]);
  if (lane == 63)
    for (int k = 0; k < 6; ++k) sm[k][wv] = a[k];
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int k = 0; k < 6; ++k) a[k] = rdl(wave_reduce(0, lane < SCHUR_BS / 64 ? sm[k][lane] : 0.0), 63);
  const double sb0 = a[0], sr0 = a[1], sw0 = a[2];
  if (threadIdx.x == 0) {
    if (mode != 2) {
      out->sig_b = sb0;
      out->wdd = sw0;
      out->kdd = sw0 + diagd[pb] + dwv[pb];
      out->sd = out->kdd - sb0;
      long long np = (long long)a[3], nn = (long long)a[4], nz = (long long)a[5];
      if (out->sd > 0.0) ++np;
      else if (out->sd < 0.0) ++nn;
      else ++nz;
      out->npos = np;
      out->nneg = nn;
      out->nzero = nz;
    }
    if (mode != 0) {
      out->sig_r = sr0;
      out->rd = rd[pb];
      out->dd = (rd[pb] - sr0) / out->sd;
    }
  }
}

// sol = solr - solb * dd_p on the stage entries, sol[d_p] = dd_p
__global__ void k_combine(const double* __restrict__ solr, const double* __restrict__ solb,
                          const DevScalars* __restrict__ sc, const StageInfo* __restrict__ sinfo, long long nk,
                          int P, const int* __restrict__ pmask, double* __restrict__ sol) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nk) {
    const int p = sinfo[i / NK].p;
    if (!pmask || pmask[p]) sol[i] = solr[i] - solb[i] * sc[p].dd;
  } else if (i < nk + P) {
    if (!pmask || pmask[i - nk]) sol[i] = sc[i - nk].dd;
  }
}

// ---------------------------------------------------------------- design vector (npar > 1)
// With one diameter per column section the border of a scenario block has one
// column b_k per section (nonzero at the hydraulic-dual rows of that section's
// stages).  The factorisation solves with b_0; the other columns are solved
// with the stored factors; the Schur complement S = K_dd - sum_w B^T K_w^{-1} B
// is a dense npar x npar matrix per problem.

// right-hand side holding the border column of section k
__global__ void k_border_rhs(const double* __restrict__ rec, const StageInfo* __restrict__ sinfo, long long nks,
                             long long nkkt, int jd, int npar, int k, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nkkt) return;
  double v = 0.0;
  if (i < nks && i % NK == NK - 1) {
    const long long t = i / NK;
    const StageInfo si = sinfo[t];
    if (section_of(si.n, si.N, npar) == k) v = rec[t * REC + jd];
  }
  out[i] = v;
}

// per chain (one thread each): mode 0/1: b_k . v_l, b_k . u and W_dd per
// section; mode 2: b_k . u only (u: the solution with the right-hand side)
__global__ void k_design_dots(int mode, const double* __restrict__ rec, const int* __restrict__ chain0,
                              const int* __restrict__ chain_p, int W, int jd, int npar, long long nks,
                              const double* __restrict__ solr, const double* __restrict__ solb,
                              const double* __restrict__ solbk, const int* __restrict__ pmask,
                              double* __restrict__ pdots) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  if (pmask && !pmask[chain_p[w]]) return;
  const long long t0 = chain0[w];
  const int N = chain0[w + 1] - (int)t0;
  double S[MAX_NPAR * MAX_NPAR], r[MAX_NPAR], wd[MAX_NPAR];
#pragma unroll
  for (int q = 0; q < MAX_NPAR * MAX_NPAR; ++q) S[q] = 0.0;
#pragma unroll
  for (int q = 0; q < MAX_NPAR; ++q) r[q] = wd[q] = 0.0;
  for (int n = 0; n < N; ++n) {
    const long long t = t0 + n;
    const int k = section_of(n, N, npar);
    const double bn = rec[t * REC + jd];
    const long long hy = t * NK + NK - 1;
    const double u = bn * solr[hy];
#pragma unroll
    for (int q = 0; q < MAX_NPAR; ++q) r[q] += q == k ? u : 0.0;
    if (mode != 2) {
      const double wdd = rec[t * REC + REC_WDD];
#pragma unroll
      for (int q = 0; q < MAX_NPAR; ++q) wd[q] += q == k ? wdd : 0.0;
#pragma unroll
      for (int l = 0; l < MAX_NPAR; ++l) {
        if (l >= npar) break;
        const double v = bn * (l == 0 ? solb[hy] : solbk[(long long)(l - 1) * nks + hy]);
#pragma unroll
        for (int q = 0; q < MAX_NPAR; ++q) S[q * MAX_NPAR + l] += q == k ? v : 0.0;
      }
    }
  }
  double* o = pdots + (long long)w * PDOT;
  if (mode != 2) {
#pragma unroll
    for (int q = 0; q < MAX_NPAR * MAX_NPAR; ++q) o[q] = S[q];
#pragma unroll
    for (int q = 0; q < MAX_NPAR; ++q) o[MAX_NPAR * MAX_NPAR + MAX_NPAR + q] = wd[q];
  }
#pragma unroll
  for (int q = 0; q < MAX_NPAR; ++q) o[MAX_NPAR * MAX_NPAR + q] = r[q];
}

// eigenvalues of a symmetric n x n matrix (n <= MAX_NPAR) by cyclic Jacobi
// rotations (a fixed number of sweeps: deterministic)
// (loops over the static bound MAX_NPAR with guards, so that every index is a
// compile-time constant and the matrix stays in registers)
__device__ void sym_eigenvalues(double (&A)[MAX_NPAR][MAX_NPAR], int n, double (&ev)[MAX_NPAR]) {
  for (int sweep = 0; sweep < 30; ++sweep)
#pragma unroll
    for (int p = 0; p < MAX_NPAR - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < MAX_NPAR; ++q) {
        if (q >= n) continue;
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
        for (int k = 0; k < MAX_NPAR; ++k) {  // rotate columns p, q (entries past n stay 0)
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < MAX_NPAR; ++k) {  // rotate rows p, q
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
      }
#pragma unroll
  for (int k = 0; k < MAX_NPAR; ++k) ev[k] = A[k][k];
}

// per problem (one wave each): fixed-order sums of the chains' partials, then
// mode 0/1: S, its inertia (plus the chains' counts) and the K_dd diagonal;
// mode 1/2: delta theta = S^{-1} (r_theta - sum b_k . u) by Gaussian
// elimination with partial pivoting
constexpr int DSCH_BS = 256;
__global__ __launch_bounds__(DSCH_BS) void k_design_schur(int mode, const double* __restrict__ pdots,
                                                          const int* __restrict__ inert,
                                                          const int* __restrict__ pchain,
                                                          const double* __restrict__ diagx, long long nxs,
                                                          const double* __restrict__ dwv,
                                                          const double* __restrict__ rhs, long long nks, int npar,
                                                          const int* __restrict__ pmask,
                                                          DevScalars* __restrict__ scal, double* __restrict__ dsc) {
  constexpr int NQ = PDOT + 3;
  __shared__ double sm[NQ][DSCH_BS / 64];
  const int pb = blockIdx.x;
  if (pmask && !pmask[pb]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double a[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) a[q] = 0.0;
  // thread i takes chains i, i + DSCH_BS, ...; then a fixed shuffle tree in each
  // wave and across the waves
  for (int w = pchain[pb] + (int)threadIdx.x; w < pchain[pb + 1]; w += DSCH_BS) {
    const double* o = pdots + (long long)w * PDOT;
    if (mode != 2) {
#pragma unroll
      for (int q = 0; q < PDOT; ++q) a[q] += o[q];
      a[PDOT] += inert[w * 4];
      a[PDOT + 1] += inert[w * 4 + 1];
      a[PDOT + 2] += inert[w * 4 + 2];
    } else {
#pragma unroll
      for (int q = 0; q < MAX_NPAR; ++q) a[MAX_NPAR * MAX_NPAR + q] += o[MAX_NPAR * MAX_NPAR + q];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] += __shfl_down(a[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sm[q][wv] = a[q];
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    a[q] = lane < DSCH_BS / 64 ? sm[q][lane] : 0.0;
#pragma unroll
    for (int off = DSCH_BS / 128; off > 0; off >>= 1) a[q] += __shfl_down(a[q], off, 64);
  }
  if (lane != 0) return;
  double* D = dsc + (long long)pb * DSC;
  double* Sst = D;                                   // S [MAX_NPAR][MAX_NPAR]
  double* dth = D + MAX_NPAR * MAX_NPAR;             // delta theta
  double* wst = dth + MAX_NPAR;                      // W_dd per section
  double* kdg = wst + MAX_NPAR;                      // K_dd diagonal
  const long long ib = (long long)pb * npar;
  if (mode != 2) {
    // (static loops with guards: the partial sums stay in registers)
    double A[MAX_NPAR][MAX_NPAR] = {};
    double amax = 1.0;
#pragma unroll
    for (int k = 0; k < MAX_NPAR; ++k) {
      if (k >= npar) continue;
      const double wk = a[MAX_NPAR * MAX_NPAR + MAX_NPAR + k];
      const double kd = wk + diagx[nxs + ib + k] + dwv[pb];
      wst[k] = wk;
      kdg[k] = kd;
      amax = fmax(amax, fabs(kd));
#pragma unroll
      for (int l = 0; l < MAX_NPAR; ++l) {
        if (l >= npar) continue;
        const double sym = 0.5 * (a[k * MAX_NPAR + l] + a[l * MAX_NPAR + k]);
        A[k][l] = (k == l ? kd : 0.0) - sym;
        Sst[k * MAX_NPAR + l] = A[k][l];
      }
    }
    double ev[MAX_NPAR];
    sym_eigenvalues(A, npar, ev);
    long long np = (long long)a[PDOT], nn = (long long)a[PDOT + 1], nz = (long long)a[PDOT + 2];
    const double tiny = 1e-20 * amax;
#pragma unroll
    for (int k = 0; k < MAX_NPAR; ++k) {
      if (k >= npar) continue;
      if (ev[k] > tiny) ++np;
      else if (ev[k] < -tiny) ++nn;
      else ++nz;
    }
    DevScalars& o = scal[pb];
    o.npos = np;
    o.nneg = nn;
    o.nzero = nz;
    o.kdd = kdg[0];
    o.sd = ev[0];
  }
  if (mode != 0) {
    // Gaussian elimination with partial pivoting on S padded to MAX_NPAR x
    // MAX_NPAR with an identity block (block diagonal: the padding neither wins a
    // pivot search nor changes the solution); static indices keep it in registers
    double A[MAX_NPAR][MAX_NPAR], b[MAX_NPAR], xs[MAX_NPAR];
#pragma unroll
    for (int k = 0; k < MAX_NPAR; ++k) {
      b[k] = k < npar ? rhs[nks + ib + k] - a[MAX_NPAR * MAX_NPAR + k] : 0.0;
#pragma unroll
      for (int l = 0; l < MAX_NPAR; ++l)
        A[k][l] = (k < npar && l < npar) ? Sst[k * MAX_NPAR + l] : (k == l ? 1.0 : 0.0);
    }
#pragma unroll
    for (int c = 0; c < MAX_NPAR; ++c) {
      int piv = c;
      double best = fabs(A[c][c]);
#pragma unroll
      for (int r = c + 1; r < MAX_NPAR; ++r)
        if (fabs(A[r][c]) > best) {
          best = fabs(A[r][c]);
          piv = r;
        }
#pragma unroll
      for (int r = c + 1; r < MAX_NPAR; ++r)
        if (r == piv) {
#pragma unroll
          for (int l = 0; l < MAX_NPAR; ++l) {
            const double tmp = A[c][l];
            A[c][l] = A[r][l];
            A[r][l] = tmp;
          }
          const double tb = b[c];
          b[c] = b[r];
          b[r] = tb;
        }
#pragma unroll
      for (int r = c + 1; r < MAX_NPAR; ++r) {
        const double f = A[r][c] / A[c][c];
#pragma unroll
        for (int l = c; l < MAX_NPAR; ++l) A[r][l] -= f * A[c][l];
        b[r] -= f * b[c];
      }
    }
#pragma unroll
    for (int c = MAX_NPAR - 1; c >= 0; --c) {
      double v = b[c];
#pragma unroll
      for (int l = c + 1; l < MAX_NPAR; ++l) v -= A[c][l] * xs[l];
      xs[c] = v / A[c][c];
    }
#pragma unroll
    for (int k = 0; k < MAX_NPAR; ++k)
      if (k < npar) dth[k] = xs[k];
  }
}

// sol = u - sum_l v_l delta theta_l on the stage entries, delta theta on the design entries
__global__ void k_design_combine(const double* __restrict__ solr, const double* __restrict__ solb,
                                 const double* __restrict__ solbk, const double* __restrict__ dsc,
                                 const StageInfo* __restrict__ sinfo, long long nks, int P, int npar,
                                 const int* __restrict__ pmask, double* __restrict__ sol) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nks) {
    const int p = sinfo[i / NK].p;
    if (pmask && !pmask[p]) return;
    const double* dth = dsc + (long long)p * DSC + MAX_NPAR * MAX_NPAR;
    double v = solr[i] - solb[i] * dth[0];
    for (int l = 1; l < npar; ++l) v -= solbk[(long long)(l - 1) * nks + i] * dth[l];
    sol[i] = v;
  } else if (i < nks + (long long)P * npar) {
    const long long j = i - nks;
    const int p = (int)(j / npar);
    if (pmask && !pmask[p]) return;
    sol[i] = dsc[(long long)p * DSC + MAX_NPAR * MAX_NPAR + (j % npar)];
  }
}

}  // namespace

// ---------------------------------------------------------------- launch wrappers
hipError_t launch_factor(Handle& h, const double* diagx, const double* diags, const double* rhs, bool mask,
                         hipStream_t st, int nchain) {
  const int* fm = mask ? h.fmask : nullptr;
  const int nw = nchain < 0 || nchain > h.S ? h.S : nchain;
  prof_begin(h, 0, st);
#define ABS_FACTOR(S, W)                                                                                    \
  hipLaunchKernelGGL((k_factor<S, W>), dim3(nw), dim3(WAVE), 0, st, h.rec, h.gather, rhs, diagx, diags, h.dwv, \
                     h.dcv, h.chain0, h.chain_p, fm, h.chmask, nw, h.jac_d_index, h.npar, h.slots, h.slot_lines, \
                     h.solr, h.solb, \
                     h.inert, h.part)
  // launch shape: occupancy target (waves per SIMD 2 or 3) and row split of the update
  const int wpe = h.tune.factor_wpe, split = h.tune.factor_split;
  if (wpe == 2) {
    if (split == 1) ABS_FACTOR(1, 2);
    else if (split == 2) ABS_FACTOR(2, 2);
    else ABS_FACTOR(0, 2);
  } else {
    if (split == 1) ABS_FACTOR(1, 3);
    else if (split == 2) ABS_FACTOR(2, 3);
    else ABS_FACTOR(0, 3);
  }
#undef ABS_FACTOR
  prof_end(h, 0, st);
  h.factored = true;
  ++h.n_factor;
  return hipGetLastError();
}

hipError_t launch_solve(Handle& h, const double* rhs, hipStream_t st, int nchain, double* out, int nrhs,
                        long long stride, bool zero_masked) {
  const int nw = nchain < 0 || nchain > h.S ? h.S : nchain;
  double* const xo = out ? out : h.solr;
  if (nrhs < 1 || nrhs > MAX_NPAR - 1 || (nrhs > 1 && !out)) return hipErrorInvalidValue;
  prof_begin(h, 1, st);
  const int* pa = h.pact_on ? h.pact : nullptr;
#define ABS_SOLVE(W, RR)                                                                                          \
  hipLaunchKernelGGL((k_solve<W, RR>), dim3(nw), dim3(WAVE), 0, st, h.rec, h.slots, h.slot_lines, rhs, h.chain0,  \
                     h.chain_p, pa,                                                                             \
                     h.chmask, nw, h.jac_d_index, stride, zero_masked ? 1 : 0, xo, h.part)
  // several right-hand sides need about 190-210 VGPRs: 2 waves per SIMD (a
  // higher target would spill)
  if (nrhs == 2) ABS_SOLVE(2, 2);
  else if (nrhs == 3) ABS_SOLVE(2, 3);
  else if (h.tune.solve_wpe == 2) ABS_SOLVE(2, 1);
  else if (h.tune.solve_wpe == 4) ABS_SOLVE(4, 1);
  else ABS_SOLVE(3, 1);
#undef ABS_SOLVE
  prof_end(h, 1, st);
  ++h.n_solve;
  return hipGetLastError();
}

static hipError_t launch_design_schur(Handle& h, const double* diagx, const double* rhs, int mode, double* sol,
                                      hipStream_t st, const int* pmask) {
  const long long nks = h.nst * NK;
  if (mode != 2) {  // the other sections' border columns with the stored factors, in one pass
    for (int k = 1; k < h.npar; ++k)
      hipLaunchKernelGGL(k_border_rhs, dim3(grid_for(nks, 256)), dim3(256), 0, st, h.rec, h.sinfo, nks, nks,
                         h.jac_d_index, h.npar, k, h.brhs + (long long)(k - 1) * nks);
    const hipError_t e = launch_solve(h, h.brhs, st, -1, h.solbk, h.npar - 1, nks);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_design_dots, dim3(grid_for(h.S, 64)), dim3(64), 0, st, mode, h.rec, h.chain0, h.chain_p, h.S,
                     h.jac_d_index, h.npar, nks, h.solr, h.solb, h.solbk, pmask, h.pdots);
  hipLaunchKernelGGL(k_design_schur, dim3(h.P), dim3(DSCH_BS), 0, st, mode, h.pdots, h.inert, h.pchain, diagx,
                     h.nst * NV, h.dwv, rhs, nks, h.npar, pmask, h.scal, h.dsc);
  if (mode != 0 && sol)
    hipLaunchKernelGGL(k_design_combine, dim3(grid_for(h.nkkt, 256)), dim3(256), 0, st, h.solr, h.solb, h.solbk,
                       h.dsc, h.sinfo, nks, h.P, h.npar, pmask, sol);
  return hipGetLastError();
}

hipError_t launch_schur(Handle& h, const double* diagx, const double* rhs, int mode, double* sol, hipStream_t st,
                        const int* pmask) {
  if (h.npar > 1) return launch_design_schur(h, diagx, rhs, mode, sol, st, pmask);
  const double* rd = rhs ? rhs + h.nst * NK : nullptr;
  hipLaunchKernelGGL(k_schur, dim3(h.P), dim3(SCHUR_BS), 0, st, h.part, h.inert, h.pchain, diagx + h.nst * NV, h.dwv, rd,
                     mode, pmask, h.scal);
  if (mode != 0 && sol) {
    const long long nk = h.nst * NK;
    hipLaunchKernelGGL(k_combine, dim3(grid_for(nk + h.P, 256)), dim3(256), 0, st, h.solr, h.solb, h.scal, h.sinfo,
                       nk, h.P, pmask, sol);
  }
  return hipGetLastError();
}

}  // namespace absorber
