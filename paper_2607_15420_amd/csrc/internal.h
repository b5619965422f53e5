// Internal declarations of the absorber library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/absorber.h"
#include "model.h"

namespace absorber {

// per-stage record written by the evaluation kernel (all entries scaled)
constexpr int NJO = 107;  // OWN Jacobian entries incl. the hydraulic d-entry
constexpr int NJU = 29;   // UP entries
constexpr int NJD = 14;   // DOWN entries
constexpr int REC_OWN = 0, REC_UP = NJO, REC_DOWN = NJO + NJU, REC_H = NJO + NJU + NJD;
constexpr int REC_WDD = REC_H + NH;  // this stage's contribution to the (d,d) Hessian entry
constexpr int REC = REC_WDD + 1;     // 199 doubles

// frontal matrix of one stage: 43 own indices, 16 coupling indices of the
// next stage, 2 right-hand sides (r and the border b)
constexpr int NC = 16;
constexpr int FR = NK + NC + 2;  // 61 rows/cols
constexpr int FR_R = NK + NC;    // row 59: right-hand side r
constexpr int FR_B = FR_R + 1;   // row 60: border b
constexpr int SLOT = 64;         // doubles per stored pivot column (61 + 3 info)

// LDS source array of the gather assembly (per wave)
constexpr int SRC_ZERO = 0;
constexpr int SRC_REC = 1;                    // record of stage n (REC)
constexpr int SRC_DOWN1 = SRC_REC + REC;      // DOWN entries of stage n+1 (14)
constexpr int SRC_RHS = SRC_DOWN1 + NJD;      // right-hand side (43)
constexpr int SRC_BRD = SRC_RHS + NK;         // border entry at the hydraulic dual (1)
constexpr int SRC_DIAGX = SRC_BRD + 1;        // Sigma_x + delta_w (21)
constexpr int SRC_DC = SRC_DIAGX + NV;        // -delta_c (1)
constexpr int SRC_DHYD = SRC_DC + 1;          // -(1/(Sigma_s+delta_w) + delta_c) (1)
constexpr int SRC_CTB = SRC_DHYD + 1;         // contribution block 16 x 18
constexpr int NSRC = SRC_CTB + NC * (NC + 2); // 569
// Frontal rows whose positions take a second (GATHER2) or third (GATHER3)
// gather source in some column: every other row has at most one.  A property
// of the stage's KKT structure; the table builder rejects a table that needs more.
constexpr unsigned long long GATHER2 = 0x8000200f000a1ffull;
constexpr unsigned long long GATHER3 = 0x81ffull;

// Residual term table (one list of products K_ij x_j per KKT row of a stage):
// [NK] rows in decreasing term count, [NK + 1] starts of their lists, then per
// term a coefficient code (LDS offset from the stage's record + RT_COFF, or
// RT_DIAG + index of the stage's diagonal block) and an unknown code (LDS
// offset from the stage's unknowns + RT_XOFF, RT_XDTERM for d; RT_NBDN / RT_NBUP
// mark a neighbour below / above).
constexpr int RT_COFF = 256, RT_DIAG = 1024, RT_XOFF = 64, RT_XDTERM = 256, RT_NBDN = 512, RT_NBUP = 1024;
constexpr int RT_MAX = 2048;

// the 16 stage-local KKT indices that receive the contribution of the stage below
__host__ __device__ constexpr int coupling_index(int a) {
  return a < 9 ? a : (a == 9 ? IL : (a == 10 ? IT : (a < 15 ? NV + 7 + (a - 11) : NV + 20)));
}

struct JacEntry { int8_t row, blk, col; };

// Design vector: one diameter per column section (npar sections of near-equal
// height; stage n of an N-stage chain is in section n npar / N).  npar = 1 is
// the single shared diameter of problem (10).
constexpr int MAX_NPAR = 4;
__host__ __device__ __forceinline__ int section_of(int n, int N, int npar) { return (n * npar) / N; }

// reduction operations: 0 sum, 1 maximum, 2 minimum
__device__ __forceinline__ double red_op(int op, double a, double b) {
  return op == 0 ? a + b : (op == 1 ? fmax(a, b) : fmin(a, b));
}

// One step of a wave reduction through DPP: v = v op (v of the lane the
// control selects); a lane without a source, or in a row the mask leaves out,
// sees the identity idn.
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_step(int op, double v, double idn) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(idn), __double2loint(v), CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(idn), __double2hiint(v), CTRL, RM, 0xf, false);
  return red_op(op, v, __hiloint2double(hi, lo));
}

// Wave reduction in a fixed order (row shifts, then row broadcasts); lane 63
// ends with the result.
__device__ __forceinline__ double wave_reduce(int op, double v) {
  const double idn = op == 0 ? 0.0 : (op == 1 ? -INFINITY : INFINITY);
  v = dpp_step<0x111, 0xf>(op, v, idn);  // row_shr:1
  v = dpp_step<0x112, 0xf>(op, v, idn);  // row_shr:2
  v = dpp_step<0x114, 0xf>(op, v, idn);  // row_shr:4
  v = dpp_step<0x118, 0xf>(op, v, idn);  // row_shr:8
  v = dpp_step<0x142, 0xa>(op, v, idn);  // row_bcast:15
  v = dpp_step<0x143, 0xc>(op, v, idn);  // row_bcast:31
  return v;
}

// Block-wide copy of n (1 <= n <= CAP) elements from global memory to LDS in
// two halves: load() issues every load of the thread (threads past n reread
// element n - 1), store() writes them.  Issuing the loads of several arrays
// before their stores costs one memory round trip instead of one per pass.
template <int BSZ, int CAP, class T>
struct LdsStage {
  static constexpr int K = (CAP + BSZ - 1) / BSZ;
  T v[K];
  __device__ __forceinline__ void load(const T* __restrict__ src, int n, int tid) {
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int i = tid + u * BSZ;
      v[u] = src[i < n ? i : n - 1];
    }
  }
  __device__ __forceinline__ void store(T* dst, int n, int tid) const {
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int i = tid + u * BSZ;
      if (i < n) dst[i] = v[u];
    }
  }
};
// per-problem design data of the Schur complement for npar > 1 (doubles):
// [S (npar^2)][delta theta (npar)][W_dd per section (npar)][K_dd diagonal (npar)]
constexpr int DSC = MAX_NPAR * MAX_NPAR + 3 * MAX_NPAR;
// per-chain partial sums for npar > 1: [b_k . v_l (npar^2)][b_k . u (npar)][W_dd per section (npar)]
constexpr int PDOT = MAX_NPAR * MAX_NPAR + 2 * MAX_NPAR;

constexpr int CTL_SLOT = 64;  // bytes of solver scalars per problem in the control block
inline size_t ctl_off_fmask(int P) { return 16 * (size_t)P; }
inline size_t ctl_off_pact(int P) { return 20 * (size_t)P; }
inline size_t ctl_off_slot(int P) { return ((24 * (size_t)P + 63) / 64) * 64; }
inline size_t ctl_size(int P) { return ctl_off_slot(P) + (size_t)CTL_SLOT * P; }

// A handle holds P independent problems (P = 1 for absorber_create).  Their
// scenarios ("chains" of stages) are stored problem after problem, each chain's
// stages contiguous and bottom to top; the primal vector is [21 entries per
// stage; d of problem 0..P-1], the rows [22 per stage], the KKT unknowns
// [43 per stage; d of problem 0..P-1].
struct StageInfo {
  int w, n, N, p;  // chain, stage within the chain, chain length, problem
};
// IPM work unit: at most SEG consecutive stages of one problem, so that one
// 256-thread block covers their primal (21 SEG), row (22 SEG) and stage entries
// (the design entries on its last MAX_NPAR threads: 21 SEG + MAX_NPAR <= 256)
// and the block's partial reductions belong to a single problem
constexpr int SEG = 11;
static_assert(NV * SEG + MAX_NPAR <= 256, "a segment block must hold its primal and design entries");
struct Seg {
  int t0, t1, p, first;  // stage range, problem, npar for the problem's first segment (it also owns the design entries), else 0
};

// scalars produced by the Schur/inertia reduction (one per problem)
struct DevScalars {
  double sd, kdd, sig_b, sig_r, dd, rd, wdd, pad0;
  long long npos, nneg, nzero, pad1;
};

// scaling applied to the NLP: x = D * xt per stage-local index, rows times cs
struct Scaling {
  double D[NV];
  double Dd;
};

// launch shapes picked by measurement (autotune)
struct Tune {
  int factor_wpe = 3, factor_split = 0, solve_wpe = 3, eval_bs = 128;
  bool done = false;
  float ms_factor[2][3] = {{0, 0, 0}, {0, 0, 0}};  // [waves per SIMD 2, 3][row split 0-2]
  float ms_solve[3] = {0, 0, 0}, ms_eval[3] = {0, 0, 0};
};

// all per-handle device and host state
struct Handle {
  int P = 1;                                 // independent problems
  int npar = 1;                              // design variables per problem (section diameters)
  double cw[MAX_NPAR] = {1, 0, 0, 0};        // design-cost weight of each section diameter (its share of stages)
  bool has_op = false;                       // the objective carries the expected operating cost sum a theta^-4
  std::vector<double> opa_h;                 // [P * npar] its coefficients a_k (host)
  double* opa = nullptr;                     // device copy
  int N = 0, S = 0;                          // P == 1: stages and scenarios; otherwise the largest
                                             // stage count and the number of chains
  long long nst = 0;                         // stages of all problems
  long long nx = 0, nc = 0, nkkt = 0;       // primal incl. the d's, rows, KKT unknowns incl. the d's
  std::vector<int> pN, pS;                   // per problem: stages, scenarios
  std::vector<long long> pstage_h, pchain_h; // [P+1] first stage / first chain of each problem
  std::vector<int> pseg_h;                   // [P+1] first segment of each problem
  StageInfo* sinfo = nullptr;                // device [nst]
  int* chain0 = nullptr;                     // device [chains+1] first stage of each chain
  int* chain_p = nullptr;                    // device [chains] problem of each chain
  int* pchain = nullptr;                     // device [P+1]
  long long* pstage = nullptr;               // device [P+1]
  Seg* seg = nullptr;                        // device [nseg]
  int* pseg = nullptr;                       // device [P+1]
  int nseg = 0;
  // per-problem control arrays, one device block (ctl) with a pinned host copy
  // (ctl_h) of the same layout, so that they travel in one transfer:
  // [dwv P doubles][dcv P doubles][fmask P ints][pact P ints][CTL_SLOT bytes per problem]
  char* ctl = nullptr;
  char* ctl_h = nullptr;
  hipEvent_t ctl_ev = nullptr;  // recorded after each upload of ctl_h; waited on before ctl_h is rewritten
  bool ctl_ev_rec = false;      // ctl_ev has been recorded
  size_t ctl_bytes = 0;
  double* dwv = nullptr;                     // device [P] delta_w of the stored factorisation
  double* dcv = nullptr;                     // device [P] delta_c
  int* fmask = nullptr;                      // device [P] problems to (re)factorise (null: all)
  int* pact = nullptr;                       // device [P] problems the per-stage kernels work on
  char* slot_area = nullptr;                 // device [P][CTL_SLOT] the solver's per-problem scalars
  bool pact_on = false;                      // false: every problem
  int* chmask = nullptr;                     // device [chains] or null: chains the factorisation and the
                                             // stored-factor solve work on (the others get zero solutions)
  // batched refinement: per-problem max |res| and max |rhs| of the last residual,
  // and the problems a correction is computed for (the others are converged)
  double* pres = nullptr;                    // device [2P]
  double* pres_h = nullptr;                  // pinned [2P]
  int* rmask = nullptr;                      // device [P]
  int* rmask_h = nullptr;                    // pinned [2P]: kept-candidate mask, then refining mask (an async copy
                                             // reads its source when it runs, so the two never share memory)
  ModelParams mp{};
  double xL[NV], xU[NV], dL = 0, dU = 0;     // unscaled bounds per local variable
  std::vector<double> feeds_h;
  double* feeds = nullptr;                   // device [S][NF]
  std::vector<JacEntry> jac_own, jac_up, jac_down;  // per-stage Jacobian structure
  int jac_d_index = -1;                      // position of the d entry within OWN
  HessPos hpos[NH];
  int* gather = nullptr;                     // device [FR][64] packed gather table
  int* jtab = nullptr;                       // device packed Jacobian structure (row, col) per entry
  int* rtab = nullptr;                       // device residual term table (RT_*)
  int rtab_n = 0;
  int* gtab = nullptr;                       // device J^T y term table: [NV + 1] starts, then (coef, row) codes
  int gtab_n = 0;
  Scaling sc{};
  double* cs = nullptr;                      // device [S][N][NR] row scaling
  double sf = 1.0;
  // work buffers
  double* rec = nullptr;                     // [S][N][REC]
  double* slots = nullptr;                   // [S][N][NK][SLOT] stored pivot columns
  int* slot_lines = nullptr;                 // [S][N][2] per stage: the pivot columns that may hold nonzeros in
                                             // rows 0-15 / 16-31 (the leading ones; see k_factor)
  double* solr = nullptr;                    // [S][N][NK] K_w^{-1} r
  double* solb = nullptr;                    // [S][N][NK] K_w^{-1} b (for npar > 1: the border of section 0)
  double* solbk = nullptr;                   // npar > 1: [npar - 1][S][N][NK] K_w^{-1} b_k of sections 1..
  double* brhs = nullptr;                    // npar > 1: [npar - 1][43 nst] borders of sections 1.. as right-hand sides
  double* pdots = nullptr;                   // npar > 1: [chains][PDOT] per-chain partial sums
  double* dsc = nullptr;                     // npar > 1: [P][DSC] Schur complement data per problem
  int* inert = nullptr;                      // [chains][4]
  double* part = nullptr;                    // [chains][4] per-chain partial sums
  DevScalars* scal = nullptr;                // device scalars [P]
  DevScalars* scal_h = nullptr;              // pinned host mirror [P]
  double* diagx = nullptr;                   // [nx] Sigma_x for the KKT (scaled)
  double* diags = nullptr;                   // [S][N] Sigma_s
  double* kres = nullptr;                    // [nkkt] refinement residual
  double* kcor = nullptr;                    // [nkkt] second iterate buffer of the refinement
  double* kden = nullptr;                    // residual partials: 2 per stage, block maxima, per-problem d rows
  double* omega_d = nullptr;                 // [4] of the last residual: backward errors (rows, d rows), max |res|, max |rhs|
  double last_omega = 0.0;                   // componentwise backward error of the last refined solve
  Tune tune;
  double* redbuf = nullptr;                  // device reduction partials
  double* redbuf_h = nullptr;                // pinned host mirror
  int red_cap = 0;
  hipStream_t stream = nullptr;
  bool factored = false;
  double last_diag_d = 0;
  double x0[NV + 1];                         // cold-start stage vector and diameter
  float* warm_X = nullptr;                   // warm-start workspaces (allocated on first use)
  float* warm_Y = nullptr;
  double* warm_x0 = nullptr;
  double* warm_l0 = nullptr;
  int* warm_w = nullptr;
  // work vectors of the interior-point solve: one device allocation made on the
  // handle's first solve and kept (cleared at the start of every solve), and a
  // pinned [P] array for reading the d entries
  double* ipm_work = nullptr;
  size_t ipm_work_bytes = 0;
  double* ipm_dd_h = nullptr;
  long long n_factor = 0, n_solve = 0;       // launch counters
  std::vector<std::vector<absorber_ipm_log_entry>> ipm_log;  // per problem: accepted iterations of the last solve
  void* ipm_graph = nullptr;  // captured iteration graphs and their device control state (ipm.hip)
  // optional per-class kernel timing: event pairs recorded on the launch stream
  // and read back only when the profile is fetched (or the pending list is full)
  int prof = 0;  // bit mask of the profiled kernel classes
  hipEvent_t prof_open = nullptr;  // begin event of the launch being timed
  struct ProfPair {
    hipEvent_t e0, e1;
    int cls;
  };
  std::vector<ProfPair> prof_pending;
  std::vector<hipEvent_t> prof_pool;  // recorded events whose times have been read
  double prof_ms[4] = {0, 0, 0, 0};
  long long prof_calls[4] = {0, 0, 0, 0};
};

void set_error(const std::string& msg);
// Wait for the work queued on st by polling it: the solver's per-iteration
// reads of a few reduced scalars return as soon as the copy has landed,
// without the wake-up latency of a blocking wait.
hipError_t wait_stream(hipStream_t st);
// bracket a launch of class cls with profiling events (no-ops unless the class
// is profiled); prof_flush waits for the pending events and sums their times
void prof_begin(Handle& h, int cls, hipStream_t st);
void prof_end(Handle& h, int cls, hipStream_t st);
int prof_flush(Handle& h);
int initial_point(Handle& h, double* x_dev, hipStream_t st);

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      ::absorber::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));         \
      return ABS_ERR_HIP;                                                               \
    }                                                                                   \
  } while (0)

// ---- launch wrappers (kernels.hip)
// x: primal vector; scaled != 0 means x holds xt with x = D * xt.
// y: multipliers of the scaled rows [S][N][NR] (nullptr: no Hessian weights)
hipError_t launch_eval(Handle& h, const double* x, int scaled, const double* y, int full, double* c_out,
                       hipStream_t st);
// as launch_eval with an explicit variable scaling and row scaling (cs may be null)
hipError_t launch_eval_ext(Handle& h, const double* x, int scaled, const Scaling& sc, const double* cs,
                           const double* y, int full, double* c_out, hipStream_t st);
// solve with the stored factors, Schur combine and iterative refinement
// Solve with the stored factorisation and refine on the bordered system until
// ||r - K x||_inf <= target ||r||_inf (at most 10 corrections, keeping the best).
// first_residual_read: the residual of the fused solution has been computed and
// its norms copied to the last four doubles of redbuf_h.
// rel: the largest of the problems' kept relative residuals; rel_p (host [P],
// may be null): each problem's own.
// target: the relative residual at which a problem stops refining (1e-10 for
// the interior-point solves; the simulation's Newton steps take a looser one).
int kkt_solve_refined(Handle& h, const double* rhs, double* sol, bool fused_first, double* rel, hipStream_t st,
                      bool first_residual_read = false, double* rel_p = nullptr, double target = 1e-10);
// res[P]; active0 (host [P], may be null): only these problems iterate and
// are written to xout/yout/res
int ipm_solve(Handle& h, const absorber_ipm_options& o, const double* x0, const double* y0, double* xout,
              double* yout, absorber_ipm_result* res, const unsigned char* active0 = nullptr);
int solve_with_restart(Handle& h, const absorber_ipm_options& o, const double* x0, const double* y0, double* xout,
                       double* yout, absorber_ipm_result* res);
// stream of the graph-replayed iterations (created on first use; null if that fails)
hipStream_t ipm_graph_stream(Handle& h);
void free_ipm_graph(Handle& h);
// process simulation (damped Newton on every scenario's MESH block) of the
// problems in pmask (host [P], null: all) from x (unscaled, in/out)
int simulate(Handle& h, double* x_dev, const unsigned char* pmask, double tol, int max_iter, int* conv, int* iters);
// d_p = (1 + margin) * the largest hydraulic diameter of problem p's stages in x
int set_hydraulic_diameters(Handle& h, double* x_dev, double margin, hipStream_t st);
hipError_t launch_rowmax(Handle& h, const double* x, int scaled, double* rowmax, hipStream_t st);
hipError_t launch_jac_coo(Handle& h, const double* x, double* vals, hipStream_t st);
hipError_t launch_hess_coo(Handle& h, const double* x, const double* lam, double* vals, hipStream_t st);
// factorise every scenario block from the records with the per-problem
// regularisation h.dwv/h.dcv (chains of problems whose h.fmask entry is 0 are
// skipped when mask is true); solve for rhs (may be null) and b.  nchain >= 0
// limits the launch to the first nchain chains (launch-shape timing only).
hipError_t launch_factor(Handle& h, const double* diagx, const double* diags, const double* rhs, bool mask,
                         hipStream_t st, int nchain = -1);
// forward/backward with the stored factors: out (default h.solr) <- K_w^{-1} rhs (nchain as above)
// nrhs right-hand sides (1 to MAX_NPAR - 1) rhs + j * stride into out + j * stride
// (out required for nrhs > 1; the border dot of part only for nrhs = 1).
// zero_masked = false leaves the solution rows of problems outside h.pact
// unwritten (for callers that read only the masked-in problems' rows).
hipError_t launch_solve(Handle& h, const double* rhs, hipStream_t st, int nchain = -1, double* out = nullptr,
                        int nrhs = 1, long long stride = 0, bool zero_masked = true);
// Schur complement on each problem's d.  diagx: Sigma_x (its d entries are
// Sigma_d); rhs: the right-hand side (its d entries are r_d; may be null in
// mode 0).  mode 0: after launch_factor without a right-hand side (S_d,
// inertia); 1: after launch_factor with one; 2: after launch_solve.  For modes
// 1 and 2, sol (if not null) receives the combined solution of the bordered system.
// pmask (device [P], may be null): only the problems whose entry is not 0 are updated.
hipError_t launch_schur(Handle& h, const double* diagx, const double* rhs, int mode, double* sol, hipStream_t st,
                        const int* pmask = nullptr);
// residual res = rhs - K sol of the bordered systems; omega_out[0] = max
// componentwise backward error over the scenario rows, omega_out[1] over the d rows.
// zero_masked = false leaves the residual rows of problems outside h.pact
// unwritten (their partials are still zero).
hipError_t launch_residual(Handle& h, const double* diagx, const double* diags, const double* sol,
                           const double* rhs, double* res, double* omega_out, hipStream_t st,
                           bool zero_masked = true);
// per problem p: pres[2p] = max |res_i|, pres[2p + 1] = max |rhs_i| over its
// rows (stage rows and its d row) from the partials of the last launch_residual
hipError_t launch_residual_pmax(Handle& h, hipStream_t st);
// dst_i = src_i on the KKT rows of the problems whose mask entry is not 0
hipError_t launch_copy_rows(Handle& h, const int* mask, double* dst, const double* src, hipStream_t st);
// x <- the cold-start point (h.x0 in every stage, its diameter for every problem)
hipError_t launch_tile_x0(Handle& h, double* x, hipStream_t st);
// z = y + a x (z may be y)
hipError_t launch_axpy(double* z, const double* y, const double* x, double a, long long n, hipStream_t st);
// the same on the rows (stage and design rows) of the problems in mask only
hipError_t launch_axpy_rows(Handle& h, const int* mask, double* z, const double* y, const double* x, double a,
                            hipStream_t st);
// time the launch-shape candidates on the current data and keep the fastest (h.tune); x, y, c as for
// launch_eval (scaled, full), diagx/diags/rhs as for launch_factor
int autotune(Handle& h, const double* x, const double* y, double* c, const double* diagx, const double* diags,
             const double* rhs, hipStream_t st);

}  // namespace absorber

struct absorber_handle {
  absorber::Handle h;
};
