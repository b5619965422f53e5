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

// the 16 stage-local KKT indices that receive the contribution of the stage below
__host__ __device__ constexpr int coupling_index(int a) {
  return a < 9 ? a : (a == 9 ? IL : (a == 10 ? IT : (a < 15 ? NV + 7 + (a - 11) : NV + 20)));
}

struct JacEntry { int8_t row, blk, col; };

// scalars produced by the Schur/inertia reduction
struct DevScalars {
  double sd, kdd, sig_b, sig_r, dd, rd, wdd, pad0;
  long long npos, nneg, nzero, pad1;
};

// scaling applied to the NLP: x = D * xt per stage-local index, rows times cs
struct Scaling {
  double D[NV];
  double Dd;
};

// all per-handle device and host state
struct Handle {
  int N = 0, S = 0;
  long long nx = 0, nc = 0, nkkt = 0;       // primal incl. d, rows, KKT unknowns incl. d
  ModelParams mp{};
  double xL[NV], xU[NV], dL = 0, dU = 0;     // unscaled bounds per local variable
  std::vector<double> feeds_h;
  double* feeds = nullptr;                   // device [S][NF]
  std::vector<JacEntry> jac_own, jac_up, jac_down;  // per-stage Jacobian structure
  int jac_d_index = -1;                      // position of the d entry within OWN
  HessPos hpos[NH];
  int* gather = nullptr;                     // device [FR][64] packed gather table
  int* jtab = nullptr;                       // device packed Jacobian structure (row, col) per entry
  Scaling sc{};
  double* cs = nullptr;                      // device [S][N][NR] row scaling
  double sf = 1.0;
  // work buffers
  double* rec = nullptr;                     // [S][N][REC]
  double* slots = nullptr;                   // [S][N][NK][SLOT] stored pivot columns
  double* solr = nullptr;                    // [S][N][NK] K_w^{-1} r
  double* solb = nullptr;                    // [S][N][NK] K_w^{-1} b
  int* inert = nullptr;                      // [S][4]
  double* part = nullptr;                    // [S][4] per-scenario partial sums
  DevScalars* scal = nullptr;                // device scalars
  DevScalars* scal_h = nullptr;              // pinned host mirror
  double* diagx = nullptr;                   // [nx] Sigma_x for the KKT (scaled)
  double* diags = nullptr;                   // [S][N] Sigma_s
  double* kres = nullptr;                    // [nkkt] refinement residual
  double* kcor = nullptr;                    // [nkkt] refinement correction
  double* kden = nullptr;                    // [S][N] per-stage backward-error partials
  double* redbuf = nullptr;                  // device reduction partials
  double* redbuf_h = nullptr;                // pinned host mirror
  int red_cap = 0;
  hipStream_t stream = nullptr;
  double fdw = 0, fdc = 0;                   // regularisation of the stored factorisation
  bool factored = false;
  double last_diag_d = 0;
  double x0[NV + 1];                         // cold-start stage vector and diameter
  float* warm_X = nullptr;                   // warm-start workspaces (allocated on first use)
  float* warm_Y = nullptr;
  double* warm_x0 = nullptr;
  long long n_factor = 0, n_solve = 0;       // launch counters
  // optional per-class kernel timing (HIP events on the launch stream)
  int prof = 0;  // bit mask of the profiled kernel classes
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double prof_ms[4] = {0, 0, 0, 0};
  long long prof_calls[4] = {0, 0, 0, 0};
};

void set_error(const std::string& msg);
// bracket a launch with profiling events (no-ops unless profiling is enabled)
void prof_begin(Handle& h, hipStream_t st);
void prof_end(Handle& h, int cls, hipStream_t st);
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
int kkt_solve_refined(Handle& h, const double* rhs, double* sol, bool fused_first, double* rel, hipStream_t st);
int ipm_solve(Handle& h, const absorber_ipm_options& o, const double* x0, const double* y0, double* xout,
              double* yout, absorber_ipm_result* res);
hipError_t launch_rowmax(Handle& h, const double* x, int scaled, double* rowmax, hipStream_t st);
hipError_t launch_jac_coo(Handle& h, const double* x, double* vals, hipStream_t st);
hipError_t launch_hess_coo(Handle& h, const double* x, const double* lam, double* vals, hipStream_t st);
// factorise every scenario block from the records; solve for rhs (may be null) and b
hipError_t launch_factor(Handle& h, const double* diagx, const double* diags, double dw, double dc,
                         const double* rhs, hipStream_t st);
// forward/backward with the stored factors: solr <- K_w^{-1} rhs
hipError_t launch_solve(Handle& h, const double* rhs, hipStream_t st);
// Schur complement on d.  diagd: device pointer to Sigma_d; rd: device pointer to
// the d entry of the right-hand side.  mode 0: after launch_factor without a
// right-hand side (S_d, inertia); 1: after launch_factor with one; 2: after
// launch_solve.  For modes 1 and 2, sol (if not null) receives the combined
// solution of the bordered system.
hipError_t launch_schur(Handle& h, const double* diagd, double dw, const double* rd, int mode, double* sol,
                        hipStream_t st);
// residual res = rhs - K sol of the bordered system; omega_out[0] = max
// componentwise backward error over the scenario rows, omega_out[1] that of the d row
hipError_t launch_residual(Handle& h, const double* diagx, const double* diags, double dw, double dc,
                           const double* sol, const double* rhs, double* res, double* omega_out, hipStream_t st);
hipError_t launch_axpy(double* y, const double* x, double a, long long n, hipStream_t st);

}  // namespace absorber

struct absorber_handle {
  absorber::Handle h;
};
