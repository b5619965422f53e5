/*
 * absorber.h -- C ABI of the MI355X (gfx950) interior-point solver for the
 * scenario-based equilibrium CO2-absorber diameter-minimisation NLP.
 *
 * The problem is eq. (10) of the paper: minimise the shared column diameter d
 * subject to, for every scenario w and stage n, the MESH equations (material
 * balance (1), reaction equilibrium (3a), summations (4), energy balance (6),
 * Raoult/Henry VLE (9a)/(9b)) and the hydraulic inequality (10b), with bounds
 * (10c)-(10d).  Scenarios share only d (problem construction, replicated
 * scenario structure), so the primal-dual KKT matrix is block-bordered: one
 * block per scenario plus the d row/column.
 *
 * Conventions for every call:
 *  - S scenarios, N stages (numbered bottom to top), 21 free variables and 22
 *    rows per stage (see "Layouts").
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch tensors);
 *    pointers named *_host are host pointers.  The library never frees caller
 *    memory; the handle owns all of its internal buffers.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    taking a stream are asynchronous on it unless marked "blocking".
 *  - Every call returns ABS_OK (0) or a negative ABS_ERR_* code; the message of
 *    the last error of the calling thread is absorber_last_error().
 *
 * Layouts (all double precision):
 *  - primal x: length nx = S*N*21 + 1, x[(w*N + n)*21 + k], d = x[nx-1].
 *    Local k: 0-8 liquid x of MEA, MEAH+, H+, MEACOO-, HCO3-, OH-, CO3--, CO2,
 *    H2O; 9-12 vapour y of CO2, H2O, N2, O2; 13 L; 14 V; 15 T; 16-20 reaction
 *    extents of R1-R5.  The 9 variables fixed to zero per stage (vapour
 *    fractions of the 7 non-volatiles, liquid N2 and O2) are not stored.
 *  - rows c / multipliers lambda: length nc = S*N*22, c[(w*N + n)*22 + r].
 *    r: 0-10 material balances of the 11 species, 11-15 reactions R1-R5,
 *    16/17 liquid/vapour summation, 18 water VLE, 19 CO2 VLE, 20 energy
 *    balance, 21 hydraulic row g = V R T / P - u_max pi d^2 / 4 (g <= 0).
 *  - KKT vectors: length nkkt = S*N*43 + 1, v[(w*N + n)*43 + k]; k 0-20 primal,
 *    21-41 multipliers of the 21 MESH rows, 42 multiplier of the hydraulic row;
 *    the d entry last.
 *  - feeds: host array [S][18]: V0, y0 (CO2, H2O, N2, O2), T_gas, L_in,
 *    x_in (9 liquid species), T_liq, P_abs.
 */
#ifndef ABSORBER_H
#define ABSORBER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABS_OK 0
#define ABS_ERR_ARG (-1)       /* bad argument (null pointer, size out of range) */
#define ABS_ERR_HIP (-2)       /* a HIP runtime call failed */
#define ABS_ERR_OOM (-3)       /* device allocation failed */
#define ABS_ERR_STATE (-4)     /* call order violated (e.g. kkt_solve before kkt_factor) */
#define ABS_ERR_INERTIA (-10)  /* inertia correction exceeded delta_w_max */
#define ABS_ERR_LS (-11)       /* line search step below alpha_min (no restoration phase) */
#define ABS_ERR_MAXITER (-12)  /* iteration limit reached */
#define ABS_ERR_NAN (-13)      /* NaN or Inf in an evaluation */
#define ABS_ERR_DIVERGE (-14)  /* |x| above 1e20 */

typedef struct absorber_handle absorber_t;

/* Problem constants (the paper prints the model forms; the values are inputs). */
typedef struct {
  double nu[11][5];                       /* stoichiometry of R1-R5 (species x reaction) */
  double lnK_A[5], lnK_B[5], lnK_C[5], lnK_D[5]; /* ln K_r = A + B/T + C ln T + D T */
  double psat_a, psat_b;                  /* ln Psat[Pa] = a - b / T */
  double henry_lnH298, henry_kappa, henry_Tref, henry_ln_ratio_MEA;
  double Tref;                            /* enthalpy reference temperature [K] */
  double hL_ref[9], cpL_a[9], cpL_b[9];   /* liquid h_i(T) = href + a (T-Tref) + b/2 (T^2-Tref^2) */
  double hV_ref[4], cpV_a[4], cpV_b[4];   /* vapour (CO2, H2O, N2, O2) */
  double R, u_max;
  double x_lo, x_hi, y_lo, y_hi, L_lo, L_hi, V_lo, V_hi, T_lo, T_hi, d_lo, d_hi;
  double x0[21];                          /* cold-start value of every stage */
  double d0;                              /* cold-start diameter */
  double dp_stage;                        /* pressure relations (eq. 7) with a specified drop per stage [Pa]:
                                             the top stage is at the feed table's pressure, each stage below
                                             dp_stage higher; >= 0 (0 in the case study) */
  /* Expected operating cost of the scenario NLP's objective (eq. 8a), a blower
   * cost: op_weight x the power of each equally likely scenario, whose inlet gas
   * (flow, temperature, molar mass from op_molar_mass of CO2, H2O, N2, O2 [kg/mol])
   * enters at the bottom stage's pressure and loses op_loss_coef rho u^2 / 2 in
   * each stage at the superficial velocity u of its (section's) diameter; the
   * objective becomes sum_k c_k theta_k + a_k theta_k^-4.  op_weight = 0 (the
   * case study) leaves the objective d; op_weight > 0 only for single-problem
   * handles (ABS_ERR_ARG for a batch).  Both >= 0. */
  double op_weight, op_loss_coef, op_molar_mass[4];
} absorber_params;

typedef struct {
  int64_t n_var_total;   /* 30*N*S + 1, counting the fixed variables */
  int64_t n_var_free;    /* 21*N*S + 1 */
  int64_t n_eq;          /* 21*N*S MESH equalities */
  int64_t n_fixed;       /* 9*N*S variable-fixing constraints */
  int64_t n_ineq;        /* N*S hydraulic inequalities */
  int64_t nnz_jac;       /* entries of the Jacobian structure */
  int64_t nnz_hess;      /* entries of the lower-triangle Hessian structure */
  int64_t kkt_dim;       /* 43*N*S + 1 (+ p for a column in p sections) */
} absorber_dims;

/* Create a problem instance: N stages, S scenarios, feed table feeds_host[S][18].
 * Allocates the device state on the current device.  Blocking. */
int absorber_create(const absorber_params* params, int32_t n_stages, int32_t n_scen,
                    const double* feeds_host, absorber_t** out);
void absorber_destroy(absorber_t* h);
int absorber_get_dims(const absorber_t* h, absorber_dims* out);

/* Write the cold-start point (the same stage vector for every stage, d0) into
 * x_dev[nx] (unpushed: the interior-point method applies its bound push). */
int absorber_initial_point(absorber_t* h, double* x_dev, void* stream);

/* Scaling used by kkt_factor / kkt_solve: variables x = D * xt with
 * var_scale_host[22] = D of the 21 stage locals then of d; rows c~ = cs * c with
 * row_scale_dev[nc] (NULL: all ones).  Default: no scaling.  Blocking. */
int absorber_set_scaling(absorber_t* h, const double* var_scale_host, const double* row_scale_dev);

/* Residuals of all rows at x (unscaled), c_dev[nc]: the MESH rows of eq.
 * (1), (3a), (4), (9a), (9b), (6) and the hydraulic row (10b). */
int absorber_eval_cons(absorber_t* h, const double* x_dev, double* c_dev, void* stream);

/* Objective f = d (10a): f_host gets d; grad_dev[nx] = e_d.  Blocking. */
int absorber_eval_obj(absorber_t* h, const double* x_dev, double* f_host, double* grad_dev, void* stream);

/* Jacobian structure: row/col indices (host arrays of length nnz_jac).  Per
 * stage: the stage's own block, the hydraulic d entry, then (if the stage is
 * not the top one) the block of the stage above, then (if not the bottom one)
 * the block of the stage below; stages in (w, n) order.  Blocking. */
int absorber_jac_structure(const absorber_t* h, int64_t* rows_host, int64_t* cols_host);
int absorber_eval_jac(absorber_t* h, const double* x_dev, double* vals_dev, void* stream);

/* Lower-triangle structure of the Lagrangian Hessian: 48 entries per stage in
 * (w, n) order (the Hessian is block diagonal by stage), then the (d, d)
 * entry.  Blocking. */
int absorber_hess_structure(const absorber_t* h, int64_t* rows_host, int64_t* cols_host);
/* Values of obj_factor * grad^2 f + sum_j lambda_j grad^2 c_j (grad^2 f = 0). */
int absorber_eval_hess(absorber_t* h, const double* x_dev, const double* lambda_dev, double obj_factor,
                       double* vals_dev, void* stream);

/* Factorise the slack-reduced primal-dual KKT matrix (the Newton system of
 * the interior-point solver of the numerical results, assembled and
 * factorised on the GPU; its scenario blocks are coupled only through d, the
 * structure the conclusion proposes to exploit) in the scaled variables
 *   [[W~ + diag(sigma_x) + dw I,  J~^T                                  ],
 *    [J~,                         -diag(dc (MESH rows), 1/(sigma_s+dw)+dc)]]
 * where J~ = diag(cs) J D and W~ = D (sum_j lambda_j cs_j grad^2 c_j) D at x
 * (original units), lambda_dev[nc] the multipliers of the scaled rows,
 * sigma_x_dev[nx] (scaled variables, entry nx-1 belongs to d) and
 * sigma_s_dev[S*N].  Each scenario block is factorised by a block LDL^T over
 * its stages with Bunch-Kaufman pivoting inside every stage tile, and the d row
 * by the Schur complement S_d.  inertia_host[3] = (n+, n-, n0) of the whole
 * matrix (Haynsworth: sum of the blocks' inertias plus the sign of S_d).  The
 * factors stay in the handle for kkt_solve.  Blocking. */
int absorber_kkt_factor(absorber_t* h, const double* x_dev, const double* lambda_dev,
                        const double* sigma_x_dev, const double* sigma_s_dev, double delta_w,
                        double delta_c, int64_t* inertia_host, void* stream);

/* Solve with the last factorisation: sol_dev[nkkt] = K^{-1} rhs_dev[nkkt]
 * (the block LDL^T solves of every scenario, then the Schur complement step on
 * d: Delta d = (r_d - sum_w b_w^T K_w^{-1} r_w) / S_d and
 * Delta_w = K_w^{-1} (r_w - b_w Delta d)), iteratively refined on the whole
 * bordered system until the relative residual ||rhs - K sol||_inf /
 * ||rhs||_inf is <= 1e-10 or stops decreasing (at most 10 corrections; the
 * best iterate is kept).  rel_resid_host gets that relative residual.  This is
 * the GPU-resident solve of the interior-point Newton system the paper's
 * numerical results time, in the scenario-block form its conclusion names as
 * the structure to exploit.  ABS_ERR_STATE before any absorber_kkt_factor.
 * Blocking. */
int absorber_kkt_solve(absorber_t* h, const double* rhs_dev, double* sol_dev, double* rel_resid_host,
                       void* stream);

/* Interior-point options; absorber_ipm_default_options fills the defaults. */
typedef struct {
  double tol;               /* scaled optimality error E_0 (1e-8) */
  int32_t max_iter;         /* 500 */
  int32_t warm_start;       /* 0: cold start; 1: x0/y0 given, small mu0 and bound push */
  double mu_init;           /* 0.1 */
  double warm_mu_init;      /* 1e-6 */
  double bound_push;        /* 1e-2 (kappa_1 = kappa_2) */
  double warm_bound_push;   /* 1e-8 */
  double nlp_scaling_max_gradient; /* 100 */
  int32_t print_level;      /* 0 silent, 1 one line per iteration to stderr */
  int32_t use_graph;        /* 1: the per-problem decisions of each iteration (convergence test, barrier
                               update, inertia correction, refinement stop, filter line search, step
                               acceptance) are taken on the device, and the iteration's launches replay
                               as captured HIP graphs, one per phase, with one status read per replay
                               pass (the usual iteration is one pass); 0: the host takes the decisions
                               between launches (default 0).  Both take the same decisions. */
  int32_t feasibility_restart; /* 1: a problem that stops without converging (line search, inertia,
                                  iteration limit) is solved again from its simulated states
                                  (absorber_simulate, d at 1.001 x its hydraulic minimum) with the
                                  warm-start options; 0: report the failure (default 1) */
  int32_t autotune;         /* 1: on the handle's first factorisation, time the launch-shape candidates
                               (absorber_tuning) on its own data and keep the fastest (default 1) */
  double delta_w_max;       /* inertia correction: a problem whose delta_w would exceed this value stops
                               with ABS_ERR_INERTIA (default 1e40) */
} absorber_ipm_options;

typedef struct {
  int32_t status;           /* ABS_OK or an ABS_ERR_* code */
  int32_t iterations;
  double E0;                /* final scaled optimality error */
  double inf_pr, inf_du, compl_;
  double d;                 /* optimal diameter */
  double seconds;           /* wall time of the solve */
  int32_t n_inertia_corrections;
  int32_t n_factorizations;
  double max_lin_resid;     /* largest relative linear residual ||r - K x||_inf / ||r||_inf of this
                               problem's own rows over its KKT solves */
  int32_t feasibility_restarts; /* 1 if the result comes from the feasibility restart */
  int32_t graph_replays;    /* graph launches of the solve (use_graph = 1), 0 otherwise */
} absorber_ipm_result;

void absorber_ipm_default_options(absorber_ipm_options* opts);

/* One accepted interior-point iteration of one problem, as recorded by the
 * last absorber_ipm_solve / absorber_batch_solve. */
typedef struct {
  int32_t iteration;        /* 1, 2, ... */
  int32_t n_factorizations; /* factorisations of the inertia-correction loop in this iteration */
  int32_t n_trials;         /* line-search trial points */
  int32_t pad;
  double mu;                /* barrier parameter of the iteration */
  double theta;             /* constraint violation ||c||_1 (scaled rows) at the start of the iteration */
  double alpha;             /* accepted primal step */
  double alpha_z;           /* bound-multiplier step */
  double delta_w;           /* primal regularisation of the accepted factorisation */
  double delta_c;           /* dual regularisation of the accepted factorisation */
  double d;                 /* diameter after the step */
  double E0;                /* scaled optimality error at the start of the iteration */
} absorber_ipm_log_entry;

/* Copy the iteration log of problem `problem` from the last solve on the
 * handle into out[0..max_entries) and the number of entries it holds into
 * *n_out (which may exceed max_entries).  For a problem that went through the
 * feasibility restart the log is that of the restarted run.  Blocking. */
int absorber_ipm_log_get(const absorber_t* h, int32_t problem, int32_t max_entries, absorber_ipm_log_entry* out,
                         int32_t* n_out);

/* A batch of P independent problems in one handle (the batched form): problem
 * p has n_stages[p] stages and n_scen[p] scenarios; feeds_host holds the
 * scenarios of problem 0, then problem 1, ... ([sum n_scen][18]).  Layouts:
 * the primal vector is the stage vectors of all problems' scenarios in that
 * order ([sum N_p S_p][21]) followed by the P diameters d_0..d_{P-1}; the rows
 * [sum N_p S_p][22].  absorber_batch_solve runs the interior-point method on
 * all problems at once, each with its own barrier parameter, filter, step
 * sizes and regularisation (one launch per kernel over all problems), and
 * fills results[P].  Only absorber_batch_solve, absorber_eval_cons,
 * absorber_initial_point, absorber_get_dims and the warm-start calls accept a
 * batch handle; the other calls return ABS_ERR_ARG for P > 1. */
int absorber_create_batch(const absorber_params* params, int32_t n_problems, const int32_t* n_stages,
                          const int32_t* n_scen, const double* feeds_host, absorber_t** out);
/* Blocking.  Returns ABS_OK when every problem converged, otherwise the status
 * of the first problem that did not; x0/lambda0 as for absorber_ipm_solve. */
int absorber_batch_solve(absorber_t* h, const absorber_ipm_options* opts, const double* x0_dev,
                         const double* lambda0_dev, double* x_out_dev, double* lambda_out_dev,
                         absorber_ipm_result* results);

/* A column in p sections, each with its own diameter: the general scenario NLP
 * (eq. 8) with the design vector theta in R^p, p = n_sections in 1..min(4, N).
 * Stage n (0-based, top to bottom) belongs to section floor(n p / N); its
 * hydraulic row (eq. 9c) takes that section's diameter.  The design cost is
 * sum_k c_k theta_k with c_k = (stages in section k) / N, so a column with
 * equal diameters costs d as in problem (10).  Layout: x = [N S stage
 * vectors of 21][theta_0 .. theta_{p-1}] (kkt_dim = 43 N S + p).  Accepted by
 * get_dims, initial_point (every theta_k = d0), eval_cons, eval_obj,
 * simulate (theta_k = the largest hydraulic minimum of section k),
 * ipm_solve, kkt_factor and kkt_solve; the Schur complement on theta is a
 * dense p x p matrix whose inertia comes from its eigenvalues.
 * absorber_ipm_result.d reports the design cost sum_k c_k theta_k.  The
 * warm start takes the predicted states (theta_k = (1 + margin) x the largest
 * predicted hydraulic diameter of section k) and no multipliers (lambda0 must
 * be NULL; absorber_warm_solve uses the least-squares estimate).  The COO
 * Jacobian/Hessian calls return ABS_ERR_ARG.
 * Blocking; allocates the device state on the current device. */
int absorber_create_sections(const absorber_params* params, int32_t n_stages, int32_t n_scen, int32_t n_sections,
                             const double* feeds_host, absorber_t** out);

/* Process simulation: for fixed feeds each scenario's MESH equations are a
 * square system in its stage states (the equilibrium model's degrees of
 * freedom), solved here by Newton's method for every scenario of every
 * problem at once (mole fractions stepped in their logarithm, log-steps capped
 * at 5, backtracking on each scenario's scaled residual; each Newton system is
 * solved to a relative residual of 1e-6, enough for the step).  x_dev [nx]: start
 * point in, states out; the d entries are set to each problem's hydraulic
 * minimum max sqrt(4 V R T / (pi u_max P)).  Stops when every scenario's
 * scaled MESH residual inf-norm is <= tol or after max_iter steps;
 * converged_host [P] (may be NULL) flags the problems whose scenarios all
 * converged.  Blocking; invalidates a factorisation from absorber_kkt_factor. */
int absorber_simulate(absorber_t* h, double* x_dev, double tol, int32_t max_iter, int32_t* converged_host,
                      int32_t* iterations_host);

/* Run the interior-point method to E_0 <= tol.  x0_dev[nx] (original units) and
 * lambda0_dev[nc] may be NULL (cold start).  On return x_out_dev[nx] and
 * lambda_out_dev[nc] (may be NULL) hold the final iterate.  Blocking. */
int absorber_ipm_solve(absorber_t* h, const absorber_ipm_options* opts, const double* x0_dev,
                       const double* lambda0_dev, double* x_out_dev, double* lambda_out_dev,
                       absorber_ipm_result* result);

/* Per-kernel-class timing with HIP events recorded on the stream each kernel is
 * launched on.  Classes: 0 block LDL^T factorisation (with its fused solve),
 * 1 solve with stored factors, 2 stage evaluation, 3 bordered residual.
 * absorber_profile_enable(h, mask) resets the counters and times the classes
 * whose bit is set in mask (bit k = class k); mask 0 stops timing.  The events
 * add no host synchronisation to the timed work: their times are read (waiting
 * for the recorded launches) by absorber_profile_get and absorber_profile_enable,
 * and every 512 timed launches. */
typedef struct {
  double ms[4];        /* summed kernel time per class */
  int64_t calls[4];    /* launches per class */
  int64_t bytes_factor_slots; /* bytes of pivot columns one factorisation writes */
} absorber_profile;
int absorber_profile_enable(absorber_t* h, int32_t mask);

/* Launch shapes chosen by the autotuner (absorber_ipm_options.autotune): for
 * the block LDL^T factorisation the occupancy target (waves per SIMD 2 or 3,
 * which fixes each wave's register budget) and the row split of its trailing
 * update (0: updates from rows 0/16/32 of the frontal tile, 1: from rows 0/24,
 * 2: from rows 0/8/16/24/32/40; rows whose pivots are all eliminated are never
 * updated again); the occupancy target of the stored-factor solve (waves per
 * SIMD 2, 3 or 4); the block size of the stage evaluation (64, 128 or 256).
 * The measured time of each candidate is in ms (factor_ms[waves 2, 3][split];
 * the other arrays in the order listed; the factorisation and the solve are
 * timed on at most the first 12288 scenario chains).  tuned = 0 until the first
 * factorisation of a solve with autotune on. */
typedef struct {
  int32_t tuned;
  int32_t factor_waves_per_simd, factor_row_split, solve_waves_per_simd, eval_block;
  float factor_ms[2][3], solve_ms[3], eval_ms[3];
} absorber_tuning;
int absorber_tuning_get(const absorber_t* h, absorber_tuning* out);
/* Pin the launch shapes (factor_waves_per_simd 2 or 3, factor_row_split 0-2,
 * solve_waves_per_simd 2-4, eval_block 64/128/256; the timing arrays are
 * ignored) and mark them tuned, so the autotuner does not run; ABS_ERR_ARG for
 * a shape outside those sets.  The shapes change the speed, not the results. */
int absorber_tuning_set(absorber_t* h, const absorber_tuning* in);
int absorber_profile_get(const absorber_t* h, absorber_profile* out);

/* ------------------------------------------------------------------------
 * Warm-start network.  Not part of the paper's method: a multilayer
 * perceptron  inputs -> [Linear -> GELU(erf)] x n_layers -> Linear -> outputs
 * that predicts a scenario's converged stage states from its feed, used to
 * start the interior-point solve near the solution.  GEMM operands are
 * bfloat16 (round to nearest even) on the matrix cores with float32
 * accumulation; biases, pre-activations and the optimiser state are float32.
 *
 * Parameters (host or device, float32) use one flat layout: for each linear
 * layer l = 0..n_layers, W_l [out][in] row-major, then b_l [out].
 * Inputs and targets are float32 row-major [n][n_in] / [n][n_out] in their own
 * units; the network standardises them with per-column mean and standard
 * deviation (identity until set or fitted) and returns outputs in the units
 * of the targets.  Training minimises the mean squared error of the
 * standardised outputs with Adam (Kingma & Ba 2015) and a cosine learning
 * rate, over shuffled mini-batches (the last partial batch of an epoch is
 * dropped).
 * ------------------------------------------------------------------------ */
typedef struct absorber_mlp absorber_mlp;

typedef struct {
  int32_t n_in;       /* input features, 1..32 (3: gas flow, CO2 fraction, gas temperature) */
  int32_t n_hidden;   /* width of every hidden layer, a multiple of 32 (256) */
  int32_t n_layers;   /* hidden layers, >= 1 (3) */
  int32_t n_out;      /* outputs (21 N: one stage vector per stage) */
  int32_t max_batch;  /* rows per forward chunk and largest training batch, a multiple of 32 (512) */
} absorber_mlp_config;

typedef struct {
  int32_t epochs;     /* 300 */
  int32_t batch;      /* rows per step, a multiple of 32, <= max_batch (512) */
  double lr;          /* peak learning rate (1e-3) */
  double beta1, beta2, eps;  /* Adam constants (0.9, 0.999, 1e-8) */
  uint64_t seed;      /* shuffling seed */
  int32_t cosine;     /* 1: lr * (1 + cos(pi step / steps)) / 2; 0: constant lr */
} absorber_mlp_train_options;

typedef struct {
  double final_loss;  /* mean squared error of the last batch (standardised units) */
  double seconds;     /* wall time of the training call */
  int64_t steps;      /* optimiser steps taken */
} absorber_mlp_train_result;

void absorber_mlp_default_config(absorber_mlp_config* cfg);
void absorber_mlp_default_train_options(absorber_mlp_train_options* opts);
/* He-normal weights from seed, zero biases.  Blocking.  ABS_ERR_ARG on a bad
 * configuration, ABS_ERR_OOM when device memory runs out. */
int absorber_mlp_create(const absorber_mlp_config* cfg, uint64_t seed, absorber_mlp** out);
void absorber_mlp_destroy(absorber_mlp* net);
int absorber_mlp_get_config(const absorber_mlp* net, absorber_mlp_config* out);
int64_t absorber_mlp_num_params(const absorber_mlp* net);
/* Copy the flat float32 parameters in (resets the Adam state) or out.  Blocking. */
int absorber_mlp_set_params(absorber_mlp* net, const float* params_host);
int absorber_mlp_get_params(const absorber_mlp* net, float* params_host);
/* Standardisation constants, host arrays of n_in / n_out floats.  Blocking. */
int absorber_mlp_set_normalization(absorber_mlp* net, const float* in_mean, const float* in_std,
                                   const float* out_mean, const float* out_std);
int absorber_mlp_get_normalization(const absorber_mlp* net, float* in_mean, float* in_std, float* out_mean,
                                   float* out_std);
/* Set the standardisation from data: column means and standard deviations of
 * X_dev [n][n_in] and T_dev [n][n_out] (sd floored at 1e-6 (1 + |mean|)). */
int absorber_mlp_fit_normalization(absorber_mlp* net, const float* X_dev, const float* T_dev, int64_t n,
                                   void* stream);
/* Y_dev [n][n_out] = network(X_dev [n][n_in]), any n >= 0 (processed in
 * chunks of max_batch rows).  The caller must not run two calls on one
 * network concurrently (they share its activation buffers). */
int absorber_mlp_forward(absorber_mlp* net, const float* X_dev, int64_t n, float* Y_dev, void* stream);
/* One mini-batch of n rows (n a multiple of 32, <= max_batch): the gradient of
 * the mean squared error of the standardised outputs with respect to the flat
 * parameters into grad_dev [num_params]; the loss into *loss_host (may be
 * NULL).  Blocking (it reads the loss). */
int absorber_mlp_loss_grad(absorber_mlp* net, const float* X_dev, const float* T_dev, int64_t n, float* grad_dev,
                           double* loss_host, void* stream);
/* One Adam step with gradient grad_dev [num_params] and learning rate lr
 * (beta1, beta2, eps from opts); also refreshes the bfloat16 weights. */
int absorber_mlp_adam_step(absorber_mlp* net, const float* grad_dev, const absorber_mlp_train_options* opts,
                           double lr, void* stream);
/* Fit the standardisation to the data, then train for opts->epochs epochs on
 * X_dev [n][n_in], T_dev [n][n_out] (n >= opts->batch).  Blocking, null stream. */
int absorber_mlp_train(absorber_mlp* net, const float* X_dev, const float* T_dev, int64_t n,
                       const absorber_mlp_train_options* opts, absorber_mlp_train_result* result);

/* Warm-start encoding of the absorber problem (every problem of the handle
 * must have the same stage count N).  A network row describes one scenario:
 * its N stage vectors (21 values each: ln of the 13 mole fractions, floored at
 * 1e-30, then L, V, T and the 5 extents), and for a primal-dual network its N
 * row-multiplier vectors (22 values each, asinh(lambda / 1e-6)); n_out = 21 N
 * (primal) or 43 N (primal-dual).
 * features: X_dev [S][3] float = (flue-gas flow, CO2 fraction, temperature) of
 *   each scenario's feed.
 * targets: T_dev [S][n_out] from a primal vector x_dev[nx] and, for n_out = 43 N,
 *   the row multipliers lambda_dev[nc] (NULL: primal only).
 * point: decodes Y_dev [S][n_out] into x0_dev[nx]: the stage vectors, and each
 *   problem's d = (1 + d_margin) * the largest hydraulic diameter
 *   sqrt(4 V R T / (pi u_max P)) of its decoded stages (d_margin >= 0); with a
 *   primal-dual row and lambda0_dev[nc] non-NULL, the multipliers of each
 *   problem's worst scenario (the one holding that largest diameter, the only
 *   one whose hydraulic rows are active at the optimum) and 0 for the others.
 * warm_start: features -> network -> point, with caller workspaces
 *   X_work_dev [S][3] and Y_work_dev [S][n_out]; the network must have 3 inputs.
 * All four are asynchronous on stream. */
int absorber_warm_features(absorber_t* h, float* X_dev, void* stream);
int absorber_warm_targets(absorber_t* h, const double* x_dev, const double* lambda_dev, float* T_dev,
                          void* stream);
int absorber_warm_point(absorber_t* h, const float* Y_dev, int32_t n_out, double d_margin, double* x0_dev,
                        double* lambda0_dev, void* stream);
int absorber_warm_start(absorber_t* h, absorber_mlp* net, float* X_work_dev, float* Y_work_dev, double d_margin,
                        double* x0_dev, double* lambda0_dev, void* stream);
/* absorber_warm_start for callers that cannot allocate device memory (code
 * being captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc): the same result, with the network inputs, its outputs and the
 * per-problem worst-scenario index in a static device workspace of the
 * library (32 MiB on each GPU it runs on, held until the process ends)
 * instead of caller workspaces; it calls no allocating routine.  Requires
 * 256-aligned S*3*4 + S*n_out*4 + P*4 bytes <= 32 MiB (5000 scenarios of a
 * 430-output network take 8.7 MB); larger sizes return ABS_ERR_ARG with the
 * byte counts.  Every call on one GPU shares that workspace: calls that
 * overlap on one GPU (other threads, other streams) race.  Asynchronous on
 * stream. */
int absorber_warm_start_noalloc(absorber_t* h, absorber_mlp* net, double d_margin, double* x0_dev,
                                double* lambda0_dev, void* stream);
/* Warm-started solve with cold-start fallback: warm_start (workspaces owned by
 * the handle, allocated on the first call), then absorber_ipm_solve with
 * opts->warm_start = 1 and the predicted multipliers (primal-dual network) or
 * the least-squares multiplier estimate (primal network); if that does
 * not reach opts->tol, a cold-started solve from the paper's initial point.
 * *used_warm (may be NULL) is 1 when the warm solve succeeded.  result->seconds
 * covers the whole call and result->iterations both solves.  Blocking. */
int absorber_warm_solve(absorber_t* h, absorber_mlp* net, const absorber_ipm_options* opts, double d_margin,
                        double* x_out_dev, double* lambda_out_dev, absorber_ipm_result* result, int32_t* used_warm);

const char* absorber_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ABSORBER_H */
