// Equilibrium absorber stage model: residuals, exact first derivatives and the
// Lagrangian Hessian block of one stage, hand-derived.
//
// Equations (paper): material balance (1) with zero side feeds; reaction
// equilibrium in activities (3a) with ideal-liquid activities and the
// Kent-Eisenberg ln K_r(T); summations (4); Raoult's law for water (9a) and
// Henry's law for CO2 (9b); stage energy balance (6) with Q = 0 and
// ideal-mixture enthalpies; hydraulic constraint (10b).
//
// Stage-local variable order (21): x of MEA, MEAH+, H+, MEACOO-, HCO3-, OH-,
// CO3--, CO2, H2O (0-8); y of CO2, H2O, N2, O2 (9-12); L 13; V 14; T 15;
// reaction extents 16-20.  Row order (22): material balances of the 11
// species (0-10), reactions R1-R5 (11-15), liquid and vapour summation (16,
// 17), water VLE (18), CO2 VLE (19), energy balance (20), hydraulic (21).
//
// Every derivative of stage n's rows with respect to stage n's variables
// depends on stage n alone (the coupling terms are the products L x, V y,
// L h, V h of one neighbouring stage), and the Lagrangian Hessian is block
// diagonal by stage.  The Jacobian is therefore emitted in three blocks per
// stage: OWN (d c_n / d z_n), UP (d c_n / d z_{n+1}), DOWN (d c_n / d z_{n-1}),
// plus the single d-column entry of the hydraulic row.
#pragma once
#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define ABS_HD __host__ __device__ __forceinline__
#else
#define ABS_HD inline
#endif

namespace absorber {

constexpr int NV = 21;     // free variables per stage
constexpr int NR = 22;     // rows per stage (21 MESH + hydraulic)
constexpr int NE = 21;     // MESH equalities per stage
constexpr int NK = 43;     // KKT unknowns per stage: 21 primal, 21 MESH duals, 1 hydraulic dual
constexpr int NF = 18;     // feed-table doubles per scenario
constexpr int NH = 48;     // unique lower-triangle Hessian entries per stage
constexpr int IX = 0, IY = 9, IL = 13, IV = 14, IT = 15, IE = 16;

constexpr int BLK_OWN = 0, BLK_UP = 1, BLK_DOWN = 2, BLK_D = 3;

// physical constants of the model (copied from the problem data)
struct ModelParams {
  double nu[11][5];
  double A[5], B[5], C[5], D[5];
  double psat_a, psat_b;
  double lnH298, kH, TH, lnr;
  double Tref;
  double hL_ref[9], cpL_a[9], cpL_b[9];
  double hV_ref[4], cpV_a[4], cpV_b[4];
  double R, u_max;
  double dp;  // specified pressure drop per stage (pressure relations, eq. 7)
};

// pressure of stage n (0 = bottom) of an N-stage column whose top stage is at
// P_top: eq. (7) with a specified drop, P_n = P_{n+1} + dp
ABS_HD double stage_pressure(const ModelParams& p, double P_top, int n, int N) {
  return P_top + (double)(N - 1 - n) * p.dp;
}

// inflow of a stage: liquid from above (L, x, T) and vapour from below (V, y, T)
struct Inflow {
  double L_up, x_up[9], T_up;
  double V_dn, y_dn[4], T_dn;
};

ABS_HD double hL(const ModelParams& p, int i, double T) {
  return p.hL_ref[i] + p.cpL_a[i] * (T - p.Tref) + 0.5 * p.cpL_b[i] * (T * T - p.Tref * p.Tref);
}
ABS_HD double cpL(const ModelParams& p, int i, double T) { return p.cpL_a[i] + p.cpL_b[i] * T; }
ABS_HD double hV(const ModelParams& p, int j, double T) {
  return p.hV_ref[j] + p.cpV_a[j] * (T - p.Tref) + 0.5 * p.cpV_b[j] * (T * T - p.Tref * p.Tref);
}
ABS_HD double cpV(const ModelParams& p, int j, double T) { return p.cpV_a[j] + p.cpV_b[j] * T; }

// inflow of stage n from the neighbouring stage vectors or the feed row
ABS_HD void make_inflow(const double* zdn, const double* zup, const double* feed, Inflow& f) {
  if (zup) {
    f.L_up = zup[IL];
    for (int i = 0; i < 9; ++i) f.x_up[i] = zup[IX + i];
    f.T_up = zup[IT];
  } else {
    f.L_up = feed[6];
    for (int i = 0; i < 9; ++i) f.x_up[i] = feed[7 + i];
    f.T_up = feed[16];
  }
  if (zdn) {
    f.V_dn = zdn[IV];
    for (int j = 0; j < 4; ++j) f.y_dn[j] = zdn[IY + j];
    f.T_dn = zdn[IT];
  } else {
    f.V_dn = feed[0];
    for (int j = 0; j < 4; ++j) f.y_dn[j] = feed[1 + j];
    f.T_dn = feed[5];
  }
}

// Henry constant pieces of (9b): H(T, xapp) and its derivatives
struct Henry {
  double H, HT, HTT;        // d/dT
  double Ha, HW;            // d/dA (amine sum), d/dW (water)
  double Haa, HaW, HWW;     // second derivatives in (A, W)
  double HaT, HWT;
};

ABS_HD Henry henry(const ModelParams& p, const double* z) {
  Henry h;
  const double T = z[IT];
  const double A = z[0] + z[1] + z[3];
  const double W = z[8];
  const double s = A + W;
  const double xa = A / s;
  const double xa_A = W / (s * s), xa_W = -A / (s * s);
  const double s3 = s * s * s;
  const double xa_AA = -2.0 * W / s3, xa_AW = (A - W) / s3, xa_WW = 2.0 * A / s3;
  const double rho = p.lnr;
  h.H = exp(p.lnH298 + p.kH * (1.0 / p.TH - 1.0 / T) + xa * rho);
  const double g = p.kH / (T * T);            // d lnH / dT
  const double gT = -2.0 * p.kH / (T * T * T);
  h.HT = h.H * g;
  h.HTT = h.H * (g * g + gT);
  h.Ha = h.H * rho * xa_A;
  h.HW = h.H * rho * xa_W;
  h.Haa = h.H * (rho * rho * xa_A * xa_A + rho * xa_AA);
  h.HaW = h.H * (rho * rho * xa_A * xa_W + rho * xa_AW);
  h.HWW = h.H * (rho * rho * xa_W * xa_W + rho * xa_WW);
  h.HaT = h.Ha * g;
  h.HWT = h.HW * g;
  return h;
}

// ---------------------------------------------------------------- residuals
// c[0..21] of one stage (unscaled); d is the diameter, P the absorber pressure
ABS_HD void stage_residuals(const ModelParams& p, const double* z, const Inflow& f, double P, double d,
                            double* c) {
  const double* x = z + IX;
  const double* y = z + IY;
  const double L = z[IL], V = z[IV], T = z[IT];
  const double* e = z + IE;
  for (int i = 0; i < 11; ++i) {
    double r = 0.0;
    if (i < 9) r += L * x[i] - f.L_up * f.x_up[i];
    if (i >= 7) r += V * y[i - 7] - f.V_dn * f.y_dn[i - 7];
    for (int k = 0; k < 5; ++k) r -= p.nu[i][k] * e[k];
    c[i] = r;
  }
  double lx[9];
  for (int i = 0; i < 9; ++i) lx[i] = log(x[i]);
  const double lT = log(T);
  for (int k = 0; k < 5; ++k) {
    double r = 0.0;
    for (int i = 0; i < 9; ++i) r += p.nu[i][k] * lx[i];
    c[11 + k] = r - (p.A[k] + p.B[k] / T + p.C[k] * lT + p.D[k] * T);
  }
  double sl = 0.0, sv = 0.0;
  for (int i = 0; i < 9; ++i) sl += x[i];
  for (int j = 0; j < 4; ++j) sv += y[j];
  c[16] = sl - 1.0;
  c[17] = sv - 1.0;
  const double psat = exp(p.psat_a - p.psat_b / T);
  c[18] = P * y[1] - x[8] * psat;
  const Henry h = henry(p, z);
  c[19] = P * y[0] - x[7] * h.H;
  double hl = 0.0, hv = 0.0, hlu = 0.0, hvd = 0.0;
  for (int i = 0; i < 9; ++i) {
    hl += x[i] * hL(p, i, T);
    hlu += f.x_up[i] * hL(p, i, f.T_up);
  }
  for (int j = 0; j < 4; ++j) {
    hv += y[j] * hV(p, j, T);
    hvd += f.y_dn[j] * hV(p, j, f.T_dn);
  }
  c[20] = L * hl + V * hv - f.L_up * hlu - f.V_dn * hvd;
  c[21] = V * p.R * T / P - p.u_max * M_PI * d * d * 0.25;
}

// ---------------------------------------------------------------- Jacobian
// Emits every structural nonzero of stage n's rows through sink(row, block,
// col, value) in a fixed order that depends only on (nu, has_up, has_down).
template <class Sink>
ABS_HD void stage_jacobian(const ModelParams& p, const double* z, const Inflow& f, double P, double d,
                           bool has_up, bool has_down, Sink& J) {
  const double* x = z + IX;
  const double* y = z + IY;
  const double L = z[IL], V = z[IV], T = z[IT];
  // ---- OWN block
  for (int i = 0; i < 11; ++i) {
    if (i < 9) {
      J(i, BLK_OWN, IX + i, L);
      J(i, BLK_OWN, IL, x[i]);
    }
    if (i >= 7) {
      J(i, BLK_OWN, IY + i - 7, V);
      J(i, BLK_OWN, IV, y[i - 7]);
    }
    for (int k = 0; k < 5; ++k)
      if (p.nu[i][k] != 0.0) J(i, BLK_OWN, IE + k, -p.nu[i][k]);
  }
  for (int k = 0; k < 5; ++k) {
    for (int i = 0; i < 9; ++i)
      if (p.nu[i][k] != 0.0) J(11 + k, BLK_OWN, IX + i, p.nu[i][k] / x[i]);
    const double dlnK = -p.B[k] / (T * T) + p.C[k] / T + p.D[k];
    J(11 + k, BLK_OWN, IT, -dlnK);
  }
  for (int i = 0; i < 9; ++i) J(16, BLK_OWN, IX + i, 1.0);
  for (int j = 0; j < 4; ++j) J(17, BLK_OWN, IY + j, 1.0);
  const double psat = exp(p.psat_a - p.psat_b / T);
  const double psat_T = psat * p.psat_b / (T * T);
  J(18, BLK_OWN, IY + 1, P);
  J(18, BLK_OWN, IX + 8, -psat);
  J(18, BLK_OWN, IT, -x[8] * psat_T);
  const Henry h = henry(p, z);
  J(19, BLK_OWN, IY + 0, P);
  J(19, BLK_OWN, IX + 7, -h.H);
  J(19, BLK_OWN, IT, -x[7] * h.HT);
  J(19, BLK_OWN, IX + 0, -x[7] * h.Ha);
  J(19, BLK_OWN, IX + 1, -x[7] * h.Ha);
  J(19, BLK_OWN, IX + 3, -x[7] * h.Ha);
  J(19, BLK_OWN, IX + 8, -x[7] * h.HW);
  double hl = 0.0, hv = 0.0, cpl = 0.0, cpv = 0.0;
  for (int i = 0; i < 9; ++i) {
    const double hi = hL(p, i, T);
    J(20, BLK_OWN, IX + i, L * hi);
    hl += x[i] * hi;
    cpl += x[i] * cpL(p, i, T);
  }
  J(20, BLK_OWN, IL, hl);
  for (int j = 0; j < 4; ++j) {
    const double hj = hV(p, j, T);
    J(20, BLK_OWN, IY + j, V * hj);
    hv += y[j] * hj;
    cpv += y[j] * cpV(p, j, T);
  }
  J(20, BLK_OWN, IV, hv);
  J(20, BLK_OWN, IT, L * cpl + V * cpv);
  J(21, BLK_OWN, IV, p.R * T / P);
  J(21, BLK_OWN, IT, V * p.R / P);
  J(21, BLK_D, 0, -p.u_max * M_PI * d * 0.5);
  // ---- UP block: d c_n / d z_{n+1} (liquid entering from above)
  if (has_up) {
    for (int i = 0; i < 9; ++i) {
      J(i, BLK_UP, IX + i, -f.L_up);
      J(i, BLK_UP, IL, -f.x_up[i]);
    }
    double hlu = 0.0, cplu = 0.0;
    for (int i = 0; i < 9; ++i) {
      const double hi = hL(p, i, f.T_up);
      J(20, BLK_UP, IX + i, -f.L_up * hi);
      hlu += f.x_up[i] * hi;
      cplu += f.x_up[i] * cpL(p, i, f.T_up);
    }
    J(20, BLK_UP, IL, -hlu);
    J(20, BLK_UP, IT, -f.L_up * cplu);
  }
  // ---- DOWN block: d c_n / d z_{n-1} (vapour entering from below)
  if (has_down) {
    for (int i = 7; i < 11; ++i) {
      J(i, BLK_DOWN, IY + i - 7, -f.V_dn);
      J(i, BLK_DOWN, IV, -f.y_dn[i - 7]);
    }
    double hvd = 0.0, cpvd = 0.0;
    for (int j = 0; j < 4; ++j) {
      const double hj = hV(p, j, f.T_dn);
      J(20, BLK_DOWN, IY + j, -f.V_dn * hj);
      hvd += f.y_dn[j] * hj;
      cpvd += f.y_dn[j] * cpV(p, j, f.T_dn);
    }
    J(20, BLK_DOWN, IV, -hvd);
    J(20, BLK_DOWN, IT, -f.V_dn * cpvd);
  }
}

// ---------------------------------------------------------------- Hessian
// Positions (row >= col, stage-local) of the 48 unique Hessian entries.
struct HessPos { int8_t r, c; };

// Fills the position table; the order below is the order of stage_hessian's output.
ABS_HD void hess_positions(HessPos* pos) {
  int n = 0;
  for (int i = 0; i < 9; ++i) pos[n++] = {(int8_t)IL, (int8_t)(IX + i)};        // 0-8   (L, x_i)
  for (int j = 0; j < 4; ++j) pos[n++] = {(int8_t)IV, (int8_t)(IY + j)};        // 9-12  (V, y_j)
  for (int i = 0; i < 9; ++i) pos[n++] = {(int8_t)(IX + i), (int8_t)(IX + i)};  // 13-21 (x_i, x_i)
  const int8_t am[3] = {0, 1, 3};
  pos[n++] = {1, 0};  // 22
  pos[n++] = {3, 0};  // 23
  pos[n++] = {3, 1};  // 24
  for (int a = 0; a < 3; ++a) pos[n++] = {7, am[a]};  // 25-27 (x_CO2, amine)
  for (int a = 0; a < 3; ++a) pos[n++] = {8, am[a]};  // 28-30 (x_H2O, amine)
  pos[n++] = {8, 7};                                  // 31
  for (int i = 0; i < 9; ++i) pos[n++] = {(int8_t)IT, (int8_t)(IX + i)};        // 32-40 (T, x_i)
  for (int j = 0; j < 4; ++j) pos[n++] = {(int8_t)IT, (int8_t)(IY + j)};        // 41-44 (T, y_j)
  pos[n++] = {(int8_t)IT, (int8_t)IL};                                          // 45
  pos[n++] = {(int8_t)IT, (int8_t)IV};                                          // 46
  pos[n++] = {(int8_t)IT, (int8_t)IT};                                          // 47
}

// Lagrangian Hessian block of stage n with respect to z_n.
// lam_dn, lam, lam_up: row weights (22 each) of stages n-1, n, n+1 (nullptr when
// the stage does not exist).  H[48] in the hess_positions order.
ABS_HD void stage_hessian(const ModelParams& p, const double* z, double P, const double* lam_dn,
                          const double* lam, const double* lam_up, double* H) {
  const double* x = z + IX;
  const double* y = z + IY;
  const double L = z[IL], V = z[IV], T = z[IT];
  // weights of the liquid (L x, L hL) and vapour (V y, V hV) terms: own row
  // minus the row of the stage the stream flows into
  double wMBl[9], wMBv[4];
  for (int i = 0; i < 9; ++i) wMBl[i] = lam[i] - (lam_dn ? lam_dn[i] : 0.0);
  for (int j = 0; j < 4; ++j) wMBv[j] = lam[7 + j] - (lam_up ? lam_up[7 + j] : 0.0);
  const double wEBl = lam[20] - (lam_dn ? lam_dn[20] : 0.0);
  const double wEBv = lam[20] - (lam_up ? lam_up[20] : 0.0);
  double cpl_mix = 0.0, cpv_mix = 0.0, dcpl_mix = 0.0, dcpv_mix = 0.0;
  for (int i = 0; i < 9; ++i) {
    H[i] = wMBl[i] + wEBl * hL(p, i, T);
    cpl_mix += x[i] * cpL(p, i, T);
    dcpl_mix += x[i] * p.cpL_b[i];
  }
  for (int j = 0; j < 4; ++j) {
    H[9 + j] = wMBv[j] + wEBv * hV(p, j, T);
    cpv_mix += y[j] * cpV(p, j, T);
    dcpv_mix += y[j] * p.cpV_b[j];
  }
  // reaction equilibria: -nu/x^2 on the diagonal
  for (int i = 0; i < 9; ++i) {
    double s = 0.0;
    for (int k = 0; k < 5; ++k) s += lam[11 + k] * p.nu[i][k];
    H[13 + i] = -s / (x[i] * x[i]);
  }
  double HTT = 0.0;
  for (int k = 0; k < 5; ++k) HTT -= lam[11 + k] * (2.0 * p.B[k] / (T * T * T) - p.C[k] / (T * T));
  // water VLE: -x_W Psat(T)
  const double psat = exp(p.psat_a - p.psat_b / T);
  const double b = p.psat_b;
  const double psat_T = psat * b / (T * T);
  const double psat_TT = psat * (b * b / (T * T * T * T) - 2.0 * b / (T * T * T));
  const double lw = lam[18];
  HTT += -lw * x[8] * psat_TT;
  // CO2 VLE: -x_C H(T, A, W)
  const Henry h = henry(p, z);
  const double lc = lam[19];
  const double xc = x[7];
  const double vaa = -lc * xc * h.Haa;
  H[13 + 0] += vaa;
  H[13 + 1] += vaa;
  H[13 + 3] += vaa;
  H[13 + 8] += -lc * xc * h.HWW;
  H[22] = vaa;
  H[23] = vaa;
  H[24] = vaa;
  for (int a = 0; a < 3; ++a) H[25 + a] = -lc * h.Ha;
  for (int a = 0; a < 3; ++a) H[28 + a] = -lc * xc * h.HaW;
  H[31] = -lc * h.HW;
  HTT += -lc * xc * h.HTT;
  // (T, x_i): energy balance liquid terms, VLE pieces
  for (int i = 0; i < 9; ++i) H[32 + i] = wEBl * L * cpL(p, i, T);
  H[32 + 8] += -lw * psat_T;
  H[32 + 0] += -lc * xc * h.HaT;
  H[32 + 1] += -lc * xc * h.HaT;
  H[32 + 3] += -lc * xc * h.HaT;
  H[32 + 7] += -lc * h.HT;
  H[32 + 8] += -lc * xc * h.HWT;
  for (int j = 0; j < 4; ++j) H[41 + j] = wEBv * V * cpV(p, j, T);
  H[45] = wEBl * cpl_mix;
  H[46] = wEBv * cpv_mix + lam[21] * p.R / P;
  HTT += wEBl * L * dcpl_mix + wEBv * V * dcpv_mix;
  H[47] = HTT;
}

// (d, d) Hessian entry contributed by one hydraulic row with weight lam_h
ABS_HD double hess_dd(const ModelParams& p, double lam_h) { return -lam_h * p.u_max * M_PI * 0.5; }

}  // namespace absorber
