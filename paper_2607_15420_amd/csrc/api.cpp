// C ABI of the absorber library: handle management, structures, evaluation and
// the KKT factorise/solve entry points.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace absorber {

namespace {
thread_local std::string g_last_error;

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

struct StructSink {
  std::vector<JacEntry>* own;
  std::vector<JacEntry>* up;
  std::vector<JacEntry>* down;
  int d_index = -1;
  void operator()(int r, int blk, int col, double) {
    JacEntry e{(int8_t)r, (int8_t)blk, (int8_t)col};
    if (blk == BLK_OWN || blk == BLK_D) {
      if (blk == BLK_D) d_index = (int)own->size();
      own->push_back(e);
    } else if (blk == BLK_UP) {
      up->push_back(e);
    } else {
      down->push_back(e);
    }
  }
};

int coupling_slot_of(int local) {  // inverse of coupling_index, -1 if not a coupling index
  for (int a = 0; a < NC; ++a)
    if (coupling_index(a) == local) return a;
  return -1;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

// Build the Jacobian structure (by running the same emission code as the
// device kernels on a dummy interior point) and the frontal gather table.
static int build_tables(Handle& h) {
  double z[NV];
  for (int k = 0; k < NV; ++k) z[k] = 0.1 + 0.01 * k;
  z[IT] = 320.0;
  double feed[NF];
  for (int i = 0; i < NF; ++i) feed[i] = 0.1;
  feed[16] = feed[5] = 320.0;
  feed[17] = 1e5;
  Inflow f;
  make_inflow(z, z, feed, f);
  StructSink ss{&h.jac_own, &h.jac_up, &h.jac_down};
  stage_jacobian(h.mp, z, f, 1e5, 1.0, true, true, ss);
  h.jac_d_index = ss.d_index;
  if ((int)h.jac_own.size() != NJO || (int)h.jac_up.size() != NJU || (int)h.jac_down.size() != NJD) {
    set_error("unexpected Jacobian structure (the stoichiometry must have the pattern of R1-R5)");
    return ABS_ERR_ARG;
  }
  hess_positions(h.hpos);
  // gather table: up to three LDS source indices per frontal position
  std::vector<int> cnt(FR * 64, 0), tab(FR * 64, 0);
  bool overflow = false;
  auto put = [&](int i, int j, int src) {
    const int p = i * 64 + j;
    if (cnt[p] >= 3) {
      overflow = true;
      return;
    }
    tab[p] |= src << (10 * cnt[p]);
    ++cnt[p];
  };
  auto put2 = [&](int i, int j, int src) {
    put(i, j, src);
    if (i != j) put(j, i, src);
  };
  for (int e = 0; e < NJO; ++e) {
    const JacEntry& je = h.jac_own[e];
    if (je.blk == BLK_D) {
      put2(NK - 1, FR_B, SRC_BRD);
      continue;
    }
    const int lr = je.row < NE ? NV + je.row : NK - 1;
    put2(lr, je.col, SRC_REC + REC_OWN + e);
  }
  for (int e = 0; e < NJU; ++e) {
    const JacEntry& je = h.jac_up[e];
    const int a = coupling_slot_of(je.col);
    put2(NK + a, NV + je.row, SRC_REC + REC_UP + e);
  }
  for (int e = 0; e < NJD; ++e) {
    const JacEntry& je = h.jac_down[e];
    const int a = coupling_slot_of(NV + je.row);
    put2(NK + a, je.col, SRC_DOWN1 + e);
  }
  for (int e = 0; e < NH; ++e) put2(h.hpos[e].r, h.hpos[e].c, SRC_REC + REC_H + e);
  for (int k = 0; k < NV; ++k) put(k, k, SRC_DIAGX + k);
  for (int r = 0; r < NE; ++r) put(NV + r, NV + r, SRC_DC);
  put(NK - 1, NK - 1, SRC_DHYD);
  for (int k = 0; k < NK; ++k) put2(FR_R, k, SRC_RHS + k);
  for (int a = 0; a < NC; ++a) {
    for (int b = 0; b < NC; ++b) put(coupling_index(b), coupling_index(a), SRC_CTB + a * (NC + 2) + b);
    put2(FR_R, coupling_index(a), SRC_CTB + a * (NC + 2) + NC);
    put2(FR_B, coupling_index(a), SRC_CTB + a * (NC + 2) + NC + 1);
  }
  for (int e = 0; e < NJU; ++e)
    if (coupling_slot_of(h.jac_up[e].col) < 0) overflow = true;
  for (int e = 0; e < NJD; ++e)
    if (coupling_slot_of(NV + h.jac_down[e].row) < 0) overflow = true;
  for (int i = 0; i < FR; ++i) {
    const int cap = 1 + (int)((GATHER2 >> i) & 1ull) + (int)((GATHER3 >> i) & 1ull);
    for (int j = 0; j < 64; ++j)
      if (cnt[i * 64 + j] > cap) overflow = true;
  }
  if (overflow) {
    set_error("internal: frontal gather table does not fit the stage structure");
    return ABS_ERR_ARG;
  }
  HIP_TRY(dalloc(&h.gather, tab.size()));
  HIP_TRY(hipMemcpy(h.gather, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
  std::vector<int> jt;
  for (auto& e : h.jac_own) jt.push_back(e.row | (e.col << 8) | (e.blk << 16));
  for (auto& e : h.jac_up) jt.push_back(e.row | (e.col << 8) | (e.blk << 16));
  for (auto& e : h.jac_down) jt.push_back(e.row | (e.col << 8) | (e.blk << 16));
  HIP_TRY(dalloc(&h.jtab, jt.size()));
  HIP_TRY(hipMemcpy(h.jtab, jt.data(), jt.size() * sizeof(int), hipMemcpyHostToDevice));
  // Residual terms: for each KKT row i of a stage, the products K_ij x_j that
  // make up (K x)_i, as (coefficient, unknown) codes.  The same matrix as the
  // frontal gather above (own block, couplings to both neighbours, border),
  // without the factorisation's right-hand side and Schur contributions.
  enum { X0, XDN, XUP, XD };
  std::vector<std::vector<std::pair<int, int>>> terms(NK);
  auto rterm = [&](int row, int coef, int xkind, int xidx) {  // coef: record offset (may lie in a neighbour)
    const int xc = xkind == XD ? RT_XDTERM
                               : (xidx + (xkind == XDN ? -NK : (xkind == XUP ? NK : 0)) + RT_XOFF) |
                                     (xkind == XDN ? RT_NBDN : (xkind == XUP ? RT_NBUP : 0));
    terms[(size_t)row].push_back({coef + RT_COFF, xc});
  };
  auto dterm = [&](int row, int didx) { terms[(size_t)row].push_back({RT_DIAG + didx, row + RT_XOFF}); };
  for (int e = 0; e < NJO; ++e) {
    const JacEntry& je = h.jac_own[(size_t)e];
    if (je.blk == BLK_D) {
      rterm(NK - 1, REC_OWN + e, XD, 0);  // hydraulic row x border (the d row is reduced separately)
      continue;
    }
    const int lr = je.row < NE ? NV + je.row : NK - 1;
    rterm(lr, REC_OWN + e, X0, je.col);
    rterm(je.col, REC_OWN + e, X0, lr);
  }
  for (int e = 0; e < NJU; ++e) {  // own rows x the stage above; our variables' rows see the stage below's
    const JacEntry& je = h.jac_up[(size_t)e];
    rterm(NV + je.row, REC_UP + e, XUP, je.col);
    rterm(je.col, REC_UP + e - REC, XDN, NV + je.row);
  }
  for (int e = 0; e < NJD; ++e) {  // own rows x the stage below; our variables' rows see the stage above's
    const JacEntry& je = h.jac_down[(size_t)e];
    rterm(NV + je.row, REC_DOWN + e, XDN, je.col);
    rterm(je.col, REC_DOWN + e + REC, XUP, NV + je.row);
  }
  for (int e = 0; e < NH; ++e) {
    rterm(h.hpos[e].r, REC_H + e, X0, h.hpos[e].c);
    if (h.hpos[e].r != h.hpos[e].c) rterm(h.hpos[e].c, REC_H + e, X0, h.hpos[e].r);
  }
  for (int k = 0; k < NV; ++k) dterm(k, k);                 // Sigma_x + delta_w
  for (int r = 0; r < NE; ++r) dterm(NV + r, NV);           // -delta_c
  dterm(NK - 1, NV + 1);                                    // -(1/(Sigma_s + delta_w) + delta_c)
  std::vector<int> order(NK);
  for (int i = 0; i < NK; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return terms[(size_t)a].size() > terms[(size_t)b].size(); });
  std::vector<int> rt(order.begin(), order.end());
  rt.push_back(0);
  for (int i = 0; i < NK; ++i) rt.push_back(rt.back() + (int)terms[(size_t)order[(size_t)i]].size());
  for (int i = 0; i < NK; ++i)
    for (auto& pr : terms[(size_t)order[(size_t)i]]) {
      rt.push_back(pr.first);
      rt.push_back(pr.second);
    }
  if ((int)rt.size() > RT_MAX) {
    set_error("internal: residual term table too large");
    return ABS_ERR_ARG;
  }
  HIP_TRY(dalloc(&h.rtab, rt.size()));
  HIP_TRY(hipMemcpy(h.rtab, rt.data(), rt.size() * sizeof(int), hipMemcpyHostToDevice));
  h.rtab_n = (int)rt.size();
  // Lagrangian gradient terms J^T y for the NV variables of a stage: the terms
  // of the residual rows 0..NV-1 whose unknown is a multiplier, with the
  // unknown re-indexed into the row vector (row r of this stage or a neighbour)
  std::vector<int> gt(NV + 1, 0);
  std::vector<int> gterms;
  for (int k = 0; k < NV; ++k) {
    for (auto& pr : terms[(size_t)k]) {
      const int xc = pr.second;
      if (xc & RT_XDTERM) continue;
      const int nb = xc & (RT_NBDN | RT_NBUP);
      const int off = (xc & (RT_XDTERM - 1)) - RT_XOFF;                    // offset in KKT unknowns
      const int local = off - (nb == RT_NBDN ? -NK : (nb == RT_NBUP ? NK : 0));  // index in the stage
      if (local < NV) continue;                                          // Hessian or diagonal term
      const int yoff = (local - NV) + (nb == RT_NBDN ? -NR : (nb == RT_NBUP ? NR : 0));
      gterms.push_back(pr.first);
      gterms.push_back((yoff + RT_XOFF) | nb);
    }
    gt[(size_t)k + 1] = (int)gterms.size() / 2;
  }
  gt.insert(gt.end(), gterms.begin(), gterms.end());
  if ((int)gt.size() > RT_MAX) {
    set_error("internal: gradient term table too large");
    return ABS_ERR_ARG;
  }
  HIP_TRY(dalloc(&h.gtab, gt.size()));
  HIP_TRY(hipMemcpy(h.gtab, gt.data(), gt.size() * sizeof(int), hipMemcpyHostToDevice));
  h.gtab_n = (int)gt.size();
  return ABS_OK;
}

int initial_point(Handle& h, double* x_dev, hipStream_t st) {
  HIP_TRY(launch_tile_x0(h, x_dev, st));
  return ABS_OK;
}

hipError_t wait_stream(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
  }
}

static hipEvent_t prof_event(Handle& h) {
  if (!h.prof_pool.empty()) {
    hipEvent_t e = h.prof_pool.back();
    h.prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing only: no system-scope fence (no cache writeback) when the event is recorded
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(Handle& h, int cls, hipStream_t st) {
  if (!(h.prof & (1 << cls))) return;
  if (!h.prof_open) h.prof_open = prof_event(h);
  if (h.prof_open) (void)hipEventRecord(h.prof_open, st);
}

void prof_end(Handle& h, int cls, hipStream_t st) {
  if (!(h.prof & (1 << cls)) || !h.prof_open) return;
  hipEvent_t e1 = prof_event(h);
  if (!e1) return;
  (void)hipEventRecord(e1, st);
  h.prof_pending.push_back({h.prof_open, e1, cls});
  h.prof_open = nullptr;
  if (h.prof_pending.size() >= 512) (void)prof_flush(h);
}

int prof_flush(Handle& h) {
  size_t done = 0;
  hipError_t err = hipSuccess;
  for (; done < h.prof_pending.size(); ++done) {
    const auto& q = h.prof_pending[done];
    err = hipEventSynchronize(q.e1);  // returns at once for an event already reached
    if (err != hipSuccess) break;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, q.e0, q.e1) == hipSuccess) {
      h.prof_ms[q.cls] += ms;
      h.prof_calls[q.cls] += 1;
    }
    h.prof_pool.push_back(q.e0);
    h.prof_pool.push_back(q.e1);
  }
  // each event is either still pending or back in the pool, never both
  h.prof_pending.erase(h.prof_pending.begin(), h.prof_pending.begin() + (long)done);
  HIP_TRY(err);
  return ABS_OK;
}

static void free_handle(Handle& h) {
  free_ipm_graph(h);
  if (!h.prof_pending.empty()) (void)hipEventSynchronize(h.prof_pending.back().e1);
  for (const auto& q : h.prof_pending) {
    (void)hipEventDestroy(q.e0);
    (void)hipEventDestroy(q.e1);
  }
  for (hipEvent_t e : h.prof_pool) (void)hipEventDestroy(e);
  if (h.prof_open) (void)hipEventDestroy(h.prof_open);
  void* ptrs[] = {h.feeds, h.gather, h.rtab, h.gtab, h.jtab, h.cs, h.rec, h.slots, h.slot_lines, h.solr, h.solb, h.inert, h.part,
                  h.scal, h.diagx, h.diags, h.kres, h.kcor, h.kden, h.omega_d, h.redbuf,
                  h.warm_X, h.warm_Y, h.warm_x0, h.warm_l0, h.warm_w, h.sinfo, h.chain0, h.chain_p, h.pchain, h.pstage,
                  h.seg, h.pseg, h.ctl, h.ipm_work, h.pres, h.rmask, h.solbk, h.brhs, h.pdots, h.dsc, h.opa};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h.scal_h) (void)hipHostFree(h.scal_h);
  if (h.redbuf_h) (void)hipHostFree(h.redbuf_h);
  if (h.ctl_h) (void)hipHostFree(h.ctl_h);
  if (h.ipm_dd_h) (void)hipHostFree(h.ipm_dd_h);
  if (h.pres_h) (void)hipHostFree(h.pres_h);
  if (h.rmask_h) (void)hipHostFree(h.rmask_h);
  if (h.ctl_ev) (void)hipEventDestroy(h.ctl_ev);
}

// (re)allocate the scaled row-scale vector as ones
static int reset_row_scale(Handle& h) {
  std::vector<double> ones((size_t)h.nc, 1.0);
  HIP_TRY(hipMemcpy(h.cs, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice));
  return ABS_OK;
}

}  // namespace absorber

using namespace absorber;

extern "C" {

const char* absorber_last_error(void) { return g_last_error.c_str(); }

static int create_impl(const absorber_params* prm, int32_t n_problems, const int32_t* n_stages,
                       const int32_t* n_scen, const double* feeds_host, int npar, absorber_t** out);

int absorber_create_batch(const absorber_params* prm, int32_t n_problems, const int32_t* n_stages,
                          const int32_t* n_scen, const double* feeds_host, absorber_t** out) {
  if (!prm || !feeds_host || !out || !n_stages || !n_scen || n_problems < 1) {
    set_error("absorber_create_batch: bad argument");
    return ABS_ERR_ARG;
  }
  return create_impl(prm, n_problems, n_stages, n_scen, feeds_host, 1, out);
}

int absorber_create_sections(const absorber_params* prm, int32_t n_stages, int32_t n_scen, int32_t n_sections,
                             const double* feeds_host, absorber_t** out) {
  if (!prm || !feeds_host || !out || n_stages < 1 || n_scen < 1 || n_stages > 4096 || n_sections < 1 ||
      n_sections > MAX_NPAR || n_sections > n_stages) {
    set_error("absorber_create_sections: bad argument (1 <= n_sections <= min(4, n_stages))");
    return ABS_ERR_ARG;
  }
  return create_impl(prm, 1, &n_stages, &n_scen, feeds_host, n_sections, out);
}

static int create_impl(const absorber_params* prm, int32_t n_problems, const int32_t* n_stages,
                       const int32_t* n_scen, const double* feeds_host, int npar, absorber_t** out) {
  long long nst = 0, W = 0;
  int Nmax = 0;
  for (int p = 0; p < n_problems; ++p) {
    if (n_stages[p] < 1 || n_stages[p] > 4096 || n_scen[p] < 1) {
      set_error("absorber_create_batch: stage counts must be 1..4096 and scenario counts >= 1");
      return ABS_ERR_ARG;
    }
    nst += (long long)n_stages[p] * n_scen[p];
    W += n_scen[p];
    Nmax = std::max(Nmax, (int)n_stages[p]);
  }
  if (W > 2147483647LL / 4 || nst > 2147483647LL) {
    set_error("absorber_create_batch: too many stages");
    return ABS_ERR_ARG;
  }
  if (!(prm->dp_stage >= 0.0) || !std::isfinite(prm->dp_stage)) {
    set_error("absorber_create: dp_stage must be finite and >= 0");
    return ABS_ERR_ARG;
  }
  if (!(prm->op_weight >= 0.0) || !std::isfinite(prm->op_weight) || !(prm->op_loss_coef >= 0.0) ||
      !std::isfinite(prm->op_loss_coef)) {
    set_error("absorber_create: op_weight and op_loss_coef must be finite and >= 0");
    return ABS_ERR_ARG;
  }
  if (prm->op_weight > 0.0 && n_problems > 1) {
    set_error("absorber_create_batch: the operating cost is for single-problem handles (one objective scaling)");
    return ABS_ERR_ARG;
  }
  auto* H = new (std::nothrow) absorber_handle();
  if (!H) return ABS_ERR_OOM;
  Handle& h = H->h;
  h.P = n_problems;
  h.npar = npar;
  if (npar > 1) {
    for (int k = 0; k < MAX_NPAR; ++k) h.cw[k] = 0.0;
    for (int n = 0; n < n_stages[0]; ++n) h.cw[section_of(n, n_stages[0], npar)] += 1.0 / n_stages[0];
  }
  h.N = Nmax;
  h.S = (int)W;
  h.nst = nst;
  h.pN.assign(n_stages, n_stages + n_problems);
  h.pS.assign(n_scen, n_scen + n_problems);
  h.nx = nst * NV + (long long)h.P * npar;
  h.nc = nst * NR;
  h.nkkt = nst * NK + (long long)h.P * npar;
  ModelParams& mp = h.mp;
  memcpy(mp.nu, prm->nu, sizeof(mp.nu));
  for (int k = 0; k < 5; ++k) {
    mp.A[k] = prm->lnK_A[k];
    mp.B[k] = prm->lnK_B[k];
    mp.C[k] = prm->lnK_C[k];
    mp.D[k] = prm->lnK_D[k];
  }
  mp.psat_a = prm->psat_a;
  mp.psat_b = prm->psat_b;
  mp.lnH298 = prm->henry_lnH298;
  mp.kH = prm->henry_kappa;
  mp.TH = prm->henry_Tref;
  mp.lnr = prm->henry_ln_ratio_MEA;
  mp.Tref = prm->Tref;
  for (int i = 0; i < 9; ++i) {
    mp.hL_ref[i] = prm->hL_ref[i];
    mp.cpL_a[i] = prm->cpL_a[i];
    mp.cpL_b[i] = prm->cpL_b[i];
  }
  for (int j = 0; j < 4; ++j) {
    mp.hV_ref[j] = prm->hV_ref[j];
    mp.cpV_a[j] = prm->cpV_a[j];
    mp.cpV_b[j] = prm->cpV_b[j];
  }
  mp.R = prm->R;
  mp.u_max = prm->u_max;
  mp.dp = prm->dp_stage;
  for (int k = 0; k < NV; ++k) {
    h.xL[k] = -INFINITY;
    h.xU[k] = INFINITY;
  }
  for (int i = 0; i < 9; ++i) {
    h.xL[IX + i] = prm->x_lo;
    h.xU[IX + i] = prm->x_hi;
  }
  for (int j = 0; j < 4; ++j) {
    h.xL[IY + j] = prm->y_lo;
    h.xU[IY + j] = prm->y_hi;
  }
  h.xL[IL] = prm->L_lo;
  h.xU[IL] = prm->L_hi;
  h.xL[IV] = prm->V_lo;
  h.xU[IV] = prm->V_hi;
  h.xL[IT] = prm->T_lo;
  h.xU[IT] = prm->T_hi;
  h.dL = prm->d_lo;
  h.dU = prm->d_hi;
  for (int k = 0; k < NV; ++k) h.sc.D[k] = 1.0;
  h.sc.Dd = 1.0;
  h.feeds_h.assign(feeds_host, feeds_host + (size_t)h.S * NF);
  // chain, stage and segment tables
  std::vector<StageInfo> sinfo((size_t)nst);
  std::vector<int> chain0((size_t)W + 1), chain_p((size_t)W), pchain((size_t)h.P + 1), pseg((size_t)h.P + 1);
  std::vector<long long> pstage((size_t)h.P + 1);
  std::vector<Seg> segs;
  {
    long long t = 0;
    int w = 0;
    for (int p = 0; p < h.P; ++p) {
      pchain[p] = w;
      pstage[p] = t;
      pseg[p] = (int)segs.size();
      const long long ts = t;
      for (int q = 0; q < h.pS[p]; ++q, ++w) {
        chain0[w] = (int)t;
        chain_p[w] = p;
        for (int n = 0; n < h.pN[p]; ++n, ++t) sinfo[(size_t)t] = StageInfo{w, n, h.pN[p], p};
      }
      for (long long a = ts; a < t; a += SEG) segs.push_back(Seg{(int)a, (int)std::min(t, a + SEG), p, a == ts ? npar : 0});
    }
    chain0[W] = (int)t;
    pchain[h.P] = w;
    pstage[h.P] = t;
    pseg[h.P] = (int)segs.size();
  }
  h.nseg = (int)segs.size();
  h.pchain_h.assign(pchain.begin(), pchain.end());
  h.pstage_h = pstage;
  h.pseg_h = pseg;
  static_assert(sizeof(absorber_params) > 0, "");
  for (int k = 0; k < NV; ++k) h.x0[k] = prm->x0[k];
  h.x0[NV] = prm->d0;
  int rc = ABS_OK;
  auto fail = [&](int code) {
    free_handle(h);
    delete H;
    return code;
  };
#define ALLOC(ptr, n)                                                     \
  do {                                                                    \
    if (dalloc(&(ptr), (size_t)(n)) != hipSuccess) {                      \
      set_error("absorber_create: device allocation failed (" #ptr ")"); \
      return fail(ABS_ERR_OOM);                                           \
    }                                                                     \
  } while (0)
  ALLOC(h.feeds, (size_t)h.S * NF);
  ALLOC(h.cs, h.nc);
  ALLOC(h.rec, nst * REC);
  ALLOC(h.slots, nst * NK * SLOT);
  ALLOC(h.slot_lines, nst * 2);
  ALLOC(h.solr, nst * NK);
  ALLOC(h.solb, nst * NK);
  ALLOC(h.inert, (size_t)h.S * 4);
  ALLOC(h.part, (size_t)h.S * 4);
  ALLOC(h.scal, h.P);
  if (npar > 1) {
    ALLOC(h.solbk, nst * NK * (npar - 1));
    ALLOC(h.brhs, nst * NK * (npar - 1));
    ALLOC(h.pdots, (size_t)h.S * PDOT);
    ALLOC(h.dsc, (size_t)h.P * DSC);
  }
  ALLOC(h.opa, (size_t)h.P * npar);
  ALLOC(h.sinfo, nst);
  ALLOC(h.chain0, W + 1);
  ALLOC(h.chain_p, W);
  ALLOC(h.pchain, h.P + 1);
  ALLOC(h.pstage, h.P + 1);
  ALLOC(h.seg, h.nseg);
  ALLOC(h.pseg, h.P + 1);
  h.ctl_bytes = ctl_size(h.P);
  ALLOC(h.ctl, h.ctl_bytes);
  h.dwv = reinterpret_cast<double*>(h.ctl);
  h.dcv = h.dwv + h.P;
  h.fmask = reinterpret_cast<int*>(h.ctl + ctl_off_fmask(h.P));
  h.pact = reinterpret_cast<int*>(h.ctl + ctl_off_pact(h.P));
  h.slot_area = h.ctl + ctl_off_slot(h.P);
  ALLOC(h.omega_d, 8);
  ALLOC(h.pres, 2LL * h.P);
  ALLOC(h.rmask, h.P);
  ALLOC(h.diagx, h.nx);
  ALLOC(h.diags, nst);
  ALLOC(h.kres, h.nkkt);
  ALLOC(h.kcor, h.nkkt);
  ALLOC(h.kden, 3 * nst + 5LL * h.nseg + 4LL * h.P + 64);  // per-stage scratch; residual partials
  h.red_cap = (int)std::max<long long>(
      64 * 1024, std::max<long long>(9 * ((std::max<long long>(h.nx, std::max(h.nc, h.nkkt)) + 255) / 256),
                                     9LL * (h.nseg + h.P)) + 64);
  ALLOC(h.redbuf, h.red_cap);
#undef ALLOC
  if (hipHostMalloc((void**)&h.scal_h, sizeof(DevScalars) * h.P, 0) != hipSuccess ||
      hipHostMalloc((void**)&h.redbuf_h, sizeof(double) * h.red_cap, 0) != hipSuccess ||
      hipHostMalloc((void**)&h.ctl_h, h.ctl_bytes, 0) != hipSuccess ||
      hipHostMalloc((void**)&h.pres_h, sizeof(double) * 2 * h.P, 0) != hipSuccess ||
      hipHostMalloc((void**)&h.rmask_h, sizeof(int) * 2 * h.P, 0) != hipSuccess ||
      hipEventCreateWithFlags(&h.ctl_ev, hipEventDisableTiming) != hipSuccess) {
    set_error("absorber_create: pinned host allocation failed");
    return fail(ABS_ERR_OOM);
  }
  if (hipMemcpy(h.feeds, feeds_host, sizeof(double) * (size_t)h.S * NF, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.sinfo, sinfo.data(), sizeof(StageInfo) * sinfo.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.chain0, chain0.data(), sizeof(int) * chain0.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.chain_p, chain_p.data(), sizeof(int) * chain_p.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.pchain, pchain.data(), sizeof(int) * pchain.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.pstage, pstage.data(), sizeof(long long) * pstage.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.seg, segs.data(), sizeof(Seg) * segs.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h.pseg, pseg.data(), sizeof(int) * pseg.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h.dwv, 0, sizeof(double) * h.P) != hipSuccess ||
      hipMemset(h.dcv, 0, sizeof(double) * h.P) != hipSuccess)
    return fail(ABS_ERR_HIP);
  // coefficients a_k of the expected operating cost sum_k a_k theta_k^-4 (eq. 8a):
  // the weight times the blower power of each equally likely scenario, whose
  // inlet gas (flow V0, temperature T, molar mass of its composition) enters at
  // the bottom stage's pressure and loses loss_coef rho u^2 / 2 in each stage of
  // section k at the superficial velocity u = Q / (pi theta_k^2 / 4)
  h.opa_h.assign((size_t)h.P * npar, 0.0);
  h.has_op = prm->op_weight > 0.0;
  if (h.has_op) {
    long long w0 = 0;
    for (int p = 0; p < n_problems; ++p) {
      const int N = n_stages[p];
      double acc = 0.0;
      for (int s = 0; s < n_scen[p]; ++s) {
        const double* f = feeds_host + (size_t)(w0 + s) * NF;
        const double p_in = stage_pressure(h.mp, f[17], 0, N);
        const double Q = f[0] * prm->R * f[5] / p_in;
        double Mg = 0.0;
        for (int j = 0; j < 4; ++j) Mg += f[1 + j] * prm->op_molar_mass[j];
        const double rho = p_in * Mg / (prm->R * f[5]);
        acc += rho * Q * Q * Q;
      }
      acc /= n_scen[p];
      for (int n = 0; n < N; ++n)
        h.opa_h[(size_t)p * npar + section_of(n, N, npar)] +=
            prm->op_weight * 8.0 * prm->op_loss_coef / (M_PI * M_PI) * acc;
      w0 += n_scen[p];
    }
  }
  if (hipMemcpy(h.opa, h.opa_h.data(), sizeof(double) * h.opa_h.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(ABS_ERR_HIP);
  if ((rc = build_tables(h)) != ABS_OK) return fail(rc);
  if ((rc = reset_row_scale(h)) != ABS_OK) return fail(rc);
  if (hipMemset(h.rec, 0, sizeof(double) * nst * REC) != hipSuccess) return fail(ABS_ERR_HIP);
  *out = H;
  return ABS_OK;
}

int absorber_create(const absorber_params* prm, int32_t n_stages, int32_t n_scen, const double* feeds_host,
                    absorber_t** out) {
  if (!prm || !feeds_host || !out || n_stages < 1 || n_scen < 1 || n_stages > 4096) {
    set_error("absorber_create: bad argument");
    return ABS_ERR_ARG;
  }
  return absorber_create_batch(prm, 1, &n_stages, &n_scen, feeds_host, out);
}

void absorber_destroy(absorber_t* H) {
  if (!H) return;
  free_handle(H->h);
  delete H;
}

int absorber_get_dims(const absorber_t* H, absorber_dims* out) {
  if (!H || !out) {
    set_error("absorber_get_dims: bad argument");
    return ABS_ERR_ARG;
  }
  const Handle& h = H->h;
  const long long nst = h.nst;
  out->n_var_total = 30 * nst + (long long)h.P * h.npar;
  out->n_var_free = 21 * nst + (long long)h.P * h.npar;
  out->n_eq = 21 * nst;
  out->n_fixed = 9 * nst;
  out->n_ineq = nst;
  long long nnz = 0;
  for (int p = 0; p < h.P; ++p)
    nnz += (long long)h.pS[p] * ((long long)h.pN[p] * NJO + (long long)(h.pN[p] - 1) * (NJU + NJD));
  out->nnz_jac = nnz;
  out->nnz_hess = nst * NH + h.P;
  out->kkt_dim = nst * NK + (long long)h.P * h.npar;
  return ABS_OK;
}

int absorber_initial_point(absorber_t* H, double* x_dev, void* stream) {
  if (!H || !x_dev) {
    set_error("absorber_initial_point: bad argument");
    return ABS_ERR_ARG;
  }
  return initial_point(H->h, x_dev, (hipStream_t)stream);
}

int absorber_profile_enable(absorber_t* H, int32_t on) {
  if (!H) {
    set_error("absorber_profile_enable: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  const int rc = prof_flush(h);  // pending times belong to the previous setting
  if (rc != ABS_OK) return rc;
  for (int k = 0; k < 4; ++k) {
    h.prof_ms[k] = 0.0;
    h.prof_calls[k] = 0;
  }
  h.prof = on;
  return ABS_OK;
}

int absorber_profile_get(const absorber_t* H, absorber_profile* out) {
  if (!H || !out) {
    set_error("absorber_profile_get: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = const_cast<Handle&>(H->h);
  const int rc = prof_flush(h);
  if (rc != ABS_OK) return rc;
  for (int k = 0; k < 4; ++k) {
    out->ms[k] = h.prof_ms[k];
    out->calls[k] = h.prof_calls[k];
  }
  out->bytes_factor_slots = (int64_t)h.nst * NK * SLOT * (int64_t)sizeof(double);
  return ABS_OK;
}

int absorber_set_scaling(absorber_t* H, const double* var_scale_host, const double* row_scale_dev) {
  if (!H) {
    set_error("absorber_set_scaling: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_set_scaling: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  for (int k = 0; k < NV; ++k) h.sc.D[k] = var_scale_host ? var_scale_host[k] : 1.0;
  h.sc.Dd = var_scale_host ? var_scale_host[NV] : 1.0;
  if (row_scale_dev) {
    HIP_TRY(hipMemcpy(h.cs, row_scale_dev, sizeof(double) * h.nc, hipMemcpyDeviceToDevice));
  } else {
    return reset_row_scale(h);
  }
  return ABS_OK;
}

int absorber_eval_cons(absorber_t* H, const double* x_dev, double* c_dev, void* stream) {
  if (!H || !x_dev || !c_dev) {
    set_error("absorber_eval_cons: bad argument");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  Scaling one{};
  for (int k = 0; k < NV; ++k) one.D[k] = 1.0;
  one.Dd = 1.0;
  HIP_TRY(launch_eval_ext(h, x_dev, 0, one, nullptr, nullptr, 0, c_dev, (hipStream_t)stream));
  return ABS_OK;
}

int absorber_eval_obj(absorber_t* H, const double* x_dev, double* f_host, double* grad_dev, void* stream) {
  if (!H || !x_dev) {
    set_error("absorber_eval_obj: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_eval_obj: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  hipStream_t st = (hipStream_t)stream;
  // f = sum_k c_k theta_k + a_k theta_k^-4 (c_k: the share of stages in section k,
  // a_k: the expected operating cost's coefficients; f = d for problem (10))
  const long long nd = h.npar, nxs = h.nx - nd;
  double th[MAX_NPAR], g[MAX_NPAR];
  HIP_TRY(hipMemcpyAsync(th, x_dev + nxs, sizeof(double) * nd, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double f = 0.0;
  for (int k = 0; k < nd; ++k) {
    const double a = h.opa_h[(size_t)k], t4 = th[k] * th[k] * th[k] * th[k];
    f += h.cw[k] * th[k] + (a != 0.0 ? a / t4 : 0.0);
    g[k] = h.cw[k] - (a != 0.0 ? 4.0 * a / (t4 * th[k]) : 0.0);
  }
  if (grad_dev) {
    HIP_TRY(hipMemsetAsync(grad_dev, 0, sizeof(double) * nxs, st));
    HIP_TRY(hipMemcpyAsync(grad_dev + nxs, g, sizeof(double) * nd, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  if (f_host) *f_host = f;
  return ABS_OK;
}

int absorber_jac_structure(const absorber_t* H, int64_t* rows, int64_t* cols) {
  if (!H || !rows || !cols) {
    set_error("absorber_jac_structure: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_jac_structure: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  if (H->h.npar != 1) {
    set_error("absorber_jac_structure: handles with one diameter only (a section handle is solved by absorber_ipm_solve)");
    return ABS_ERR_ARG;
  }
  const Handle& h = H->h;
  long long k = 0;
  const long long dcol = h.nx - 1;
  for (int w = 0; w < h.S; ++w)  // single problem: chain w holds stages w N .. w N + N - 1
    for (int n = 0; n < h.N; ++n) {
      const long long t = (long long)w * h.N + n;
      for (auto& e : h.jac_own) {
        rows[k] = t * NR + e.row;
        cols[k] = e.blk == BLK_D ? dcol : t * NV + e.col;
        ++k;
      }
      if (n < h.N - 1)
        for (auto& e : h.jac_up) {
          rows[k] = t * NR + e.row;
          cols[k] = (t + 1) * NV + e.col;
          ++k;
        }
      if (n > 0)
        for (auto& e : h.jac_down) {
          rows[k] = t * NR + e.row;
          cols[k] = (t - 1) * NV + e.col;
          ++k;
        }
    }
  return ABS_OK;
}

int absorber_eval_jac(absorber_t* H, const double* x_dev, double* vals_dev, void* stream) {
  if (!H || !x_dev || !vals_dev) {
    set_error("absorber_eval_jac: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_eval_jac: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  if (H->h.npar != 1) {
    set_error("absorber_eval_jac: handles with one diameter only (a section handle is solved by absorber_ipm_solve)");
    return ABS_ERR_ARG;
  }
  HIP_TRY(launch_jac_coo(H->h, x_dev, vals_dev, (hipStream_t)stream));
  return ABS_OK;
}

int absorber_hess_structure(const absorber_t* H, int64_t* rows, int64_t* cols) {
  if (!H || !rows || !cols) {
    set_error("absorber_hess_structure: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_hess_structure: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  if (H->h.npar != 1) {
    set_error("absorber_hess_structure: handles with one diameter only (a section handle is solved by absorber_ipm_solve)");
    return ABS_ERR_ARG;
  }
  const Handle& h = H->h;
  long long k = 0;
  for (long long t = 0; t < h.nst; ++t)
    for (int e = 0; e < NH; ++e) {
      rows[k] = t * NV + h.hpos[e].r;
      cols[k] = t * NV + h.hpos[e].c;
      ++k;
    }
  rows[k] = cols[k] = h.nx - 1;
  return ABS_OK;
}

int absorber_eval_hess(absorber_t* H, const double* x_dev, const double* lambda_dev, double obj_factor,
                       double* vals_dev, void* stream) {
  (void)obj_factor;  // the objective d is linear
  if (!H || !x_dev || !lambda_dev || !vals_dev) {
    set_error("absorber_eval_hess: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_eval_hess: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  if (H->h.npar != 1) {
    set_error("absorber_eval_hess: handles with one diameter only (a section handle is solved by absorber_ipm_solve)");
    return ABS_ERR_ARG;
  }
  HIP_TRY(launch_hess_coo(H->h, x_dev, lambda_dev, vals_dev, (hipStream_t)stream));
  return ABS_OK;
}

int absorber_kkt_factor(absorber_t* H, const double* x_dev, const double* lambda_dev, const double* sigma_x_dev,
                        const double* sigma_s_dev, double delta_w, double delta_c, int64_t* inertia_host,
                        void* stream) {
  if (!H || !x_dev || !lambda_dev || !sigma_x_dev || !sigma_s_dev || !(delta_w >= 0) || !(delta_c >= 0)) {
    set_error("absorber_kkt_factor: bad argument");
    return ABS_ERR_ARG;
  }
  if (H->h.P != 1) {
    set_error("absorber_kkt_factor: single-problem handles only (use absorber_batch_solve for a batch)");
    return ABS_ERR_ARG;
  }
  Handle& h = H->h;
  hipStream_t st = (hipStream_t)stream;
  // the record is evaluated at x in original units with the handle's scaling
  HIP_TRY(launch_eval(h, x_dev, 0, lambda_dev, 1, h.kres, st));
  HIP_TRY(hipMemcpyAsync(h.diagx, sigma_x_dev, sizeof(double) * h.nx, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(h.diags, sigma_s_dev, sizeof(double) * h.nst, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(h.dwv, &delta_w, sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(h.dcv, &delta_c, sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_factor(h, h.diagx, h.diags, nullptr, false, st));
  HIP_TRY(launch_schur(h, h.diagx, nullptr, 0, nullptr, st));
  HIP_TRY(hipMemcpyAsync(h.scal_h, h.scal, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (inertia_host) {
    inertia_host[0] = h.scal_h->npos;
    inertia_host[1] = h.scal_h->nneg;
    inertia_host[2] = h.scal_h->nzero;
  }
  return ABS_OK;
}

}  // extern "C"
