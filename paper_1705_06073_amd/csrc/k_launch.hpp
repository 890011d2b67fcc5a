// Host-callable launch wrappers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "driver.hpp"
#include "sfls_kernels.hpp"

namespace sfls {

// Base pointers of every per-instance pool the driver kernel touches.
struct DrvPools {
  DrvState* st;
  double* th;
  double* ga;
  double* th_e;
  double* ga_e;
  double* g;
  double* d;
  double* gt;
  double* q_save;
  double* Sm;
  double* Ym;
  double* rhom;
  double* am;
  int32_t* K_e;
  int32_t* req;
  double* beta_e;
  double* gbar_e;
  double* zeta_e;
  // the evaluation's outputs (a driver that takes a shadow's evaluation
  // copies it here)
  cd* ev_q;
  cd* ev_r;
  cd* ev_u;
  cd* ev_s;
  cd* ev_t;
  cd* ev_v;
  cd* ev_x;
  double* logdet;
  double* yCy;
  double* ww;
  const int32_t* lev_status;
  const int32_t* cand;
  const int32_t* ncand;
  const cd* cand_q;
  const double* cand_s;
  double* cbuf_dl;
  double* cbuf_gh;
  int32_t* cbuf_l;
  int64_t* out_K;
  double* out_theta;
  cd* out_alpha;
  double* out_gamma;
  double* out_beta;
  double* out_zeta;
  double* out_obj;
  int32_t* out_iters;
  int32_t* out_evals;
  int32_t* out_status;
  const int64_t* out_koff;
  int32_t* notdone;
  // optional host-mapped copy of the request bits (pinned host memory the
  // device writes directly), so the host reads them without a copy per round
  int32_t* req_host;
  // the requests of the round's grid stage, which runs after the first
  // driver pass (the grid bits, else 0): those the round began with, and
  // grid sweeps at the point just evaluated that the first pass requested
  // (run at once instead of a round later; the host-mapped copy marks the
  // latter, for the host's accounting)
  int32_t* req2;
  int32_t* req2_host;
  // optional host-mapped copy of the number of components of each request
  // (the host's accounting of algorithmic work per round)
  int32_t* kev_host = nullptr;
  // observation vectors (Sec. V) and the vector strides (complex elements) of
  // ev_q/ev_r/ev_u/q_save, cand_q and out_alpha
  int32_t G = 1;
  int64_t kstride = 0, cstride = 0, ostride = 0;
  // shadow evaluation slots (speculative line-search trials): instance b's
  // shadow is instance b + nsh of the launch (nsh = 0: none); wish[b] marks
  // a shadow point the driver wrote this round
  int32_t nsh = 0;
  int32_t* wish = nullptr;
};

hipError_t launch_twiddles(cd* tw64, cf* tw32, cd* tws64, cf* tws32, int logtw, hipStream_t st);
// Shadow requests of the next round.  Workgroup i of a launch runs on the
// CU slot i mod ncu, so shadow workgroup nsh + j shares its slot with the
// instance's workgroup (nsh + j) mod ncu (nsh <= ncu): the shadows granted
// (wishes in instance order, req[nsh + b] = REQ_EVAL) are placed, through
// the launch order ord[nsh + j], on the slots whose instance requested no
// evaluation; the other shadows fill the remaining slots with no request.
// Wishes are cleared.  ord[0..nsh) is the order of the instances.
hipError_t launch_spec_grant(int32_t* req, int32_t* wish, int32_t* ord, int nsh, int ncu,
                             hipStream_t st);
// a1, direct sums and (per instance, by use_nufft_col) the type-1 NUFFT in
// the instance's scratch (4 P + padded(P) complex elements at poff).
hipError_t launch_toeplitz_column(const InstInfo* info, const int32_t* req, const int32_t* Kcnt,
                                  const double* theta, const double* gamma, const double* beta,
                                  cd* c, int B, int maxN, hipStream_t st, int nmode = 1,
                                  const cd* tws = nullptr, cd* scratch = nullptr, int maxP = 0);
// `order` (optional, B entries): the instance each workgroup of the launch
// takes, so that a batch of uneven sizes starts its longest instances first
// (identity when null).  Taken by the per-instance kernels whose time grows
// with N: the recursion, the GS apply and refinement, and the omega sums.
hipError_t launch_levinson(const InstInfo* info, const int32_t* req, const cd* c, cd* rho,
                           double* delta, double* logdet, int32_t* status, int64_t* failed, int B,
                           int maxN, hipStream_t st);
hipError_t launch_schur(const InstInfo* info, const int32_t* req, const SchurLayout* lay,
                        const SchurAct* acts, const cd* c, const cd* tw, int logtw,
                        const cd* tws, cd* scratch,
                        cd* rho, double* delta, double* logdet, int32_t* status, int64_t* failed,
                        int B, int Fmax, hipStream_t st, const int32_t* order = nullptr);
hipError_t launch_gs_apply(const InstInfo* info, const int32_t* req, const void* y, int ydtype,
                           const cd* rho, const double* delta, const cd* tw, int logtw,
                           const cd* tws, cd* scratch, cd* w, double* yCy, double* ww, int B,
                           int maxP,
                           hipStream_t st, const int32_t* order = nullptr, Vecs vv = Vecs{});
hipError_t launch_gen_refine(const InstInfo* info, const int32_t* req, const int32_t* status,
                             const cd* c, cd* rho, double* delta, const cd* tw, int logtw,
                             const cd* tws, cd* scratch, cd* r, cd* dx, int B, int maxP,
                             hipStream_t st, const int32_t* order = nullptr);
hipError_t launch_logdet_lemma(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                               const double* theta, const double* gamma,
                               const double* beta, const int32_t* status, double* logdet, int B,
                               hipStream_t st, const int32_t* order = nullptr);
hipError_t launch_omega(const InstInfo* info, const int32_t* req, const cd* rho,
                        const double* delta, const SepCoef* coef, const cd* tws,
                        cd* scratch, int which, int have_g0, cd* oms, cd* o_s, cd* o_t,
                        cd* o_v, cd* o_x, int B, int maxP, hipStream_t st,
                        const int32_t* order = nullptr);
hipError_t launch_grid(int prec, const InstInfo* info, const int32_t* req, const cd* w,
                       const cd* oms, const double* gbar, const double* zeta, const void* tw,
                       int logtw, int Rmax, int B, int maxM, void* qG, void* sG, void* dL,
                       double* part_val, int64_t* part_idx, hipStream_t st, Vecs vv = Vecs{});
hipError_t launch_grid_deriv(int prec, const InstInfo* info, const int32_t* req, const cd* w,
                             const cd* omt, const void* tw, int logtw, int Rmax, int B, int maxM,
                             void* rG, void* tG, hipStream_t st);
hipError_t launch_argmin_out(const InstInfo* info, int Rmax, const double* part_val,
                             const int64_t* part_idx, int64_t* amin, double* aval, int B,
                             hipStream_t st);
hipError_t launch_select(int prec, const InstInfo* info, const int32_t* req, const void* dL,
                         int Rmax, const double* part_val, const int64_t* part_idx,
                         double approx_ratio, double slack_rel, int cand_cap, int32_t* cand,
                         int32_t* ncand, int32_t* overflow, int B, hipStream_t st);
hipError_t launch_active(const InstInfo* info, const int32_t* req, const int32_t* Keval,
                         const int32_t* ncand, int32_t* prefix, int B, const double* theta,
                         const int32_t* cand, const cd* w, const cd* rho, const double* delta,
                         const SepCoef* coef, cd* oq, cd* orr, cd* ou, cd* os, cd* ot, cd* ov,
                         cd* ox, cd* cq, double* cs, int nblocks, int nmode, const cd* tws,
                         cd* scratch, int maxP, hipStream_t st, Vecs vv = Vecs{},
                         const int32_t* order = nullptr);
hipError_t launch_init_state(const InstInfo* info, const void* y, int ydtype, DrvState* st,
                             int32_t* req, int B, hipStream_t s, const int32_t* list = nullptr,
                             Vecs vv = Vecs{});
hipError_t launch_slots_idle(DrvState* st, int32_t* req, int B, hipStream_t s);
hipError_t launch_admit(const AdmitRec* recs, int n, const InstInfo* hinfo, const SepCoef* hcoef,
                        const SchurLayout* hlay, const int64_t* hkoff, InstInfo* dinfo,
                        SepCoef* dcoef, SchurLayout* dlay, int64_t* dkoff, void* ypool,
                        hipStream_t s);
hipError_t launch_gather_results(const int32_t* list, const int64_t* doff, int n,
                                 const int64_t* koff, const int64_t* oK, const double* otheta,
                                 const cd* oalpha, const double* ogamma, const double* obeta,
                                 const double* ozeta, const double* oobj, const int32_t* oiters,
                                 const int32_t* oevals, const int32_t* ostatus, SlotResult* res,
                                 double* comp, hipStream_t s);
// pass 0: every unfinished instance whose request has no grid sweep takes
// its step (with pools.req2: the others are deferred to pass 1); pass 1:
// the instances of pools.req2, after the round's grid stage has run; pass 2:
// only the instances in their initial phase (newly admitted ones, stepped
// before the round's evaluation kernels so that the round evaluates them).
hipError_t launch_driver(const InstInfo* info, const DrvParams* prm, DrvPools pools, int B,
                         hipStream_t st, int pass = 0);
hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st);

// Incomplete observations (Sec. IV), the semifast evaluation at the requested
// points (REQ_EVAL): phase tables (tabs, at tboff), Gram sums, the K x K
// Cholesky and inverse, ln|C|, s, t,
// v, x; then C^{-1} y on the observed samples (wM), y^H C^{-1} y, ||wM||^2,
// q, r, u.  status[b] = SFLS_ENOTPD when K_s is not positive definite.
hipError_t launch_sf_eval(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                          const double* theta, const double* gamma, const double* beta,
                          const void* y, int ydtype, const int32_t* idx, const cd* phi,
                          cd* sfm, cd* h, cd* cvec, cd* tabs, cd* wM, double* logdet, double* yCy,
                          double* ww, int32_t* status, cd* oq, cd* orr, cd* ou, cd* os, cd* ot,
                          cd* ov, cd* ox, int B, hipStream_t st);
// Grid-stage inputs at the evaluated point (REQ_GRID): w = Phi^H C^{-1} y as an
// N-vector at off, the columns U at uoff, and omega_s (lag i at i mod P) at
// poff of oms; scratch: the instance's P blocks (running sums, transform).
hipError_t launch_sf_grid_inputs(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                                 const double* theta, const double* gamma, const double* beta,
                                 const int32_t* idx, const cd* phi, const cd* wM, const cd* sfm,
                                 const cd* tabs, const cd* tws, cd* w, cd* U, cd* scratch,
                                 cd* oms, int B, int maxP, hipStream_t st);
// bad[b] = 1 when instance b's observed indices are not strictly increasing in
// [0, N) or a weight is zero or not finite (checked before any other use).
hipError_t launch_sf_check(const InstInfo* info, const int32_t* idx, const cd* phi, int32_t* bad,
                           int B, hipStream_t st);
// q and s at the grid candidates (REQ_GRID).
hipError_t launch_sf_cand(const InstInfo* info, const int32_t* req, const int32_t* Kev,
                          const double* beta, const int32_t* idx, const cd* phi, const cd* wM,
                          const cd* U, const int32_t* cand, const int32_t* ncand, cd* cq, double* cs,
                          int B, int maxN, hipStream_t st);

}  // namespace sfls
