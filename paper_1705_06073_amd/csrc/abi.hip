// C-ABI of the superfast-LSE library: argument checks, workspace, launch
// sequencing and the estimate round loop.  All arithmetic of the method runs
// in the kernels of k_*.hip; this file only moves sizes and pointers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "host_internal.hpp"

using namespace sfls;
using namespace sfls_host;

static_assert(sizeof(sfls_params) == 136, "sfls_params layout is part of the ABI");

const char* const kKernelNames[KID_COUNT] = {"toeplitz_column", "factor", "refine", "gs_apply",
                                             "omega", "grid", "select", "active", "driver"};

namespace sfls_host {

const char* kVersion = "sfls 0.1 (gfx950)";

sfls_status fail(sfls_ctx* ctx, sfls_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return s;
}


// grow-only named workspace buffer, within the context's HBM budget
sfls_status ws(sfls_ctx* ctx, const char* name, size_t bytes, void** out) {
  DevBuf& b = ctx->bufs[name];
  if (bytes == 0) bytes = 256;
  if (b.n < bytes) {
    size_t want = bytes + bytes / 4;
    if (ctx->hbm_budget && ctx->ws_bytes - b.n + want > ctx->hbm_budget) {
      want = bytes;  // no growth margin at the budget's edge
      if (ctx->ws_bytes - b.n + want > ctx->hbm_budget)
        return fail(ctx, SFLS_ENOMEM,
                    "workspace %s needs %zu bytes: the context's HBM budget of %zu bytes "
                    "(%zu in use) does not allow it", name, bytes, ctx->hbm_budget,
                    ctx->ws_bytes);
    }
    if (b.p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(b.p);
      ctx->ws_bytes -= b.n;
      b.p = nullptr;
      b.n = 0;
    }
    if (hipMalloc(&b.p, want) != hipSuccess) {
      b.p = nullptr;
      return fail(ctx, SFLS_ENOMEM, "workspace allocation of %zu bytes for %s failed", want, name);
    }
    b.n = want;
    ctx->ws_bytes += want;
  }
  *out = b.p;
  return SFLS_OK;
}

template <typename T>
sfls_status wsT(sfls_ctx* ctx, const char* name, size_t count, T** out) {
  void* p = nullptr;
  sfls_status s = ws(ctx, name, count * sizeof(T), &p);
  *out = static_cast<T*>(p);
  return s;
}

template <typename T>
sfls_status upload(sfls_ctx* ctx, const char* name, const std::vector<T>& v, hipStream_t st,
                   T** out) {
  sfls_status s = wsT<T>(ctx, name, v.size() ? v.size() : 1, out);
  if (s != SFLS_OK) return s;
  if (!v.empty()) {
    HIP_TRY(hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return SFLS_OK;
}

std::vector<int32_t> longest_first(int64_t B, const int64_t* n) {
  std::vector<int32_t> o;
  if (B < 2 || std::all_of(n, n + B, [&](int64_t v) { return v == n[0]; })) return o;
  o.resize((size_t)B);
  for (int64_t b = 0; b < B; ++b) o[(size_t)b] = (int32_t)b;
  std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
  return o;
}

int ilog2_ceil(int64_t v) {
  int l = 0;
  while (((int64_t)1 << l) < v) ++l;
  return l;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

hipError_t spin_wait(hipEvent_t ev) {
  for (;;) {
    const hipError_t q = hipEventQuery(ev);
    if (q != hipErrorNotReady) return q;
  }
}

// Polynomial coefficients of the diagonal-sum weights in centred variables
// x = q - c, y = p - c (p = q + i, c = (N-1)/2).  With S_k(n) = sum_{a=0}^n a^k,
// the Gohberg-Semencul form gives, for a row weight f,
//   omega_f(i) = delta^{-1} sum_q [S_f(q) - S_f(N-2-p)] rho_q conj(rho_p)
// (the ranges of the two triangular factors telescope; Appendix B):
//   s: S_0,  t: 2pi S_1,  v: (2pi)^2 S_2,  x: (2pi)^2 [S_2 + i S_1] (row and column weight).
void sep_coef(int N, SepCoef& out) {
  const double c = 0.5 * (double)(N - 1);
  const double d = (double)(N - 2) - c;
  const double Sk[3][4] = {{1.0, 1.0, 0.0, 0.0}, {0.0, 0.5, 0.5, 0.0},
                           {0.0, 1.0 / 6.0, 0.5, 1.0 / 3.0}};
  const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
  double Sq[3][4] = {}, Sm[3][4] = {};
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i <= j; ++i) {
        Sq[k][i] += Sk[k][j] * binom[j][i] * std::pow(c, j - i);
        Sm[k][i] += Sk[k][j] * binom[j][i] * std::pow(d, j - i) * ((i & 1) ? -1.0 : 1.0);
      }
  const double tp = 2.0 * M_PI, tp2 = tp * tp;
  std::memset(&out, 0, sizeof out);
  auto diff = [&](double* C, int k, double sc) {
    for (int i = 0; i < 4; ++i) {
      C[i * 4 + 0] += sc * Sq[k][i];
      C[0 * 4 + i] -= sc * Sm[k][i];
    }
  };
  diff(out.c[0], 0, 1.0);
  diff(out.c[1], 1, tp);
  diff(out.c[2], 2, tp2);
  diff(out.c[3], 2, tp2);
  // x: + (y - x) (S_1(c + x) - S_1(d - y))
  double* C = out.c[3];
  for (int i = 0; i < 3; ++i) {
    C[i * 4 + 1] += tp2 * Sq[1][i];        // a_i x^i y
    C[(i + 1) * 4 + 0] -= tp2 * Sq[1][i];  // -a_i x^{i+1}
    C[0 * 4 + (i + 1)] -= tp2 * Sm[1][i];  // -b_i y^{i+1}
    C[1 * 4 + i] += tp2 * Sm[1][i];        // +b_i x y^i
  }
}

sfls_status check_batch(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                        int64_t nmin) {
  if (B < 0) return fail(ctx, SFLS_EINVAL, "B = %lld < 0", (long long)B);
  if (B > 0 && (!n || !off)) return fail(ctx, SFLS_EINVAL, "n and off must be non-NULL");
  for (int64_t b = 0; b < B; ++b) {
    if (n[b] < nmin) return fail(ctx, SFLS_EINVAL, "n[%lld] = %lld < %lld", (long long)b, (long long)n[b], (long long)nmin);
    if (n[b] > SFLS_MAX_N)
      return fail(ctx, SFLS_EUNSUPPORTED, "n[%lld] = %lld exceeds SFLS_MAX_N = %d", (long long)b,
                  (long long)n[b], SFLS_MAX_N);
    if (off[b] < 0) return fail(ctx, SFLS_EINVAL, "off[%lld] < 0", (long long)b);
  }
  return SFLS_OK;
}

// Base InstInfo: N, P, off, poff (4 P scratch per instance).
std::vector<InstInfo> base_info(int64_t B, const int64_t* n, const int64_t* off, Sizes& sz,
                                int64_t& ptotal) {
  std::vector<InstInfo> v((size_t)B);
  ptotal = 0;
  for (int64_t b = 0; b < B; ++b) {
    InstInfo& in = v[(size_t)b];
    std::memset(&in, 0, sizeof in);
    in.N = (int32_t)n[b];
    in.logP = ilog2_ceil(2 * n[b] - 1 > 1 ? 2 * n[b] - 1 : 2);
    in.P = 1 << in.logP;
    in.logM = ilog2_ceil(n[b]);
    in.M = 1 << in.logM;
    in.off = off[b];
    in.poff = ptotal;
    ptotal += 4 * (int64_t)in.P + (in.P > CONV_LDS_P ? (int64_t)padded(in.P) : 0);
    sz.maxN = std::max(sz.maxN, in.N);
    sz.maxP = std::max(sz.maxP, in.P);
    sz.maxM = std::max(sz.maxM, in.M);
  }
  return v;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ----------------------------------------------------------------------------
// Superfast Schur plans: the recursion of each N flattened into actions.
// ----------------------------------------------------------------------------
void schur_rec(SchurPlan& P, int n0, int m, int level, int side, int win, int Nroot) {
  const bool root = level == 0;
  P.nlev = std::max(P.nlev, level + 1);
  P.mmax[level] = std::max(P.mmax[level], m);
  if (m <= 64 && !(root && m > 63)) {
    P.acts.push_back(SchurAct{root ? SCH_ROOT_LEAF : SCH_LEAF_ACT, n0, m, 0, level, side, win, 0});
    return;
  }
  const int m1 = m / 2, m2 = m - m1;
  const int logF = ilog2_ceil(root ? Nroot : m);
  P.fspec[level] = std::max(P.fspec[level], 1 << logF);
  schur_rec(P, n0, m1, level + 1, 0, win, Nroot);
  P.acts.push_back(SchurAct{SCH_MID, n0, m, m1, level, side, win, logF});
  schur_rec(P, n0 + m1, m2, level + 1, 1, level + 1, Nroot);
  P.acts.push_back(SchurAct{root ? SCH_ROOT : SCH_POST, n0, m, m1, level, side, win, logF});
}

// Algorithmic FP64 flops of one superfast factorisation (complex multiply-add
// = 8 flops, a complex transform of size F = 5 F log2 F):
//   leaf of m steps: 2 multiply-adds per live window entry (m - s at step s)
//     and 4 per live Theta coefficient (s + 1), i.e. 24 m (m + 1);
//   direct merge: window 4 m1 m2, product (first row) 4 m1 m2 multiply-adds;
//   transform merge: 6 transforms + 6 F multiply-adds (window), 4 transforms +
//   7 F (first row of the product); root product 3 transforms + 8 F.
double schur_flops(const SchurPlan& P) {
  double f = 0.0;
  for (const SchurAct& a : P.acts) {
    const double m = a.m, m1 = a.m1, m2 = a.m - a.m1, F = std::ldexp(1.0, a.logF);
    const double tr = 5.0 * F * a.logF;
    switch (a.type) {
      case SCH_LEAF_ACT:
      case SCH_ROOT_LEAF: f += 24.0 * m * (m + 1.0); break;
      case SCH_MID: f += (a.m <= SCH_DIRECT) ? 32.0 * m1 * m2 : 6.0 * tr + 48.0 * F; break;
      case SCH_POST: f += (a.m <= SCH_DIRECT) ? 32.0 * m1 * m2 : 4.0 * tr + 56.0 * F; break;
      case SCH_ROOT: f += (a.m <= SCH_DIRECT) ? 32.0 * m1 * m2 : 3.0 * tr + 64.0 * F; break;
      default: break;
    }
  }
  return f;
}

SchurPlan schur_plan(int64_t N) {
  SchurPlan P;
  if (N > 1) schur_rec(P, 0, (int)N - 1, 0, 0, -1, (int)N);
  return P;
}

int64_t schur_layout(const SchurPlan& P, SchurLayout& L, int* fm_out, int lds_f) {
  std::memset(&L, 0, sizeof L);
  L.nact = (int32_t)P.acts.size();
  int64_t o = 0;
  int fm = 64, fbig = 0;  // the leaves use the transform buffers as 64-element scratch
  for (int l = 0; l < P.nlev; ++l) {
    L.mmax[l] = P.mmax[l];
    L.win[l] = o;
    o += 2 * (int64_t)P.mmax[l];
    L.res[l] = o;
    o += 8 * (int64_t)P.mmax[l];
    L.spec[l] = o;
    o += 2 * (int64_t)P.fspec[l];
    if (P.fspec[l] > lds_f) fbig = std::max(fbig, P.fspec[l]);
    else fm = std::max(fm, P.fspec[l]);
    if (P.mmax[l] <= SCH_DIRECT) fm = std::max(fm, 8 * P.mmax[l] + 256);
  }
  L.xbig = o;
  if (fbig) o += 2 * (int64_t)padded(fbig);
  L.Fmax = fm;
  L.ldsF = lds_f;
  *fm_out = fm;
  return o;
}

// Build per-instance layouts and the action pool for a batch; returns the
// scratch size (complex elements), the largest FFT size and the algorithmic
// flops of each instance.
void schur_plans(int64_t B, const int64_t* n, std::vector<SchurLayout>& lay,
                 std::vector<SchurAct>& pool, int64_t& scr_total, int& Fmax,
                 std::vector<double>& flops, int lds_f) {
  std::map<int64_t, std::pair<int64_t, SchurPlan>> byN;  // N -> (act offset, plan)
  lay.assign((size_t)B, SchurLayout{});
  flops.assign((size_t)B, 0.0);
  pool.clear();
  scr_total = 0;
  Fmax = 64;  // the leaves use the transform buffers as 64-element scratch
  for (int64_t b = 0; b < B; ++b) {
    const int64_t N = n[b];
    auto it = byN.find(N);
    if (it == byN.end()) {
      SchurPlan P = schur_plan(N);
      const int64_t aoff = (int64_t)pool.size();
      pool.insert(pool.end(), P.acts.begin(), P.acts.end());
      it = byN.emplace(N, std::make_pair(aoff, P)).first;
    }
    const SchurPlan& P = it->second.second;
    flops[(size_t)b] = schur_flops(P);
    SchurLayout& L = lay[(size_t)b];
    int fm = 64;
    const int64_t o = schur_layout(P, L, &fm, lds_f);
    L.act_off = it->second.first;
    L.scr_off = scr_total;
    Fmax = std::max(Fmax, fm);
    scr_total += o;
  }
  for (auto& L : lay) L.Fmax = Fmax;
}


DrvParams drv_params(const sfls_params& p) {
  DrvParams dp;
  dp.tau = p.tau; dp.tol_obj = p.tol_obj; dp.tol_newton = p.tol_newton;
  dp.eps_beta_rel = p.eps_beta_rel; dp.eps_L = p.eps_L; dp.approx_ratio = p.approx_ratio;
  dp.approx_min_dist = p.approx_min_dist; dp.ls_c1 = p.ls_c1; dp.curv_eps = p.curv_eps;
  dp.polish_tol = p.polish_tol; dp.polish_ftol = p.polish_ftol; dp.J = p.lbfgs_J;
  dp.max_inner = p.max_inner; dp.max_outer = p.max_outer;
  dp.approx_max_iters = p.approx_max_iters; dp.approx_use_tau = p.approx_use_tau;
  dp.ls_max = p.ls_max; dp.polish_max_iters = p.polish_max_iters; dp.cand_cap = p.cand_cap;
  return dp;
}

bool params_valid(const sfls_params& p) {
  return p.L_mult > 0 && p.lbfgs_J >= 1 && p.lbfgs_J <= 16 && p.max_inner >= 0 &&
         p.max_outer >= 1 && p.ls_max >= 1 && p.polish_max_iters >= 0 && p.cand_cap >= 1 &&
         p.cand_cap <= 2048 && (p.precision == SFLS_FP64 || p.precision == SFLS_MIXED);
}

}  // namespace sfls_host

// Buffers of the generator refinement that follows the superfast recursion:
// transform scratch (4 P per instance at poff) and two sample-length arrays.
struct RefineBufs {
  cd* scratch = nullptr;
  cd* r = nullptr;
  cd* dx = nullptr;
  int maxP = 0;
};

// Factor a batch (Levinson, or superfast Schur followed by one step of
// iterative refinement of the generator, by the context's choice).
static sfls_status run_recursion(sfls_ctx* ctx, int64_t B, const InstInfo* dinfo,
                                 const int32_t* req, const cd* c, cd* rho, double* delta,
                                 double* logdet, int32_t* status, int64_t* failed, int maxN,
                                 hipStream_t st, const SchurLayout* dlay, const SchurAct* dacts,
                                 cd* sscr, int Fmax, const int32_t* order = nullptr) {
  if (dlay) {
    HIP_TRY(launch_schur(dinfo, req, dlay, dacts, c, ctx->tw64, ctx->logtw, ctx->tws64, sscr, rho,
                         delta, logdet, status, failed, (int)B, Fmax, st, order));
  } else {
    HIP_TRY(launch_levinson(dinfo, req, c, rho, delta, logdet, status, failed, (int)B, maxN, st));
  }
  return SFLS_OK;
}

static sfls_status run_refine(sfls_ctx* ctx, int64_t B, const InstInfo* dinfo, const int32_t* req,
                              const cd* c, cd* rho, double* delta, int32_t* status,
                              hipStream_t st, const SchurLayout* dlay, const RefineBufs& rf,
                              const int32_t* order = nullptr) {
  if (dlay)
    HIP_TRY(launch_gen_refine(dinfo, req, status, c, rho, delta, ctx->tw64, ctx->logtw,
                              ctx->tws64, rf.scratch, rf.r, rf.dx, (int)B, rf.maxP, st, order));
  return SFLS_OK;
}

static sfls_status run_factor(sfls_ctx* ctx, int64_t B, const int64_t* n, const InstInfo* dinfo,
                              const int32_t* req, const cd* c, cd* rho, double* delta,
                              double* logdet, int32_t* status, int64_t* failed, int maxN,
                              hipStream_t st, const SchurLayout* dlay, const SchurAct* dacts,
                              cd* sscr, int Fmax, const RefineBufs& rf) {
  (void)n;
  sfls_status s = run_recursion(ctx, B, dinfo, req, c, rho, delta, logdet, status, failed, maxN,
                                st, dlay, dacts, sscr, Fmax);
  if (s != SFLS_OK) return s;
  return run_refine(ctx, B, dinfo, req, c, rho, delta, status, st, dlay, rf);
}

bool sfls_host::use_schur(const sfls_ctx* ctx, int maxN) {
  if (ctx->factor_algo == SFLS_FACTOR_SCHUR) return maxN > 1;
  if (ctx->factor_algo == SFLS_FACTOR_LEVINSON) return false;
  return maxN >= kSchurMinN;
}

static sfls_status check_factor_size(sfls_ctx* ctx, int maxN) {
  if (!use_schur(ctx, maxN) && maxN > kLevinsonMaxN)
    return fail(ctx, SFLS_EUNSUPPORTED, "the Levinson recursion supports n <= %d (got %d)",
                kLevinsonMaxN, maxN);
  return SFLS_OK;
}

// Grid sub-FFT size: M = min(2^ceil(log2 N), cap) with the cap set by what
// two M-point buffers of the grid's precision fit in LDS.
void sfls_host::cap_grid_m(InstInfo& in, int precision) {
  const int cap = precision == SFLS_FP64 ? GRID_LOGM_F64 : GRID_LOGM_F32;
  if (in.logM > cap) {
    in.logM = cap;
    in.M = 1 << cap;
  }
}

// Upload the Schur plans of a batch when the context uses that path.
static sfls_status prepare_schur(sfls_ctx* ctx, int64_t B, const int64_t* n, int maxN,
                                 hipStream_t st, const char* tag, SchurLayout** dlay,
                                 SchurAct** dacts, cd** sscr, int* Fmax,
                                 std::vector<double>* flops = nullptr) {
  *dlay = nullptr;
  *dacts = nullptr;
  *sscr = nullptr;
  *Fmax = 0;
  if (!use_schur(ctx, maxN)) return SFLS_OK;
  std::vector<SchurLayout> lay;
  std::vector<SchurAct> pool;
  std::vector<double> fl;
  int64_t tot = 0;
  schur_plans(B, n, lay, pool, tot, *Fmax, fl, ctx->schur_lds_f);
  if (flops) *flops = fl;
  if (pool.empty()) pool.push_back(SchurAct{});
  sfls_status s;
  std::string a = std::string(tag) + "_slay", b = std::string(tag) + "_sact";
  if ((s = upload(ctx, a.c_str(), lay, st, dlay)) != SFLS_OK) return s;
  if ((s = upload(ctx, b.c_str(), pool, st, dacts)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "schur_scr", (size_t)std::max<int64_t>(tot, 1), sscr)) != SFLS_OK) return s;
  return SFLS_OK;
}

extern "C" {

void sfls_params_default(sfls_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->L_mult = 8.0;
  p->tau = 5.0;
  p->lbfgs_J = 10;
  p->max_inner = 5;
  p->max_outer = 200;
  p->approx_max_iters = 10;
  p->approx_use_tau = 0;
  p->ls_max = 30;
  p->polish_max_iters = 30;
  p->cand_cap = 256;
  p->tol_obj = 1e-7;
  p->tol_newton = 1e-8;
  p->eps_beta_rel = 1e-10;
  p->eps_L = 2.220446049250313e-16;
  p->approx_ratio = 5.0;
  p->approx_min_dist = 0.05;
  p->ls_c1 = 1e-4;
  p->curv_eps = 1e-12;
  p->polish_tol = 1e-12;
  p->polish_ftol = 1e-13;
  p->precision = SFLS_FP64;
}

const char* sfls_version(void) { return kVersion; }

const char* sfls_strerror(sfls_status s) {
  switch (s) {
    case SFLS_OK: return "ok";
    case SFLS_NOTCONV: return "iteration cap reached before convergence";
    case SFLS_EINVAL: return "invalid argument";
    case SFLS_ENOMEM: return "device memory allocation failed";
    case SFLS_EDEVICE: return "HIP runtime error";
    case SFLS_ENOTPD: return "Toeplitz matrix not positive definite";
    case SFLS_ECAPACITY: return "component capacity exceeded";
    case SFLS_EUNSUPPORTED: return "size not supported by this build";
    case SFLS_EAGAIN: return "no free slot or device memory for the request now";
  }
  return "unknown status";
}

const char* sfls_last_error(const sfls_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

sfls_status sfls_create(sfls_ctx** out, int device, size_t hbm_budget_bytes) {
  if (!out) return SFLS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SFLS_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return SFLS_EDEVICE;
  sfls_ctx* ctx = new sfls_ctx();
  ctx->device = device;
  ctx->hbm_budget = hbm_budget_bytes;
  const size_t nt = (size_t)1 << (ctx->logtw - 1);
  if (hipMalloc(&ctx->tw64, nt * sizeof(cd)) != hipSuccess ||
      hipMalloc(&ctx->tw32, nt * sizeof(cf)) != hipSuccess ||
      hipMalloc(&ctx->tws64, 2 * nt * sizeof(cd)) != hipSuccess ||
      hipMalloc(&ctx->tws32, 2 * nt * sizeof(cf)) != hipSuccess) {
    sfls_destroy(ctx);
    return SFLS_ENOMEM;
  }
  if (launch_twiddles(ctx->tw64, ctx->tw32, ctx->tws64, ctx->tws32, ctx->logtw, nullptr) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    sfls_destroy(ctx);
    return SFLS_EDEVICE;
  }
  for (int k = 0; k < KID_COUNT; ++k)
    std::snprintf(ctx->kst[k].name, sizeof ctx->kst[k].name, "%s", kKernelNames[k]);
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) ==
            hipSuccess && ncu > 0)
      ctx->ncu = ncu;
  }
  if (hipEventCreateWithFlags(&ctx->ev_rounds[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_rounds[1], hipEventDisableTiming) != hipSuccess ||
      noalloc_init(ctx) != SFLS_OK) {
    sfls_destroy(ctx);
    return SFLS_EDEVICE;
  }
  *out = ctx;
  return SFLS_OK;
}

sfls_status sfls_set_factor(sfls_ctx* ctx, int32_t algo) {
  if (!ctx) return SFLS_EINVAL;
  if (algo != SFLS_FACTOR_AUTO && algo != SFLS_FACTOR_LEVINSON && algo != SFLS_FACTOR_SCHUR)
    return fail(ctx, SFLS_EINVAL, "unknown factorisation %d", algo);
  ctx->factor_algo = algo;
  return SFLS_OK;
}

sfls_status sfls_set_schur_lds(sfls_ctx* ctx, int32_t max_f) {
  if (!ctx) return SFLS_EINVAL;
  if (max_f < SCH_LDS_F_MIN || max_f > SCH_LDS_F || !is_pow2(max_f))
    return fail(ctx, SFLS_EINVAL, "LDS transform limit %d: a power of two in %d..%d", max_f,
                SCH_LDS_F_MIN, SCH_LDS_F);
  ctx->schur_lds_f = max_f;
  return SFLS_OK;
}

sfls_status sfls_set_nufft(sfls_ctx* ctx, int32_t mode) {
  if (!ctx) return SFLS_EINVAL;
  if (mode != SFLS_NUFFT_AUTO && mode != SFLS_NUFFT_OFF && mode != SFLS_NUFFT_ON)
    return fail(ctx, SFLS_EINVAL, "unknown NUFFT mode %d", mode);
  ctx->nufft_mode = mode;
  return SFLS_OK;
}

sfls_status sfls_set_speculation(sfls_ctx* ctx, int32_t enable) {
  if (!ctx) return SFLS_EINVAL;
  if (enable != 0 && enable != 1) return fail(ctx, SFLS_EINVAL, "speculation mode %d", (int)enable);
  ctx->spec = enable;
  return SFLS_OK;
}

sfls_status sfls_set_timing(sfls_ctx* ctx, int32_t enable) {
  if (!ctx) return SFLS_EINVAL;
  if (enable && !ctx->ev[0]) {
    for (auto& e : ctx->ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(ctx, SFLS_EDEVICE, "hipEventCreate failed");
  }
  if (enable < 0 || enable > 2) return fail(ctx, SFLS_EINVAL, "timing mode %d", (int)enable);
  ctx->timing = enable;
  return SFLS_OK;
}

void sfls_reset_stats(sfls_ctx* ctx) {
  if (!ctx) return;
  for (int k = 0; k < KID_COUNT; ++k) {
    ctx->kst[k].launches = 0;
    ctx->kst[k].seconds = 0.0;
    ctx->kst[k].flops = 0.0;
    ctx->kst[k].bytes = 0.0;
  }
}

int32_t sfls_kernel_stats(const sfls_ctx* ctx, sfls_kernel_stat* out, int32_t cap) {
  if (!ctx) return 0;
  const int32_t n = cap < KID_COUNT ? cap : KID_COUNT;
  for (int32_t k = 0; k < n && out; ++k) out[k] = ctx->kst[k];
  return KID_COUNT;
}

sfls_status sfls_last_run(const sfls_ctx* ctx, sfls_run_stats* stats, double* timeline,
                          int64_t cap, int64_t* ntimeline) {
  if (!ctx) return SFLS_EINVAL;
  if (stats) *stats = ctx->last;
  const int64_t nt = (int64_t)ctx->timeline.size();
  if (ntimeline) *ntimeline = nt;
  for (int64_t i = 0; timeline && i < nt && i < cap; ++i) timeline[i] = ctx->timeline[(size_t)i];
  return SFLS_OK;
}

sfls_status sfls_destroy(sfls_ctx* ctx) {
  if (!ctx) return SFLS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (ctx->tw64) (void)hipFree(ctx->tw64);
  if (ctx->tw32) (void)hipFree(ctx->tw32);
  if (ctx->tws64) (void)hipFree(ctx->tws64);
  if (ctx->tws32) (void)hipFree(ctx->tws32);
  if (ctx->host_req) (void)hipHostFree(ctx->host_req);
  if (ctx->upload) (void)hipStreamDestroy(ctx->upload);
  for (auto& e : ctx->ev_rounds)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return SFLS_OK;
}

sfls_status sfls_toeplitz_column(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                                 const int64_t* K, const int64_t* koff, const double* theta,
                                 const double* gamma, const double* beta, double* c,
                                 void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (!K || !koff || !beta || !c) return fail(ctx, SFLS_EINVAL, "NULL argument");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  std::vector<int32_t> kc((size_t)B);
  for (int64_t b = 0; b < B; ++b) {
    if (K[b] < 0 || koff[b] < 0) return fail(ctx, SFLS_EINVAL, "K/koff[%lld] < 0", (long long)b);
    if (K[b] > 0 && (!theta || !gamma)) return fail(ctx, SFLS_EINVAL, "theta/gamma NULL");
    info[(size_t)b].koff = koff[b];
    kc[(size_t)b] = (int32_t)K[b];
  }
  InstInfo* dinfo;
  int32_t* dK;
  if ((s = upload(ctx, "tc_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = upload(ctx, "tc_K", kc, st, &dK)) != SFLS_OK) return s;
  cd* tscr = nullptr;
  if (sz.maxP > CONV_LDS_P && (s = wsT(ctx, "tc_scr", (size_t)pt, &tscr)) != SFLS_OK) return s;
  HIP_TRY(launch_toeplitz_column(dinfo, nullptr, dK, theta, gamma, beta, (cd*)c, (int)B, sz.maxN,
                                 st, ctx->nufft_mode, ctx->tws64, tscr, sz.maxP));
  return SFLS_OK;
}

sfls_status sfls_factor(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                        const double* c, double* rho, double* delta, double* logdet,
                        int32_t* status, int64_t* failed_step, void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (!c || !rho) return fail(ctx, SFLS_EINVAL, "c and rho must be non-NULL");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  if ((s = check_factor_size(ctx, sz.maxN)) != SFLS_OK) return s;
  InstInfo* dinfo;
  if ((s = upload(ctx, "f_info", info, st, &dinfo)) != SFLS_OK) return s;
  SchurLayout* dlay;
  SchurAct* dacts;
  cd* sscr;
  int Fmax;
  if ((s = prepare_schur(ctx, B, n, sz.maxN, st, "f", &dlay, &dacts, &sscr, &Fmax)) != SFLS_OK)
    return s;
  RefineBufs rf;
  if (dlay) {
    // the refinement needs the pivots and the status even when not requested
    const int64_t ntot = info.back().off + info.back().N;
    if (!delta && (s = wsT(ctx, "f_delta", (size_t)ntot, &delta)) != SFLS_OK) return s;
    if (!status && (s = wsT(ctx, "f_status", (size_t)B, &status)) != SFLS_OK) return s;
    if ((s = wsT(ctx, "scratch", (size_t)pt, &rf.scratch)) != SFLS_OK) return s;
    if ((s = wsT(ctx, "f_r", (size_t)ntot, &rf.r)) != SFLS_OK) return s;
    if ((s = wsT(ctx, "f_dx", (size_t)ntot, &rf.dx)) != SFLS_OK) return s;
    rf.maxP = sz.maxP;
  }
  return run_factor(ctx, B, n, dinfo, nullptr, (const cd*)c, (cd*)rho, delta, logdet, status,
                    failed_step, sz.maxN, st, dlay, dacts, sscr, Fmax, rf);
}

sfls_status sfls_gs_apply(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                          const void* y, int32_t ydtype, const double* rho, const double* delta,
                          double* w, double* yCy, double* ww, void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (!y || !rho || !delta || !w) return fail(ctx, SFLS_EINVAL, "NULL argument");
  if (ydtype != SFLS_C64 && ydtype != SFLS_C128) return fail(ctx, SFLS_EINVAL, "bad ydtype");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  InstInfo* dinfo;
  cd* scratch;
  if ((s = upload(ctx, "a_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "scratch", (size_t)pt, &scratch)) != SFLS_OK) return s;
  HIP_TRY(launch_gs_apply(dinfo, nullptr, y, ydtype, (const cd*)rho, delta, ctx->tw64,
                          ctx->logtw, ctx->tws64, scratch, (cd*)w, yCy, ww, (int)B, sz.maxP, st));
  return SFLS_OK;
}

sfls_status sfls_omega(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                       const int64_t* oout, const double* rho, const double* delta,
                       double* omega_s, double* omega_t, double* omega_v, double* omega_x,
                       void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (!oout || !rho || !delta) return fail(ctx, SFLS_EINVAL, "NULL argument");
  const int which = (omega_s ? 1 : 0) | (omega_t ? 2 : 0) | (omega_v ? 4 : 0) | (omega_x ? 8 : 0);
  if (!which) return SFLS_OK;
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  std::vector<SepCoef> coef((size_t)B);
  for (int64_t b = 0; b < B; ++b) {
    if (oout[b] < 0) return fail(ctx, SFLS_EINVAL, "oout[%lld] < 0", (long long)b);
    info[(size_t)b].ooff = oout[b];
    sep_coef((int)n[b], coef[(size_t)b]);
  }
  InstInfo* dinfo;
  SepCoef* dcoef;
  cd* scratch;
  if ((s = upload(ctx, "o_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = upload(ctx, "o_coef", coef, st, &dcoef)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "scratch", (size_t)pt, &scratch)) != SFLS_OK) return s;
  HIP_TRY(launch_omega(dinfo, nullptr, (const cd*)rho, delta, dcoef, ctx->tws64,
                       scratch, which, 0, nullptr, (cd*)omega_s, (cd*)omega_t, (cd*)omega_v,
                       (cd*)omega_x, (int)B, sz.maxP, st));
  return SFLS_OK;
}

sfls_status sfls_grid_eval(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                           const void* y, int32_t ydtype, const double* rho, const double* delta,
                           const int64_t* L, const int64_t* goff, const double* gamma_bar,
                           const double* zeta, uint32_t out_mask, void* qG, void* sG, void* rG,
                           void* tG, void* dL, int64_t* argmin, double* argmin_val,
                           int32_t precision, void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (out_mask & ~(uint32_t)SFLS_GRID_ALL) return fail(ctx, SFLS_EINVAL, "unknown out_mask bits 0x%x", out_mask);
  const bool wq = out_mask & SFLS_GRID_Q, ws = out_mask & SFLS_GRID_S, wr = out_mask & SFLS_GRID_R,
             wt = out_mask & SFLS_GRID_T, wd = out_mask & SFLS_GRID_DL,
             wa = out_mask & SFLS_GRID_ARGMIN;
  if ((wq && !qG) || (ws && !sG) || (wr && !rG) || (wt && !tG) || (wd && !dL) ||
      (wa && !argmin && !argmin_val))
    return fail(ctx, SFLS_EINVAL, "an output named in out_mask is NULL");
  const bool need_main = wq || ws || wd || wa, need_der = wr || wt;
  if (!y || !rho || !delta || !L || !goff) return fail(ctx, SFLS_EINVAL, "NULL argument");
  if ((wd || wa) && (!gamma_bar || !zeta)) return fail(ctx, SFLS_EINVAL, "NULL gamma_bar or zeta");
  if (ydtype != SFLS_C64 && ydtype != SFLS_C128) return fail(ctx, SFLS_EINVAL, "bad ydtype");
  if (precision != SFLS_FP64 && precision != SFLS_MIXED) return fail(ctx, SFLS_EINVAL, "bad precision");
  if (!need_main && !need_der) return SFLS_OK;
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0, ntot = 0, otot = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  std::vector<SepCoef> coef((size_t)B);
  std::vector<int32_t> req((size_t)B, REQ_EVAL | REQ_GRID);
  for (int64_t b = 0; b < B; ++b) {
    InstInfo& in = info[(size_t)b];
    if (!is_pow2(L[b]) || L[b] < 2 * n[b] - 1 || L[b] < in.M)
      return fail(ctx, SFLS_EINVAL, "L[%lld] = %lld must be a power of two >= 2n-1", (long long)b, (long long)L[b]);
    if (goff[b] < 0) return fail(ctx, SFLS_EINVAL, "goff[%lld] < 0", (long long)b);
    cap_grid_m(in, precision);
    in.L = (int32_t)L[b];
    in.R = (int32_t)(L[b] / in.M);
    in.goff = goff[b];
    in.ooff = otot;
    otot += 2 * n[b] - 1;
    sz.Rmax = std::max(sz.Rmax, in.R);
    sz.maxM = std::max(in.M, b == 0 ? 0 : sz.maxM);
    ntot = std::max(ntot, off[b] + n[b]);
    sep_coef((int)n[b], coef[(size_t)b]);
  }
  InstInfo* dinfo;
  SepCoef* dcoef;
  int32_t* dreq;
  cd *scratch, *w, *oms, *omt = nullptr;
  double *pv, *yCy;
  int64_t* pi;
  if ((s = upload(ctx, "g_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = upload(ctx, "g_coef", coef, st, &dcoef)) != SFLS_OK) return s;
  if ((s = upload(ctx, "g_req", req, st, &dreq)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "scratch", (size_t)pt, &scratch)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "g_w", (size_t)ntot, &w)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "g_oms", (size_t)pt, &oms)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "g_pv", (size_t)B * sz.Rmax, &pv)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "g_pi", (size_t)B * sz.Rmax, &pi)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "g_yCy", (size_t)B, &yCy)) != SFLS_OK) return s;
  if (wt && (s = wsT(ctx, "g_omt", (size_t)otot, &omt)) != SFLS_OK) return s;
  HIP_TRY(launch_gs_apply(dinfo, dreq, y, ydtype, (const cd*)rho, delta, ctx->tw64, ctx->logtw,
                          ctx->tws64, scratch, w, yCy, nullptr, (int)B, sz.maxP, st));
  if (ws || wd || wa || wt)
    HIP_TRY(launch_omega(dinfo, dreq, (const cd*)rho, delta, dcoef, ctx->tws64, scratch,
                         1 | (wt ? 2 : 0), 1, oms, nullptr, omt, nullptr, nullptr, (int)B,
                         sz.maxP, st));
  const void* tw = precision == SFLS_FP64 ? (const void*)ctx->tws64 : (const void*)ctx->tws32;
  if (need_main)
    HIP_TRY(launch_grid(precision, dinfo, dreq, w, oms, gamma_bar, zeta, tw, ctx->logtw, sz.Rmax,
                        (int)B, sz.maxM, wq ? qG : nullptr, ws ? sG : nullptr, wd ? dL : nullptr,
                        pv, pi, st));
  if (wa)
    HIP_TRY(launch_argmin_out(dinfo, sz.Rmax, pv, pi, argmin, argmin_val, (int)B, st));
  if (need_der)
    HIP_TRY(launch_grid_deriv(precision, dinfo, dreq, w, omt, tw, ctx->logtw, sz.Rmax, (int)B,
                              sz.maxM, wr ? rG : nullptr, wt ? tG : nullptr, st));
  return SFLS_OK;
}

sfls_status sfls_active_eval(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                             const double* w, const double* rho, const double* delta,
                             const int64_t* K, const int64_t* koff, const double* theta,
                             double* q, double* r, double* u, double* s_, double* t, double* v,
                             double* x, void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 1);
  if (s != SFLS_OK || B == 0) return s;
  if (!w || !rho || !delta || !K || !koff) return fail(ctx, SFLS_EINVAL, "NULL argument");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0, ktot = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  std::vector<SepCoef> coef((size_t)B);
  std::vector<int32_t> req((size_t)B, REQ_EVAL), kc((size_t)B);
  for (int64_t b = 0; b < B; ++b) {
    if (K[b] < 0 || koff[b] < 0) return fail(ctx, SFLS_EINVAL, "K/koff[%lld] < 0", (long long)b);
    if (K[b] > 0 && !theta) return fail(ctx, SFLS_EINVAL, "theta NULL");
    info[(size_t)b].koff = koff[b];
    kc[(size_t)b] = (int32_t)K[b];
    ktot = std::max(ktot, koff[b] + K[b]);
    sep_coef((int)n[b], coef[(size_t)b]);
  }
  InstInfo* dinfo;
  SepCoef* dcoef;
  int32_t *dreq, *dK, *prefix;
  if ((s = upload(ctx, "ae_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = upload(ctx, "ae_coef", coef, st, &dcoef)) != SFLS_OK) return s;
  if ((s = upload(ctx, "ae_req", req, st, &dreq)) != SFLS_OK) return s;
  if ((s = upload(ctx, "ae_K", kc, st, &dK)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "ae_prefix", (size_t)B + 1, &prefix)) != SFLS_OK) return s;
  cd *dummy, *scratch = nullptr;
  if ((s = wsT(ctx, "ae_dummy", (size_t)std::max<int64_t>(ktot, 1), &dummy)) != SFLS_OK) return s;
  if (ctx->nufft_mode != SFLS_NUFFT_OFF &&
      (s = wsT(ctx, "scratch", (size_t)pt, &scratch)) != SFLS_OK)
    return s;
  auto o = [&](double* p) { return p ? (cd*)p : dummy; };
  HIP_TRY(launch_active(dinfo, dreq, dK, nullptr, prefix, (int)B, theta, nullptr, (const cd*)w,
                        (const cd*)rho, delta, dcoef, o(q), o(r), o(u), o(s_), o(t), o(v), o(x),
                        nullptr, nullptr, 2048, ctx->nufft_mode, ctx->tws64, scratch, sz.maxP,
                        st));
  return SFLS_OK;
}

// The estimate of sfls_estimate (G = 1) and sfls_estimate_mmv (G vectors per
// instance sharing the generator, Sec. V).
// Incomplete observations (Sec. IV): instance b observes m[b] samples whose
// indices, weights and values start at moff[b] of idx, phi (NULL: unit
// weights) and y.
struct SfInput {
  const int64_t* m;
  const int64_t* moff;
  const int32_t* idx;
  const cd* phi;
};

// Observation fields of the instance table (nobs, obsoff, the semifast matrix
// and column offsets) for a semifast call, and the device check of the
// indices and weights (before any kernel indexes with them).  kc[b] is the
// component capacity, at most SF_KMAX.  Returns the totals of the observation
// arrays (sum m), the matrix blocks (sum 4 kc^2), the columns (sum m kc) and
// the phase tables (sum kc (ceil(n/64) + 64)).
static sfls_status sf_prepare(sfls_ctx* ctx, int64_t B, const SfInput& sf,
                              std::vector<InstInfo>& info, const std::vector<int32_t>& kc,
                              hipStream_t st, int64_t* mtot, int64_t* smtot, int64_t* utot,
                              int64_t* ttot) {
  if (!sf.m || !sf.moff || !sf.idx) return fail(ctx, SFLS_EINVAL, "NULL observation argument");
  int64_t mt = 0, sm = 0, ut = 0, tt = 0;
  for (int64_t b = 0; b < B; ++b) {
    InstInfo& in = info[(size_t)b];
    if (sf.m[b] < 1 || sf.m[b] > in.N || sf.moff[b] < 0)
      return fail(ctx, SFLS_EINVAL, "m/moff[%lld]: need 1 <= m <= n, moff >= 0", (long long)b);
    in.nobs = (int32_t)sf.m[b];
    in.obsoff = sf.moff[b];
    in.kcap = kc[(size_t)b];
    in.sfoff = sm;
    sm += 4 * (int64_t)in.kcap * in.kcap;
    in.uoff = ut;
    ut += (int64_t)in.nobs * in.kcap;
    in.tboff = tt;
    tt += (int64_t)in.kcap * SF_TBW(in.N);
    mt = std::max(mt, sf.moff[b] + sf.m[b]);
  }
  InstInfo* dinfo;
  int32_t* dbad;
  sfls_status s;
  if ((s = upload(ctx, "sf_chk_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "sf_chk_bad", (size_t)B, &dbad)) != SFLS_OK) return s;
  HIP_TRY(launch_sf_check(dinfo, sf.idx, sf.phi, dbad, (int)B, st));
  std::vector<int32_t> bad((size_t)B);
  HIP_TRY(hipMemcpyAsync(bad.data(), dbad, (size_t)B * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int64_t b = 0; b < B; ++b)
    if (bad[(size_t)b])
      return fail(ctx, SFLS_EINVAL,
                  "instance %lld: observed indices not strictly increasing in [0, n), or a zero "
                  "or non-finite weight", (long long)b);
  *mtot = mt;
  *smtot = sm;
  *utot = ut;
  *ttot = tt;
  return SFLS_OK;
}

static sfls_status estimate_impl(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                                 int32_t G, const void* y, int64_t ystride, int32_t ydtype,
                                 const sfls_params* params, const int64_t* kcap,
                                 const int64_t* koff, int64_t* K, double* theta, double* alpha,
                                 int64_t alpha_stride, double* gamma, double* beta, double* zeta,
                                 double* objective, int32_t* iters, int32_t* evals,
                                 int32_t* status, void* stream, const SfInput* sf = nullptr) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  sfls_status s = check_batch(ctx, B, n, off, 2);
  if (s != SFLS_OK || B == 0) return s;
  if (!y || !kcap || !koff || !K || !theta || !alpha || !gamma || !beta || !zeta || !objective ||
      !iters || !status)
    return fail(ctx, SFLS_EINVAL, "NULL argument");
  if (G < 1 || G > SFLS_MAX_VECTORS)
    return fail(ctx, SFLS_EINVAL, "G = %d outside 1..%d", G, SFLS_MAX_VECTORS);
  if (G > 1) {
    for (int64_t b = 0; b < B; ++b) {
      if (off[b] + n[b] > ystride)
        return fail(ctx, SFLS_EINVAL, "ystride %lld < off + n of instance %lld", (long long)ystride,
                    (long long)b);
      if (koff[b] + kcap[b] > alpha_stride)
        return fail(ctx, SFLS_EINVAL, "alpha_stride %lld < koff + kcap of instance %lld",
                    (long long)alpha_stride, (long long)b);
    }
  }
  if (ydtype != SFLS_C64 && ydtype != SFLS_C128) return fail(ctx, SFLS_EINVAL, "bad ydtype");
  sfls_params p;
  if (params) p = *params; else sfls_params_default(&p);
  if (!params_valid(p)) return fail(ctx, SFLS_EINVAL, "invalid sfls_params");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  // Shadow slots (complete data, one vector): instance b's shadow is
  // instance B + b of the launch, with its own copy of the signal; the driver
  // steps the B instances only, the evaluation kernels all 2B.
  const int64_t Br = B;
  // shadows double the call's workspace: a context with an HBM budget does
  // without them rather than fail a call that fits without them
  const bool spec = ctx->spec != 0 && ctx->hbm_budget == 0 && !sf && G == 1 &&
                    B <= ctx->ncu && B <= 1024;
  std::vector<int64_t> n2, off2, kcap2, koff2;
  if (spec) {
    int64_t ny = 0;
    for (int64_t b = 0; b < Br; ++b) ny = std::max(ny, off[b] + n[b]);
    n2.assign(n, n + Br);
    n2.insert(n2.end(), n, n + Br);
    off2.assign(off, off + Br);
    for (int64_t b = 0; b < Br; ++b) off2.push_back(ny + off[b]);
    kcap2.assign(kcap, kcap + Br);
    kcap2.insert(kcap2.end(), kcap, kcap + Br);
    koff2.assign(koff, koff + Br);
    koff2.insert(koff2.end(), koff, koff + Br);
    const size_t yb = (ydtype == SFLS_C64 ? 8 : 16) * (size_t)ny;
    void* y2 = nullptr;
    if ((s = ws(ctx, "e_ysh", 2 * yb, &y2)) != SFLS_OK) return s;
    HIP_TRY(hipMemcpyAsync(y2, y, yb, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync((char*)y2 + yb, y, yb, hipMemcpyDeviceToDevice, st));
    y = y2;
    n = n2.data();
    off = off2.data();
    kcap = kcap2.data();
    koff = koff2.data();
    B = 2 * Br;
  }
  Sizes sz;
  int64_t pt = 0, ntot = 0, ktot = 0, gtot = 0, ctot = 0;
  std::vector<InstInfo> info = base_info(B, n, off, sz, pt);
  if (!sf && (s = check_factor_size(ctx, sz.maxN)) != SFLS_OK) return s;
  std::vector<SepCoef> coef((size_t)B);
  std::vector<int64_t> okoff((size_t)B);
  const int cc = p.cand_cap + 1;
  for (int64_t b = 0; b < B; ++b) {
    InstInfo& in = info[(size_t)b];
    if (kcap[b] < 1 || koff[b] < 0) return fail(ctx, SFLS_EINVAL, "kcap/koff[%lld]", (long long)b);
    const int64_t Lb = (int64_t)1 << (int)std::lround(std::log2(p.L_mult * (double)n[b]));
    if (Lb < 2 * n[b] - 1 || Lb < in.M)
      return fail(ctx, SFLS_EINVAL, "grid L = %lld shorter than 2n-1 for n = %lld", (long long)Lb, (long long)n[b]);
    if (Lb > (1 << 24)) return fail(ctx, SFLS_EUNSUPPORTED, "grid too large");
    cap_grid_m(in, p.precision);
    in.L = (int32_t)Lb;
    in.R = (int32_t)(Lb / in.M);
    in.kcap = (int32_t)std::min<int64_t>(kcap[b], n[b]);
    // incomplete observations: K_max = m, and the semifast factor holds at
    // most SF_KMAX components
    if (sf) in.kcap = (int32_t)std::min<int64_t>({kcap[b], sf->m ? std::max<int64_t>(sf->m[b], 1) : 1,
                                                  (int64_t)SF_KMAX});
    in.koff = ktot;
    ktot += in.kcap;
    in.goff = gtot;
    gtot += Lb;
    in.coff = ctot;
    ctot += cc;
    sz.Rmax = std::max(sz.Rmax, in.R);
    sz.maxM = std::max(in.M, b == 0 ? 0 : sz.maxM);
    ntot = std::max(ntot, off[b] + n[b]);
    okoff[(size_t)b] = koff[b];
    sep_coef((int)n[b], coef[(size_t)b]);
  }
  std::vector<DrvParams> dpv(1, drv_params(p));
  int64_t sf_mtot = 0, sf_smtot = 0, sf_utot = 0, sf_ttot = 0;
  if (sf) {
    std::vector<int32_t> kcv((size_t)B);
    for (int64_t b = 0; b < B; ++b) kcv[(size_t)b] = info[(size_t)b].kcap;
    if ((s = sf_prepare(ctx, B, *sf, info, kcv, st, &sf_mtot, &sf_smtot, &sf_utot, &sf_ttot)) !=
        SFLS_OK)
      return s;
  }

  InstInfo* dinfo;
  SepCoef* dcoef;
  DrvParams* dprm;
  int64_t* dokoff;
  if ((s = upload(ctx, "e_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = upload(ctx, "e_coef", coef, st, &dcoef)) != SFLS_OK) return s;
  if ((s = upload(ctx, "e_prm", dpv, st, &dprm)) != SFLS_OK) return s;
  if ((s = upload(ctx, "e_okoff", okoff, st, &dokoff)) != SFLS_OK) return s;
  // a batch of uneven sizes starts its longest instances first
  int32_t* dorder = nullptr;
  if (spec) {
    // the real instances longest first (uneven N), then the shadows, whose
    // half of the order each round's grant rewrites
    const std::vector<int32_t> ro = longest_first(Br, n);
    std::vector<int32_t> ordv((size_t)B);
    for (int64_t i = 0; i < Br; ++i) {
      ordv[(size_t)i] = ro.empty() ? (int32_t)i : ro[(size_t)i];
      ordv[(size_t)(Br + i)] = (int32_t)(Br + i);
    }
    if ((s = upload(ctx, "e_order", ordv, st, &dorder)) != SFLS_OK) return s;
  } else {
    const std::vector<int32_t> order = longest_first(B, n);
    if (!order.empty() && (s = upload(ctx, "e_order", order, st, &dorder)) != SFLS_OK) return s;
  }

  const int J = p.lbfgs_J;
  const size_t esz = p.precision == SFLS_FP64 ? sizeof(double) : sizeof(float);
  cd *c, *rho, *w, *scratch, *oms;
  double *delta, *logdet, *yCy, *ww, *pv;
  int64_t *failed, *pi;
  int32_t *lev_status, *prefix, *ovf;
  void* dL;
  DrvPools P{};
#define WS(name, cnt, ptr) if ((s = wsT(ctx, name, (size_t)(cnt), &(ptr))) != SFLS_OK) return s
  WS("e_c", ntot, c);
  WS("e_rho", ntot, rho);
  WS("e_w", (int64_t)G * ntot, w);
  WS("e_delta", ntot, delta);
  WS("scratch", pt, scratch);
  WS("e_oms", pt, oms);
  RefineBufs rf;
  rf.scratch = scratch;
  rf.maxP = sz.maxP;
  WS("e_rf_r", ntot, rf.r);
  WS("e_rf_dx", ntot, rf.dx);
  WS("e_logdet", B, logdet);
  WS("e_yCy", B, yCy);
  WS("e_ww", B, ww);
  WS("e_failed", B, failed);
  WS("e_levst", B, lev_status);
  WS("e_prefix", B + 1, prefix);
  WS("e_ovf", B, ovf);
  WS("e_pv", B * sz.Rmax, pv);
  WS("e_pi", B * sz.Rmax, pi);
  if ((s = ws(ctx, "e_dL", (size_t)gtot * esz, &dL)) != SFLS_OK) return s;
  DrvState* dst;
  WS("e_state", B, dst);
  P.st = dst;
  WS("e_th", ktot, P.th);
  WS("e_ga", ktot, P.ga);
  WS("e_th_e", ktot, P.th_e);
  WS("e_ga_e", ktot, P.ga_e);
  WS("e_g", 2 * ktot, P.g);
  WS("e_d", 2 * ktot, P.d);
  WS("e_gt", 2 * ktot, P.gt);
  WS("e_qsave", 2 * (int64_t)G * ktot, P.q_save);
  WS("e_Sm", (size_t)J * 2 * ktot, P.Sm);
  WS("e_Ym", (size_t)J * 2 * ktot, P.Ym);
  WS("e_rhom", (size_t)J * B, P.rhom);
  WS("e_am", (size_t)J * B, P.am);
  WS("e_Ke", B, P.K_e);
  WS("e_req", B, P.req);
  WS("e_req2", B, P.req2);
  WS("e_beta_e", B, P.beta_e);
  WS("e_gbar_e", B, P.gbar_e);
  WS("e_zeta_e", B, P.zeta_e);
  cd *evq, *evr, *evu, *evs, *evt, *evv, *evx, *cq;
  double* cs;
  int32_t *cand, *ncand;
  WS("e_evq", (int64_t)G * ktot, evq);
  WS("e_evr", (int64_t)G * ktot, evr);
  WS("e_evu", (int64_t)G * ktot, evu);
  WS("e_evs", ktot, evs);
  WS("e_evt", ktot, evt);
  WS("e_evv", ktot, evv);
  WS("e_evx", ktot, evx);
  WS("e_cand", ctot, cand);
  WS("e_ncand", B, ncand);
  WS("e_cq", (int64_t)G * ctot, cq);
  WS("e_cs", ctot, cs);
  WS("e_cbdl", ctot, P.cbuf_dl);
  WS("e_cbgh", ctot, P.cbuf_gh);
  WS("e_cbl", ctot, P.cbuf_l);
  int32_t* notdone;
  WS("e_notdone", 1, notdone);
  if (spec) {
    WS("e_wish", Br, P.wish);
    P.nsh = (int32_t)Br;
  }
#undef WS
  P.ev_q = evq; P.ev_r = evr; P.ev_u = evu; P.ev_s = evs; P.ev_t = evt; P.ev_v = evv;
  P.ev_x = evx; P.logdet = logdet; P.yCy = yCy; P.ww = ww; P.lev_status = lev_status;
  P.cand = cand; P.ncand = ncand; P.cand_q = cq; P.cand_s = cs;
  P.out_K = K; P.out_theta = theta; P.out_alpha = (cd*)alpha; P.out_gamma = gamma;
  P.out_beta = beta; P.out_zeta = zeta; P.out_obj = objective; P.out_iters = iters;
  P.out_evals = evals; P.out_status = status; P.out_koff = dokoff; P.notdone = notdone;
  // observation vectors: strides of the per-vector arrays
  Vecs vv;
  vv.G = G;
  vv.ystride = G > 1 ? ystride : 0;
  vv.wstride = G > 1 ? ntot : 0;
  vv.kstride = G > 1 ? ktot : 0;
  vv.cstride = G > 1 ? ctot : 0;
  P.G = G;
  P.kstride = vv.kstride;
  P.cstride = vv.cstride;
  P.ostride = G > 1 ? alpha_stride : 0;

  SchurLayout* slay;
  SchurAct* sacts;
  cd* sscr;
  int sFmax;
  std::vector<double> sflops;
  if (!sf) {
    if ((s = prepare_schur(ctx, B, n, sz.maxN, st, "e", &slay, &sacts, &sscr, &sFmax,
                           &sflops)) != SFLS_OK)
      return s;
  } else {
    slay = nullptr;
    sacts = nullptr;
    sscr = nullptr;
    sFmax = 0;
  }
  // semifast workspace: the K x K matrix blocks, A^H y, c, C^{-1} y on the
  // observed samples and the grid columns U
  cd *sfm = nullptr, *sfh = nullptr, *sfc = nullptr, *sfw = nullptr, *sfU = nullptr,
     *sft = nullptr;
  if (sf) {
    if ((s = wsT(ctx, "e_sft", (size_t)std::max<int64_t>(sf_ttot, 1), &sft)) != SFLS_OK ||
        (s = wsT(ctx, "e_sfm", (size_t)std::max<int64_t>(sf_smtot, 1), &sfm)) != SFLS_OK ||
        (s = wsT(ctx, "e_sfh", (size_t)ktot, &sfh)) != SFLS_OK ||
        (s = wsT(ctx, "e_sfc", (size_t)ktot, &sfc)) != SFLS_OK ||
        (s = wsT(ctx, "e_sfw", (size_t)std::max<int64_t>(sf_mtot, 1), &sfw)) != SFLS_OK ||
        (s = wsT(ctx, "e_sfU", (size_t)std::max<int64_t>(sf_utot, 1), &sfU)) != SFLS_OK)
      return s;
  }
  const int prec = p.precision;
  const void* tw = prec == SFLS_FP64 ? (const void*)ctx->tws64 : (const void*)ctx->tws32;
  const double slack = prec == SFLS_FP64 ? 1e-9 : 1e-3;
  const int act_blocks = 2048;

  // pinned host words the driver writes directly (read back by the host
  // without a copy): per round, the request bits of every instance, the grid
  // sweeps of the round's second stage (req2) and the component count of each
  // request.  Two sets, by round parity: round r's driver passes write set
  // (r + 1) % 2 while the host reads set r % 2 (written by round r - 1).
  if (ctx->host_req_n < Br) {
    if (ctx->host_req) (void)hipHostFree(ctx->host_req);
    ctx->host_req = nullptr;
    ctx->host_req_n = 0;
    if (hipHostMalloc(&ctx->host_req, 6 * (size_t)Br * sizeof(int32_t),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
      return fail(ctx, SFLS_ENOMEM, "pinned request buffer");
    ctx->host_req_n = Br;
  }
  std::memset(ctx->host_req, 0, 6 * (size_t)Br * sizeof(int32_t));
  int32_t* hset[2] = {ctx->host_req, ctx->host_req + 3 * Br};
  int32_t* hreq_dev = nullptr;
  HIP_TRY(hipHostGetDevicePointer((void**)&hreq_dev, ctx->host_req, 0));
  int32_t* dset[2] = {hreq_dev, hreq_dev + 3 * Br};
  auto write_set = [&](int set) {
    P.req_host = dset[set];
    P.req2_host = dset[set] + Br;
    P.kev_host = dset[set] + 2 * Br;
  };
  const auto t0 = std::chrono::steady_clock::now();
  auto now_s = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  ctx->timeline.clear();
  ctx->last = sfls_run_stats{};
  const bool timing = ctx->timing != 0;
  // kernel events by round parity: [parity][stage][kernel][start, stop]
  const int EP = 2 * KID_COUNT;  // events of one stage
  bool launched[2][2][KID_COUNT];
  double kflops[2][KID_COUNT], kbytes[2][KID_COUNT];
  std::memset(launched, 0, sizeof launched);
  std::memset(kflops, 0, sizeof kflops);
  std::memset(kbytes, 0, sizeof kbytes);
  int par = 0, stage = 0;  // of the round being enqueued
  auto tstart = [&](int k) -> hipError_t {
    launched[par][stage][k] = true;
    return timing && times_kernel(ctx->timing, k)
               ? hipEventRecord(ctx->ev[(par * 2 + stage) * EP + 2 * k], st) : hipSuccess;
  };
  auto tstop = [&](int k) -> hipError_t {
    return timing && times_kernel(ctx->timing, k)
               ? hipEventRecord(ctx->ev[(par * 2 + stage) * EP + 2 * k + 1], st) : hipSuccess;
  };
  const double esz_d = (double)esz;
  // algorithmic bytes of a sweep's omega stage: rho in, omega_s out; semifast:
  // the observed C^{-1} y and the columns U written and read, omega_s out
  auto omega_bytes = [&](int64_t b, const int32_t* kev) {
    const double Nb = (double)n[b];
    if (!sf) return 16.0 * Nb + 16.0 * (2.0 * Nb - 1.0);
    const InstInfo& in = info[(size_t)b];
    return 16.0 * in.nobs + 32.0 * (double)in.nobs * kev[b] + 16.0 * (2.0 * Nb - 1.0);
  };

  // One round: the evaluations the instances asked for, the first driver
  // pass, the grid stage and the candidates' vectors (for the sweeps of
  // P.req2), the second driver pass.  Every kernel is launched; each takes
  // only the instances whose request bits name it, so the round can be
  // enqueued before the host has read those bits.
  auto enqueue_round = [&](int64_t r) -> sfls_status {
    par = (int)(r & 1);
    stage = 0;
    std::memset(launched[par], 0, sizeof launched[par]);
    write_set((int)((r + 1) & 1));
    if (sf) {
      HIP_TRY(tstart(KID_FACTOR));
      HIP_TRY(launch_sf_eval(dinfo, P.req, P.K_e, P.th_e, P.ga_e, P.beta_e, y, ydtype, sf->idx,
                             sf->phi, sfm, sfh, sfc, sft, sfw, logdet, yCy, ww, lev_status, evq,
                             evr, evu, evs, evt, evv, evx, (int)B, st));
      HIP_TRY(tstop(KID_FACTOR));
    } else {
      HIP_TRY(tstart(KID_GEN));
      HIP_TRY(launch_toeplitz_column(dinfo, P.req, P.K_e, P.th_e, P.ga_e, P.beta_e, c, (int)B,
                                     sz.maxN, st, ctx->nufft_mode, ctx->tws64, scratch,
                                     sz.maxP));
      HIP_TRY(tstop(KID_GEN));
      HIP_TRY(tstart(KID_FACTOR));
      sfls_status rs;
      if ((rs = run_recursion(ctx, B, dinfo, P.req, c, rho, delta, logdet, lev_status, failed,
                              sz.maxN, st, slay, sacts, sscr, sFmax, dorder)) != SFLS_OK)
        return rs;
      HIP_TRY(tstop(KID_FACTOR));
      HIP_TRY(tstart(KID_REFINE));
      if ((rs = run_refine(ctx, B, dinfo, P.req, c, rho, delta, lev_status, st, slay, rf,
                           dorder)) != SFLS_OK)
        return rs;
      // ln|C| over the active set (determinant lemma) where it is small enough
      HIP_TRY(launch_logdet_lemma(dinfo, P.req, P.K_e, P.th_e, P.ga_e, P.beta_e, lev_status,
                                  logdet, (int)B, st, dorder));
      HIP_TRY(tstop(KID_REFINE));
      HIP_TRY(tstart(KID_APPLY));
      HIP_TRY(launch_gs_apply(dinfo, P.req, y, ydtype, rho, delta, ctx->tw64, ctx->logtw,
                              ctx->tws64, scratch, w, yCy, ww, (int)B, sz.maxP, st, dorder, vv));
      HIP_TRY(tstop(KID_APPLY));
      // active-set vectors at the evaluated points (candidates follow the grid stage)
      HIP_TRY(tstart(KID_ACTIVE));
      HIP_TRY(launch_active(dinfo, P.req, P.K_e, nullptr, prefix, (int)B, P.th_e, cand, w, rho,
                            delta, dcoef, evq, evr, evu, evs, evt, evv, evx, cq, cs, act_blocks,
                            ctx->nufft_mode, ctx->tws64, scratch, sz.maxP, st, vv, dorder));
      HIP_TRY(tstop(KID_ACTIVE));
    }
    // first driver pass: the instances whose request had no grid sweep
    HIP_TRY(tstart(KID_DRIVER));
    HIP_TRY(launch_driver(dinfo, dprm, P, (int)Br, st));
    HIP_TRY(tstop(KID_DRIVER));
    // Grid stage, after the first pass: the grid sweeps the round began with
    // (their evaluation, if any, is done) and those the pass just requested
    // at the point this round evaluated (factor, C^-1 y and active vectors in
    // place), which so run now instead of a round later; then the candidates'
    // vectors and the second driver pass, for exactly these (P.req2).
    stage = 1;
    HIP_TRY(tstart(KID_OMEGA));
    if (sf)
      HIP_TRY(launch_sf_grid_inputs(dinfo, P.req2, P.K_e, P.th_e, P.ga_e, P.beta_e, sf->idx,
                                    sf->phi, sfw, sfm, sft, ctx->tws64, w, sfU, scratch, oms,
                                    (int)B, sz.maxP, st));
    else
      HIP_TRY(launch_omega(dinfo, P.req2, rho, delta, dcoef, ctx->tws64, scratch, 1, 1, oms,
                           nullptr, nullptr, nullptr, nullptr, (int)B, sz.maxP, st, dorder));
    HIP_TRY(tstop(KID_OMEGA));
    HIP_TRY(tstart(KID_GRID));
    HIP_TRY(launch_grid(prec, dinfo, P.req2, w, oms, P.gbar_e, P.zeta_e, tw, ctx->logtw, sz.Rmax,
                        (int)B, sz.maxM, nullptr, nullptr, dL, pv, pi, st, vv));
    HIP_TRY(tstop(KID_GRID));
    HIP_TRY(tstart(KID_SELECT));
    HIP_TRY(launch_select(prec, dinfo, P.req2, dL, sz.Rmax, pv, pi, p.approx_ratio, slack,
                          p.cand_cap, cand, ncand, ovf, (int)B, st));
    HIP_TRY(tstop(KID_SELECT));
    HIP_TRY(tstart(KID_ACTIVE));
    if (sf)
      HIP_TRY(launch_sf_cand(dinfo, P.req2, P.K_e, P.beta_e, sf->idx, sf->phi, sfw, sfU, cand,
                             ncand, cq, cs, (int)B, sz.maxN, st));
    else
      HIP_TRY(launch_active(dinfo, P.req2, P.K_e, ncand, prefix, (int)B, P.th_e, cand, w, rho,
                            delta, dcoef, evq, evr, evu, evs, evt, evv, evx, cq, cs, act_blocks,
                            ctx->nufft_mode, ctx->tws64, scratch, sz.maxP, st, vv));
    HIP_TRY(tstop(KID_ACTIVE));
    HIP_TRY(tstart(KID_DRIVER));
    HIP_TRY(launch_driver(dinfo, dprm, P, (int)Br, st, 1));
    HIP_TRY(tstop(KID_DRIVER));
    // shadow requests for the next round, on the CUs its requests leave free
    if (spec) HIP_TRY(launch_spec_grant(P.req, P.wish, dorder, (int)Br, ctx->ncu, st));
    HIP_TRY(hipEventRecord(ctx->ev_rounds[par], st));
    return SFLS_OK;
  };

  // the initial driver pass (round 0) writes the requests of round 1 into set 1
  HIP_TRY(launch_init_state(dinfo, y, ydtype, dst, P.req, (int)Br, st, nullptr, vv));
  HIP_TRY(launch_zero_i32(notdone, 1, st));
  HIP_TRY(launch_zero_i32(P.req2, (int)B, st));
  if (spec) {
    HIP_TRY(launch_zero_i32(P.req + Br, (int)Br, st));
    HIP_TRY(launch_zero_i32(P.wish, (int)Br, st));
  }
  write_set(1);
  HIP_TRY(launch_driver(dinfo, dprm, P, (int)Br, st));
  HIP_TRY(hipEventRecord(ctx->ev_rounds[0], st));
  int64_t rounds = 0, ev_total = 0, gevals = 0;
  const int64_t max_rounds = 1000000;
  // One round of lookahead: round r + 1 is enqueued while round r runs, so
  // the device never waits for the host's turn between rounds.  Iteration r
  // waits for round r - 1, reads round r's requests (set r % 2) and round
  // r - 1's grid sweeps, clears the set, and enqueues round r + 1, whose
  // driver passes write that set again.  A finished instance no longer writes
  // its words, so a set read all zero means the batch is done (round r, then
  // enqueued, finds nothing to do).
  if ((s = enqueue_round(1)) != SFLS_OK) return s;
  for (int64_t r = 1;; ++r) {
    HIP_TRY(spin_wait(ctx->ev_rounds[(r - 1) & 1]));
    ctx->timeline.push_back(now_s());
    const int rs = (int)(r & 1);
    int32_t* hq = hset[rs];
    int32_t* hq2 = hq + Br;
    int32_t* hk = hq + 2 * Br;
    if (r >= 2) {
      // round r - 1: its second stage's grid sweeps, its kernel times
      const int pp = (int)((r - 1) & 1);
      for (int64_t b = 0; b < Br; ++b) {
        if (!hq2[b]) continue;
        ++gevals;
        const double N = (double)n[b], Lb = (double)info[(size_t)b].L;
        kbytes[pp][KID_GRID] += 16.0 * N + 16.0 * (2.0 * N - 1.0) + esz_d * Lb;
        kbytes[pp][KID_OMEGA] += omega_bytes(b, hk);
        kbytes[pp][KID_ACTIVE] += 32.0 * N;  // the candidates' vectors: w, rho in
      }
      if (timing) {
        for (int k = 0; k < KID_COUNT; ++k) {
          if (!times_kernel(ctx->timing, k)) continue;
          for (int sg = 0; sg < 2; ++sg) {
            if (!launched[pp][sg][k]) continue;
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[(pp * 2 + sg) * EP + 2 * k],
                                        ctx->ev[(pp * 2 + sg) * EP + 2 * k + 1]));
            ctx->kst[k].launches += 1;
            ctx->kst[k].seconds += 1e-3 * (double)ms;
          }
          ctx->kst[k].flops += kflops[pp][k];
          ctx->kst[k].bytes += kbytes[pp][k];
        }
      }
      for (int k = 0; k < KID_COUNT; ++k) kflops[pp][k] = kbytes[pp][k] = 0.0;
    }
    // round r's requests and their algorithmic work
    int64_t nact = 0, ngrid = 0, nreq = 0;
    for (int64_t b = 0; b < Br; ++b) {
      const int32_t rq = hq[b];
      if (!rq) continue;
      ++nreq;
      const double N = (double)n[b];
      // algorithmic work per evaluation (per-instance figures of the design)
      if ((rq & REQ_EVAL) && sf) {
        // semifast: Gram sums (3 K^2 M / 2 complex MACs), the K x K Cholesky,
        // inverse and solves, the residual and q, r, u (4 K M)
        ++nact;
        const double Mo = (double)info[(size_t)b].nobs, Kc = (double)hk[b];
        kflops[rs][KID_FACTOR] += 8.0 * (1.5 * Kc * Kc * Mo + 4.0 * Kc * Mo) + 8.0 * Kc * Kc * Kc;
        kbytes[rs][KID_FACTOR] += (ydtype == SFLS_C64 ? 8.0 : 16.0) * Mo + 4.0 * Mo + 16.0 * Mo;
      } else if (rq & REQ_EVAL) {
        ++nact;
        kflops[rs][KID_FACTOR] += slay ? sflops[(size_t)b] : 8.0 * N * N;  // Schur or Levinson
        kbytes[rs][KID_FACTOR] += 40.0 * N;                    // c in, rho and delta out
        kbytes[rs][KID_GEN] += 16.0 * N;                       // c out
        if (slay) {
          const double P = (double)info[(size_t)b].P, lp = (double)info[(size_t)b].logP;
          kflops[rs][KID_REFINE] += 10.0 * 5.0 * P * lp + 96.0 * P;  // 10 transforms + pointwise
          kbytes[rs][KID_REFINE] += 48.0 * N;                  // c, rho in; rho out
        }
        kbytes[rs][KID_APPLY] += (ydtype == SFLS_C64 ? 8.0 : 16.0) * N + 32.0 * N;  // y, rho in; w out
        kbytes[rs][KID_ACTIVE] += 32.0 * N;                    // w, rho in
      }
      // grid stage: alone when the evaluation at the current point is in place
      if (rq & REQ_GRID) {
        ++ngrid;
        const double Lb = (double)info[(size_t)b].L;
        kbytes[rs][KID_GRID] += 16.0 * N + 16.0 * (2.0 * N - 1.0) + esz_d * Lb;
        kbytes[rs][KID_OMEGA] += omega_bytes(b, hk);
      }
    }
    // the set is read: clear it for round r + 1's driver passes
    std::memset(hq, 0, 3 * (size_t)Br * sizeof(int32_t));
    if (nreq == 0) {
      HIP_TRY(spin_wait(ctx->ev_rounds[rs]));  // round r, enqueued, had nothing to do
      break;
    }
    if (rounds >= max_rounds) return fail(ctx, SFLS_EDEVICE, "estimate did not finish");
    ++rounds;
    ev_total += nact;
    gevals += ngrid;
    if ((s = enqueue_round(r + 1)) != SFLS_OK) return s;
  }
  ctx->last.rounds = rounds;
  ctx->last.evals = ev_total;
  ctx->last.grid_evals = gevals;
  ctx->last.wall_seconds = now_s();
  (void)notdone;

  return SFLS_OK;
}

sfls_status sfls_estimate(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                          const void* y, int32_t ydtype, const sfls_params* params,
                          const int64_t* kcap, const int64_t* koff, int64_t* K, double* theta,
                          double* alpha, double* gamma, double* beta, double* zeta,
                          double* objective, int32_t* iters, int32_t* evals, int32_t* status,
                          void* stream) {
  return estimate_impl(ctx, B, n, off, 1, y, 0, ydtype, params, kcap, koff, K, theta, alpha, 0,
                       gamma, beta, zeta, objective, iters, evals, status, stream);
}

sfls_status sfls_estimate_mmv(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                              int32_t G, const void* y, int64_t ystride, int32_t ydtype,
                              const sfls_params* params, const int64_t* kcap, const int64_t* koff,
                              int64_t* K, double* theta, double* alpha, int64_t alpha_stride,
                              double* gamma, double* beta, double* zeta, double* objective,
                              int32_t* iters, int32_t* evals, int32_t* status, void* stream) {
  return estimate_impl(ctx, B, n, off, G, y, ystride, ydtype, params, kcap, koff, K, theta, alpha,
                       alpha_stride, gamma, beta, zeta, objective, iters, evals, status, stream);
}


// ---------------------------------------------------------------------------
// Incomplete observations (Sec. IV)
// ---------------------------------------------------------------------------

// N-space offsets of a batch (the instances' length-n arrays back to back).
static std::vector<int64_t> packed_offsets(int64_t B, const int64_t* n) {
  std::vector<int64_t> off((size_t)std::max<int64_t>(B, 1), 0);
  for (int64_t b = 1; b < B; ++b) off[(size_t)b] = off[(size_t)b - 1] + n[b - 1];
  return off;
}

sfls_status sfls_incomplete_eval(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* m,
                                 const int64_t* moff, const int32_t* idx, const double* phi,
                                 const void* y, int32_t ydtype, const int64_t* K,
                                 const int64_t* koff, const double* theta, const double* gamma,
                                 const double* beta, double* logdet, double* yCy, double* ww,
                                 double* q, double* r, double* u, double* s_, double* t, double* v,
                                 double* x, const int64_t* L, const int64_t* goff, double* qG,
                                 double* sG, const int32_t* cand, const int64_t* ncand,
                                 const int64_t* coff, double* cq, double* cs, int32_t* status,
                                 void* stream) {
  if (!ctx) return SFLS_EINVAL;
  ctx->err.clear();
  if (!n || B < 0) return fail(ctx, SFLS_EINVAL, "NULL n or B < 0");
  const std::vector<int64_t> offv = packed_offsets(B, n);
  sfls_status s = check_batch(ctx, B, n, offv.data(), 2);
  if (s != SFLS_OK || B == 0) return s;
  if (!y || !K || !koff || !beta) return fail(ctx, SFLS_EINVAL, "NULL argument");
  if (ydtype != SFLS_C64 && ydtype != SFLS_C128) return fail(ctx, SFLS_EINVAL, "bad ydtype");
  const bool grid = L != nullptr, wc = cand != nullptr;
  if (grid && (!goff || (!qG && !sG && !wc))) return fail(ctx, SFLS_EINVAL, "grid outputs need goff and qG/sG/cand");
  if (wc && (!grid || !ncand || !coff || !cq || !cs))
    return fail(ctx, SFLS_EINVAL, "candidates need L, ncand, coff, cq and cs");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = as_stream(stream);
  Sizes sz;
  int64_t pt = 0, ntot = 0, ktot = 0, ctot = 0;
  std::vector<InstInfo> info = base_info(B, n, offv.data(), sz, pt);
  std::vector<int32_t> kc((size_t)B), kev((size_t)B), nc((size_t)B, 0);
  std::vector<int32_t> req((size_t)B, REQ_EVAL | (grid ? REQ_GRID : 0));
  for (int64_t b = 0; b < B; ++b) {
    InstInfo& in = info[(size_t)b];
    if (!m || m[b] < 1 || m[b] > n[b]) return fail(ctx, SFLS_EINVAL, "m[%lld] outside 1..n", (long long)b);
    if (K[b] < 0 || K[b] > std::min<int64_t>(m[b], SF_KMAX) || koff[b] < 0)
      return fail(ctx, SFLS_EINVAL, "K[%lld] = %lld outside 0..min(m, %d), or koff < 0",
                  (long long)b, (long long)K[b], SF_KMAX);
    if (K[b] > 0 && (!theta || !gamma)) return fail(ctx, SFLS_EINVAL, "theta/gamma NULL");
    kc[(size_t)b] = (int32_t)std::max<int64_t>(K[b], 1);
    kev[(size_t)b] = (int32_t)K[b];
    in.koff = koff[b];
    ktot = std::max(ktot, koff[b] + kc[(size_t)b]);
    ntot = std::max(ntot, offv[(size_t)b] + n[b]);
    if (grid) {
      if (!is_pow2(L[b]) || L[b] < 2 * n[b] - 1 || L[b] < in.M || L[b] > (1 << 24) || goff[b] < 0)
        return fail(ctx, SFLS_EINVAL, "L[%lld] = %lld must be a power of two >= 2n-1 (<= 2^24), goff >= 0",
                    (long long)b, (long long)L[b]);
      cap_grid_m(in, SFLS_FP64);
      in.L = (int32_t)L[b];
      in.R = (int32_t)(L[b] / in.M);
      in.goff = goff[b];
      sz.Rmax = std::max(sz.Rmax, in.R);
      sz.maxM = std::max(in.M, b == 0 ? 0 : sz.maxM);
    }
    if (wc) {
      if (ncand[b] < 0 || ncand[b] > (1 << 20) || coff[b] < 0)
        return fail(ctx, SFLS_EINVAL, "ncand/coff[%lld]", (long long)b);
      nc[(size_t)b] = (int32_t)ncand[b];
      in.coff = coff[b];
      ctot = std::max(ctot, coff[b] + ncand[b]);
    }
  }
  const SfInput sfin{m, moff, idx, reinterpret_cast<const cd*>(phi)};
  int64_t mt = 0, smt = 0, ut = 0, tt = 0;
  if ((s = sf_prepare(ctx, B, sfin, info, kc, st, &mt, &smt, &ut, &tt)) != SFLS_OK) return s;
  InstInfo* dinfo;
  int32_t *dreq, *dK, *dnc = nullptr;
  if ((s = upload(ctx, "ie_info", info, st, &dinfo)) != SFLS_OK) return s;
  if ((s = upload(ctx, "ie_req", req, st, &dreq)) != SFLS_OK) return s;
  if ((s = upload(ctx, "ie_K", kev, st, &dK)) != SFLS_OK) return s;
  if (wc && (s = upload(ctx, "ie_nc", nc, st, &dnc)) != SFLS_OK) return s;
  cd *sfm, *sfh, *sfc, *sfw, *sfU, *sft;
  if ((s = wsT(ctx, "ie_sft", (size_t)std::max<int64_t>(tt, 1), &sft)) != SFLS_OK ||
      (s = wsT(ctx, "ie_sfm", (size_t)std::max<int64_t>(smt, 1), &sfm)) != SFLS_OK ||
      (s = wsT(ctx, "ie_sfh", (size_t)ktot, &sfh)) != SFLS_OK ||
      (s = wsT(ctx, "ie_sfc", (size_t)ktot, &sfc)) != SFLS_OK ||
      (s = wsT(ctx, "ie_sfw", (size_t)std::max<int64_t>(mt, 1), &sfw)) != SFLS_OK ||
      (s = wsT(ctx, "ie_sfU", (size_t)std::max<int64_t>(ut, 1), &sfU)) != SFLS_OK)
    return s;
  // outputs the caller does not want go to workspace
  double *ld = logdet, *yc = yCy, *wn = ww;
  int32_t* stt = status;
  if (!ld && (s = wsT(ctx, "ie_ld", (size_t)B, &ld)) != SFLS_OK) return s;
  if (!yc && (s = wsT(ctx, "ie_yc", (size_t)B, &yc)) != SFLS_OK) return s;
  if (!wn && (s = wsT(ctx, "ie_wn", (size_t)B, &wn)) != SFLS_OK) return s;
  if (!stt && (s = wsT(ctx, "ie_st", (size_t)B, &stt)) != SFLS_OK) return s;
  cd* vec[7] = {(cd*)q, (cd*)r, (cd*)u, (cd*)s_, (cd*)t, (cd*)v, (cd*)x};
  static const char* vnames[7] = {"ie_q", "ie_r", "ie_u", "ie_s", "ie_t", "ie_v", "ie_x"};
  for (int i = 0; i < 7; ++i)
    if (!vec[i] && (s = wsT(ctx, vnames[i], (size_t)ktot, &vec[i])) != SFLS_OK) return s;
  HIP_TRY(launch_sf_eval(dinfo, dreq, dK, theta, gamma, beta, y, ydtype, idx, sfin.phi, sfm, sfh,
                         sfc, sft, sfw, ld, yc, wn, stt, vec[0], vec[1], vec[2], vec[3], vec[4], vec[5],
                         vec[6], (int)B, st));
  if (!grid) return SFLS_OK;
  cd *scratch, *w, *oms;
  double* pv;
  int64_t* pi;
  if ((s = wsT(ctx, "scratch", (size_t)pt, &scratch)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "ie_w", (size_t)ntot, &w)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "ie_oms", (size_t)pt, &oms)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "ie_pv", (size_t)B * sz.Rmax, &pv)) != SFLS_OK) return s;
  if ((s = wsT(ctx, "ie_pi", (size_t)B * sz.Rmax, &pi)) != SFLS_OK) return s;
  HIP_TRY(launch_sf_grid_inputs(dinfo, dreq, dK, theta, gamma, beta, idx, sfin.phi, sfw, sfm,
                                sft, ctx->tws64, w, sfU, scratch, oms, (int)B, sz.maxP, st));
  if (qG || sG)
    HIP_TRY(launch_grid(SFLS_FP64, dinfo, dreq, w, oms, nullptr, nullptr, ctx->tws64, ctx->logtw,
                        sz.Rmax, (int)B, sz.maxM, qG, sG, nullptr, pv, pi, st));
  if (wc)
    HIP_TRY(launch_sf_cand(dinfo, dreq, dK, beta, idx, sfin.phi, sfw, sfU, cand, dnc, (cd*)cq, cs,
                           (int)B, sz.maxN, st));
  return SFLS_OK;
}

sfls_status sfls_estimate_incomplete(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* m,
                                     const int64_t* moff, const int32_t* idx, const double* phi,
                                     const void* y, int32_t ydtype, const sfls_params* params,
                                     const int64_t* kcap, const int64_t* koff, int64_t* K,
                                     double* theta, double* alpha, double* gamma, double* beta,
                                     double* zeta, double* objective, int32_t* iters,
                                     int32_t* evals, int32_t* status, void* stream) {
  if (!ctx) return SFLS_EINVAL;
  if (!n || B < 0) return sfls_host::fail(ctx, SFLS_EINVAL, "NULL n or B < 0");
  const std::vector<int64_t> offv = packed_offsets(B, n);
  const SfInput sfin{m, moff, idx, reinterpret_cast<const cd*>(phi)};
  return estimate_impl(ctx, B, n, offv.data(), 1, y, 0, ydtype, params, kcap, koff, K, theta,
                       alpha, 0, gamma, beta, zeta, objective, iters, evals, status, stream, &sfin);
}

}  // extern "C"
